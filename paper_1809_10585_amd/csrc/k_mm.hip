// HODLR matrix times tall-skinny block (Table 1) and the small dense products
// of the update step.
#include "kernels_common.h"
#include "kernels.h"

namespace hq {

// ------------------------------------------------------------------ HODLR x tall-skinny
__device__ __forceinline__ int mm_s(const MmJob& J, const Opnd& o) {
  return J.s_dev ? *J.s_dev : (J.s > 0 ? J.s : o.s);
}
// X and Z of a job with their leading dimensions (a slot >= 0 binds the call's operand)
__device__ __forceinline__ const double* mm_x(const MmJob& J, const Opnd& o, int& ld) {
  if (J.xs < 0) {
    ld = J.ldX;
    return J.X;
  }
  ld = o.ld[J.xs];
  return o.p[J.xs] + J.xoff;
}
__device__ __forceinline__ double* mm_z(const MmJob& J, const Opnd& o, int& ld) {
  if (J.zs < 0) {
    ld = J.ldZ;
    return J.Z;
  }
  ld = o.ld[J.zs];
  return o.p[J.zs] + J.zoff;
}

// Phase A: projections P_b = F_b^T X (F = V for op N, U for op T) of every
// block of the sub-HODLR, MM_CH rows per block of threads.  Thread t takes
// output e = t % nout (nout = k s) and every Q-th row of the chunk
// (Q = NT_MM / nout groups), so all loads of a block are in flight together;
// the Q partial sums are added in a fixed order.  A block of one chunk writes
// its projection directly, longer blocks write per-chunk partials that
// k_mm_red sums (a separate launch: no cross-block fences).
__global__ void __launch_bounds__(NT_MM) k_mm_proj(const MmJob* __restrict__ jobs,
                                                    const MmProj* __restrict__ items, int first,
                                                    double* ws, Opnd op) {
  __shared__ double part_s[NT_MM];
  const int tid = threadIdx.x;
  const MmProj it = items[first + blockIdx.x];
  const MmJob& J = jobs[it.job];
  const int s = mm_s(J, op);
  const int rld = J.rld;
  const HBlk b = (it.kind == 0 ? J.M.up : J.M.lo)[it.node];
  const int k = *b.rank;
  if (k == 0 || s == 0) return;
  const int trans = J.trans;
  const int len = trans ? b.rows : b.cols;
  const double* F = trans ? b.U : b.V;
  const int ldF = trans ? b.ldU : b.ldV;
  int ldX;
  const double* X = mm_x(J, op, ldX) + (trans ? b.r0 - J.row0 : b.c0 - J.col0);
  const int c0 = it.chunk * MM_CH;
  const int cn = min(MM_CH, len - c0);
  const int nout = k * s;
  double* dst = ws + it.part;
  if (nout <= NT_MM) {
    const int Q = NT_MM / nout;
    const int e = tid % nout, q = tid / nout;
    double acc = 0.0;
    if (q < Q) {
      const int j = e % k, c = e / k;
      const double* f = F + c0 + (int64_t)j * ldF;
      const double* x = X + c0 + (int64_t)c * ldX;
#pragma unroll 8
      for (int r = q; r < cn; r += Q) acc += f[r] * x[r];
    }
    part_s[tid] = acc;
    __syncthreads();
    if (tid < nout) {
      double sacc = 0.0;
      for (int q2 = 0; q2 < Q; ++q2) sacc += part_s[tid + q2 * nout];
      dst[(tid % k) + (tid / k) * rld] = sacc;
    }
  } else {
    for (int e = tid; e < nout; e += NT_MM) {
      const int j = e % k, c = e / k;
      const double* f = F + c0 + (int64_t)j * ldF;
      const double* x = X + c0 + (int64_t)c * ldX;
      double acc = 0.0;
      for (int r = 0; r < cn; ++r) acc += f[r] * x[r];
      dst[j + c * rld] = acc;
    }
  }
  if (tid == 0) add_flops(J.flops, J.fc, 2.0 * k * cn * s);
}

// Sum the per-chunk partials of one block projection (chunk order fixed).
__global__ void __launch_bounds__(NT_MM) k_mm_red(const MmJob* __restrict__ jobs,
                                                   const MmProj* __restrict__ items, int first,
                                                   double* ws, Opnd op) {
  const MmProj it = items[first + blockIdx.x];
  const MmJob& J = jobs[it.job];
  const int s = mm_s(J, op);
  const int rld = J.rld;
  const HBlk b = (it.kind == 0 ? J.M.up : J.M.lo)[it.node];
  const int k = *b.rank;
  const double* part0 = ws + it.part;
  double* red = ws + J.red0 + (int64_t)(2 * rel_node(it.node, J.v) + it.kind) * (rld * SMAX);
  for (int e = threadIdx.x; e < k * s; e += NT_MM) {
    const int off = (e % k) + (e / k) * rld;
    double acc = 0.0;
    for (int ch = 0; ch < it.nchunk; ++ch) acc += part0[(int64_t)ch * (rld * SMAX) + off];
    red[off] = acc;
  }
}

// Phase B: Z rows of one leaf = leaf part + the low-rank parts of every level.
// A block takes RT rows of one leaf; thread (r, g) = (tid % RT, tid / RT).
// Group g adds the leaf columns of its share and the low-rank parts of the
// ancestor levels g, g + G, ...; the groups' partial rows are then summed in a
// fixed order.  X of the leaf rows is staged in LDS, CW columns at a time
// (CW = 4 for blocks of at most 4 columns, else 16).
//  RT = 16: the group's leaf columns kk = g, g + 16, ... are loaded into
//           registers up front (short launches: one round trip of loads);
//  RT = 64: the group streams a contiguous quarter of the columns, so a wave
//           reads whole 512-byte column pieces (long launches: bandwidth); the
//           loop is unrolled 64/CW times, which keeps two wavefronts per SIMD.
//           For op(D) = D^T the rows of the output are columns of D: the
//           block reads 64 x 64 tiles of D along its columns (coalesced),
//           stores them transposed in LDS (next tile's loads in flight
//           meanwhile), and group g takes rows 16g .. 16g + 15 of each tile.
// Dynamic LDS: max(m_leaf, 256) * 17 doubles.


template <int RT>
__device__ __forceinline__ double leaf_elem(const HLeaf& lf, int kind, int trans, int R, int kk) {
  const int ii = trans ? kk : R, jj = trans ? R : kk;  // element D(ii, jj)
  if (kind == LEAF_FULL) return lf.D[ii + (int64_t)jj * lf.ld];
  if (kind == LEAF_UNIT_LOWER) return (ii > jj) ? lf.D[ii + (int64_t)jj * lf.ld] : (ii == jj ? 1.0 : 0.0);
  return (ii <= jj) ? lf.D[ii + (int64_t)jj * lf.ld] : 0.0;
}

// The rows of one item in column slabs of CW columns (CW = 4 when s <= 4:
// a quarter of the LDS reads and FMAs of the 16-wide slab).
// Tile [k0, k0 + 64) x [row0, row0 + 64) of the leaf, element (kk, R) of D
// for the transposed product, zero outside the leaf and the item's rows.
// Thread tid takes elements e = tid + 256 q: kk = k0 + e % 64, R = row0 + e / 64.
__device__ __forceinline__ void mm_tile_load(double (&tv)[16], const HLeaf& lf, int kind,
                                             const MmApply& it, int m, int k0) {
  const gdouble* D = gmem(lf.D);  // 32-bit offsets: a leaf has at most 512^2 entries
  int ld = lf.ld;
  asm volatile("" : "+v"(ld));  // recompute the 16 addresses per tile instead of holding them
  const int kk = k0 + (threadIdx.x & 63);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int rr = (threadIdx.x >> 6) + 4 * q, R = it.row0 + rr;
    const bool in = kk < m && rr < it.rows;
    // element (kk, R) of the leaf's stored part (as leaf_elem with trans)
    const bool keep = kind == LEAF_FULL || (kind == LEAF_UNIT_LOWER ? kk > R : kk <= R);
    const double x = (in && keep) ? D[kk + R * ld] : 0.0;
    tv[q] = (in && kind == LEAF_UNIT_LOWER && kk == R) ? 1.0 : x;
  }
}

template <int RT, int CW>
__device__ __forceinline__ void mm_apply_rows(const MmJob& J, const MmApply& it, const double* ws,
                                              double* shm, double* Dt, int s, const double* JX, int ldX,
                                              double* JZ, int ldZ) {
  const int rld = J.rld;
  constexpr int G = NT_MM / RT;
  // RT = 16 with 16-column slabs: the leaf part on FP64 MFMA (below), no
  // preloaded leaf column
  constexpr bool LEAF_MFMA = RT == 16 && CW == 16;
  constexpr int DMAX = (RT == 16 && !LEAF_MFMA) ? MAXLEAF / G : 1;
  const int tid = threadIdx.x;
  const int r = tid % RT, g = tid / RT;
  const HLeaf lf = J.M.leaf[it.leaf];
  const int kind = J.M.leaf_kind;
  const int trans = J.trans;
  // output rows of the leaf are its rows (op N) or columns (op T); the sum runs
  // over the other dimension (m: its length)
  const int m = trans ? lf.m : lf.n;
  const int64_t out0 = trans ? lf.c0 : lf.r0;
  const int64_t in0 = trans ? lf.r0 : lf.c0;
  const int R = it.row0 + r;  // output row of this thread within the leaf
  const bool live = r < it.rows;
  double dv[DMAX];
  if constexpr (RT == 16 && !LEAF_MFMA) {
#pragma unroll
    for (int i = 0; i < DMAX; ++i) {
      const int kk = g + G * i;
      dv[i] = (live && kk < m) ? leaf_elem<RT>(lf, kind, trans, R, kk) : 0.0;
    }
  }
  const int q = (m + G - 1) / G;  // RT = 64: columns [g q, g q + q) of this group
  const int kb0 = min(m, g * q), kb1 = min(m, g * q + q);
  const int hleaf = (1 << J.M.levels) + it.leaf;
  // RT = 16: this group's ancestor levels li = g, g + 16 (at most two): the
  // block's rank, factor row and reduced projection, read before the leaf
  // part so that these dependent loads overlap it (same order of terms as the
  // loop below)
  constexpr int NA = RT == 16 ? (MAXGROUPS + G - 1) / G : 1;
  int akb[NA], ald[NA];
  const double* aF[NA];
  const double* aR[NA];
  if constexpr (RT == 16) {
    const int dv = (31 - __clz(hleaf)) - (31 - __clz(J.v));  // levels from the leaf up to v
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const int li = g + G * a;
      akb[a] = 0;
      ald[a] = 0;
      aF[a] = nullptr;
      aR[a] = nullptr;
      if (li < dv) {
        const int child = hleaf >> li, u = child >> 1;
        const bool left = (child & 1) == 0;
        const int bk = trans ? (left ? 1 : 0) : (left ? 0 : 1);
        const HBlk* arr = bk == 0 ? J.M.up : J.M.lo;
        if (arr != nullptr) {
          const HBlk& b = arr[u];
          akb[a] = *b.rank;
          ald[a] = trans ? b.ldV : b.ldU;
          aF[a] = (trans ? b.V : b.U) + (out0 + R - (trans ? b.c0 : b.r0));
          aR[a] = ws + J.red0 + (int64_t)(2 * rel_node(u, J.v) + bk) * (rld * SMAX);
        }
      }
    }
  }
  const double* xl = JX + (in0 - (trans ? J.row0 : J.col0));
  double* Xs = shm;
  for (int c0 = 0; c0 < s; c0 += CW) {
    const int cn = min(CW, s - c0);
    for (int e = tid; e < m * CW; e += NT_MM) {
      const int kk = e % m, c = e / m;
      Xs[kk * MA_LD + c] = (c < cn) ? xl[kk + (int64_t)(c0 + c) * ldX] : 0.0;
    }
    __syncthreads();
    double acc[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) acc[c] = 0.0;
    if constexpr (LEAF_MFMA) {
      // 16 x 16 tile (the block's rows x this slab's columns) = D(rows, :) Xs:
      // wavefront wv takes the k-steps 4 wv, 4 wv + 16, ...; its partial tile
      // goes to mf (row-major) and is summed with the groups' partial rows below
      const int wv = tid >> 6, ln = tid & 63;
      const int Ra = it.row0 + (ln & 15);
      const bool ra = (ln & 15) < it.rows;
      d4_t lacc = {0.0, 0.0, 0.0, 0.0};
      for (int k0 = 4 * wv; k0 < m; k0 += 16) {
        const int kk = k0 + (ln >> 4);
        const double a = (ra && kk < m) ? leaf_elem<RT>(lf, kind, trans, Ra, kk) : 0.0;
        const double b = (kk < m) ? Xs[kk * MA_LD + (ln & 15)] : 0.0;
        lacc = mfma16(a, b, lacc);
      }
      double* mf = shm + (size_t)MA_LD * (m > 256 ? m : 256);
#pragma unroll
      for (int e = 0; e < 4; ++e) mf[wv * 256 + (4 * e + (ln >> 4)) * 16 + (ln & 15)] = lacc[e];
    } else if constexpr (RT == 16) {
#pragma unroll
      for (int i = 0; i < DMAX; ++i) {
        const int kk = g + G * i;
        if (kk < m) {
          const double d = dv[i];
#pragma unroll
          for (int c = 0; c < CW; ++c) acc[c] += d * Xs[kk * MA_LD + c];
        }
      }
    } else if (CW == 4 && trans) {
      double tv[16];
      mm_tile_load(tv, lf, kind, it, m, 0);
      for (int k0 = 0; k0 < m; k0 += 64) {
#pragma unroll
        for (int q = 0; q < 16; ++q) Dt[(tid & 63) * DT_LD + (tid >> 6) + 4 * q] = tv[q];
        __syncthreads();
        if (k0 + 64 < m) mm_tile_load(tv, lf, kind, it, m, k0 + 64);
#pragma unroll 4
        for (int i = 0; i < 16; ++i) {
          const int kl = 16 * g + i;  // g is the wavefront's index: uniform branch
          if (k0 + kl < m) {
            const double d = Dt[kl * DT_LD + r];
#pragma unroll
            for (int c = 0; c < CW; ++c) acc[c] += d * Xs[(k0 + kl) * MA_LD + c];
          }
        }
        __syncthreads();  // the tile is overwritten next
      }
    } else {
      if (live) {
#pragma unroll(64 / CW)
        for (int kk = kb0; kk < kb1; ++kk) {
          const double d = leaf_elem<RT>(lf, kind, trans, R, kk);
#pragma unroll
          for (int c = 0; c < CW; ++c) acc[c] += d * Xs[kk * MA_LD + c];
        }
      }
    }
    // low-rank parts
    if constexpr (RT == 16) {
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        const double* red = aR[a] + (int64_t)c0 * rld;
        for (int j = 0; j < akb[a]; ++j) {
          const double fv = live ? aF[a][(int64_t)j * ald[a]] : 0.0;
#pragma unroll
          for (int c = 0; c < CW; ++c)
            if (c < cn) acc[c] += fv * red[j + c * rld];
        }
      }
    }
    int child = hleaf, u = hleaf >> 1, li = 0;
    while (RT != 16 && child != J.v && u >= 1) {
      if (li % G == g) {
        const bool left = (child == 2 * u);
        const int bk = trans ? (left ? 1 : 0) : (left ? 0 : 1);
        const HBlk* arr = bk == 0 ? J.M.up : J.M.lo;
        if (arr != nullptr) {
          const HBlk& b = arr[u];
          const int kb = *b.rank;
          const double* red = ws + J.red0 + (int64_t)(2 * rel_node(u, J.v) + bk) * (rld * SMAX) +
                              (int64_t)c0 * rld;
          const double* F = trans ? b.V : b.U;
          const int ldF = trans ? b.ldV : b.ldU;
          const int64_t frow = out0 + R - (trans ? b.c0 : b.r0);
          for (int j = 0; j < kb; ++j) {
            const double fv = live ? F[frow + (int64_t)j * ldF] : 0.0;
#pragma unroll
            for (int c = 0; c < CW; ++c)
              if (c < cn) acc[c] += fv * red[j + c * rld];
          }
        }
      }
      child = u;
      u >>= 1;
      ++li;
    }
    __syncthreads();  // Xs is reused for the partial rows
#pragma unroll
    for (int c = 0; c < CW; ++c) shm[(g * RT + r) * MA_LD + c] = acc[c];
    __syncthreads();
    for (int e = tid; e < RT * CW; e += NT_MM) {
      const int rr = e % RT, c = e / RT;
      if (rr < it.rows && c < cn) {
        double sacc = 0.0;
#pragma unroll
        for (int g2 = 0; g2 < G; ++g2) sacc += shm[(g2 * RT + rr) * MA_LD + c];
        if constexpr (LEAF_MFMA) {
          const double* mf = shm + (size_t)MA_LD * (m > 256 ? m : 256);
#pragma unroll
          for (int q = 0; q < NT_MM / 64; ++q) sacc += mf[q * 256 + rr * 16 + c];
        }
        double* zp = JZ + (out0 - (trans ? J.col0 : J.row0) + it.row0 + rr) + (int64_t)(c0 + c) * ldZ;
        const double v = J.alpha * sacc;
        *zp = (J.beta == 0.0) ? v : v + J.beta * (*zp);
      }
    }
    __syncthreads();
  }
}

template <int RT>
__global__ void __launch_bounds__(NT_MM) k_mm_apply(const MmJob* __restrict__ jobs,
                                                     const MmApply* __restrict__ items, int first,
                                                     const double* __restrict__ ws, Opnd op) {
  extern __shared__ double shm[];
  double* Dt = nullptr;  // transposed leaf tile (RT = 64 only)
  if constexpr (RT == 64) {
    __shared__ double dtile[64 * DT_LD];
    Dt = dtile;
  }
  const MmApply it = items[first + blockIdx.x];
  const MmJob& J = jobs[it.job];
  const int s = mm_s(J, op);
  if (s == 0) return;
  int ldX, ldZ;
  const double* JX = mm_x(J, op, ldX);
  double* JZ = mm_z(J, op, ldZ);
  if (s <= 4)
    mm_apply_rows<RT, 4>(J, it, ws, shm, Dt, s, JX, ldX, JZ, ldZ);
  else
    mm_apply_rows<RT, 16>(J, it, ws, shm, Dt, s, JX, ldX, JZ, ldZ);
  if (threadIdx.x == 0) {
    const HLeaf lf = J.M.leaf[it.leaf];
    const int trans = J.trans;
    const int hleaf = (1 << J.M.levels) + it.leaf;
    double flops = 2.0 * it.rows * (trans ? lf.m : lf.n) * s * (J.tri ? 0.5 : 1.0);
    int child2 = hleaf, u2 = hleaf >> 1;
    while (child2 != J.v && u2 >= 1) {
      const bool left = (child2 == 2 * u2);
      const int bk = trans ? (left ? 1 : 0) : (left ? 0 : 1);
      const HBlk* arr = bk == 0 ? J.M.up : J.M.lo;
      if (arr != nullptr) flops += 2.0 * it.rows * (*arr[u2].rank) * s;
      child2 = u2;
      u2 >>= 1;
    }
    add_flops(J.flops, J.fc, flops);
  }
}

// ------------------------------------------------------------------ small GEMMs
// A, B, C and N of a job with the call's operands bound
__device__ __forceinline__ GemmJob gemm_bind(const GemmJob& J0, const Opnd& o) {
  GemmJob J = J0;
  if (J.as_ >= 0) {
    J.A = o.p[J.as_] + J.aoff;
    if (J.lda <= 0) J.lda = o.ld[J.as_];
  }
  if (J.bs_ >= 0) {
    J.B = o.p[J.bs_] + J.boff;
    if (J.ldb <= 0) J.ldb = o.ld[J.bs_];
  }
  if (J.cs_ >= 0) {
    J.C = o.p[J.cs_] + J.coff;
    if (J.ldc <= 0) J.ldc = o.ld[J.cs_];
  }
  if (J.Nd == nullptr && J.N <= 0) J.N = o.s;
  return J;
}

__device__ __forceinline__ double gA(const GemmJob& J, int r, int kk) {
  return J.ta ? J.A[kk + (int64_t)r * J.lda] : J.A[r + (int64_t)kk * J.lda];
}
__device__ __forceinline__ double gB(const GemmJob& J, int kk, int c) {
  return J.tb ? J.B[c + (int64_t)kk * J.ldb] : J.B[kk + (int64_t)c * J.ldb];
}

__global__ void __launch_bounds__(NT_MM) k_gemm_tall(const GemmJob* __restrict__ jobs,
                                                      const GemmTile* __restrict__ items, int first,
                                                      Opnd op) {
  __shared__ double At[64][33];
  __shared__ double Bt[32][65];
  const int tid = threadIdx.x;
  const GemmTile it = items[first + blockIdx.x];
  const GemmJob J = gemm_bind(jobs[it.job], op);
  const int M = J.Md ? *J.Md : J.M, N = J.Nd ? *J.Nd : J.N, K = J.Kd ? *J.Kd : J.K;
  if (it.row0 >= M || it.col0 >= N) return;
  const int mr = min(64, M - it.row0), nc = min(64, N - it.col0);
  // FP64 MFMA on 16 x 16 x 4 tiles: wavefront w takes rows 16w .. 16w + 15 of
  // the 64 x 64 block, all four 16-column tiles (those past nc skipped)
  const int w = tid >> 6, l = tid & 63;
  d4_t acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = d4_t{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < K; k0 += 32) {
    const int kn = min(32, K - k0);
    for (int e = tid; e < 64 * 32; e += NT_MM) {
      int rr, kk;
      if (J.ta) {
        kk = e % 32;
        rr = e / 32;
      } else {
        rr = e % 64;
        kk = e / 64;
      }
      At[rr][kk] = (rr < mr && kk < kn) ? gA(J, it.row0 + rr, k0 + kk) : 0.0;
    }
    for (int e = tid; e < 32 * 64; e += NT_MM) {
      int kk, cc;
      if (J.tb) {
        cc = e % 64;
        kk = e / 64;
      } else {
        kk = e % 32;
        cc = e / 32;
      }
      Bt[kk][cc] = (kk < kn && cc < nc) ? gB(J, k0 + kk, it.col0 + cc) : 0.0;
    }
    __syncthreads();
    // the tiles are zero past kn: k-steps of 4 up to kn (the K of the
    // update's products is a rank, often 1..3, not 32)
    const int k4 = (kn + 3) & ~3;
    if (16 * w < mr) {  // uniform in the wavefront
      for (int kk = 0; kk < k4; kk += 4) {
        const double a = At[16 * w + (l & 15)][kk + (l >> 4)];
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (16 * t < nc) acc[t] = mfma16(a, Bt[kk + (l >> 4)][16 * t + (l & 15)], acc[t]);
      }
    }
    __syncthreads();
  }
  // element e of lane l of tile t: C[16w + 4e + l/16][16t + l%16]
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int rr = 16 * w + 4 * e + (l >> 4), cc = 16 * t + (l & 15);
      if (rr < mr && cc < nc) {
        double* cp = J.C + (int64_t)(it.row0 + rr) + (int64_t)(it.col0 + cc) * J.ldc;
        const double v = J.alpha * acc[t][e];
        *cp = (J.beta == 0.0) ? v : v + J.beta * (*cp);
      }
    }
  }
  if (tid == 0) add_flops(J.flops, J.fc, 2.0 * mr * nc * K);
}

// C (M x N, both <= KCAP) from a long K, split into chunks; the last chunk sums.
__global__ void __launch_bounds__(NT_MM) k_gemm_red(const GemmJob* __restrict__ jobs,
                                                     const GemmRed* __restrict__ items, int first,
                                                     double* ws, int* counters, Opnd op) {
  __shared__ double At[32][KCAP + 1];
  __shared__ double Bt[32][KCAP + 1];
  __shared__ int lastf;
  const int tid = threadIdx.x;
  const GemmRed it = items[first + blockIdx.x];
  const GemmJob J = gemm_bind(jobs[it.job], op);
  const int M = J.Md ? *J.Md : J.M, N = J.Nd ? *J.Nd : J.N;
  if (M == 0 || N == 0) return;
  const int nout = M * N;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  if (nout <= 16 && it.kn <= NT_MM) {
    // small C: thread t takes K index k0 + t, all nout products of it; sums over
    // the wavefront (DPP) and then over the four wavefronts (LDS); thread e <
    // nout ends with output e in acc[0], as the staged loop below leaves it
    __shared__ double wsum[NT_MM / 64][16];
    const int kk = it.k0 + tid;
    const bool on = tid < it.kn;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      double x = 0.0;
      if (on && e < nout) x = gA(J, e % M, kk) * gB(J, kk, e / M);
      x = gsumt<64>(x);
      if ((tid & 63) == 0) wsum[tid >> 6][e] = x;
    }
    __syncthreads();
    double tot = 0.0;
    if (tid < nout)
      for (int w = 0; w < NT_MM / 64; ++w) tot += wsum[w][tid];
    acc[0] = tot;
  } else {
  for (int k0 = it.k0; k0 < it.k0 + it.kn; k0 += 32) {
    const int kn = min(32, it.k0 + it.kn - k0);
    for (int e = tid; e < 32 * KCAP; e += NT_MM) {
      const int kk = e % 32, rr = e / 32;
      At[kk][rr] = (kk < kn && rr < M) ? gA(J, rr, k0 + kk) : 0.0;
      Bt[kk][rr] = (kk < kn && rr < N) ? gB(J, k0 + kk, rr) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + q * NT_MM;
      if (e < nout) {
        const int rr = e % M, cc = e / M;
        double sacc = acc[q];
#pragma unroll 8
        for (int kk = 0; kk < 32; ++kk) sacc += At[kk][rr] * Bt[kk][cc];
        acc[q] = sacc;
      }
    }
    __syncthreads();
  }
  }
  if (it.nchunk == 1) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + q * NT_MM;
      if (e < nout) {
        double* cp = J.C + (int64_t)(e % M) + (int64_t)(e / M) * J.ldc;
        const double v = J.alpha * acc[q];
        *cp = (J.beta == 0.0) ? v : v + J.beta * (*cp);
      }
    }
  } else {
    double* part = ws + it.part;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + q * NT_MM;
      if (e < nout) part[(e % M) + (e / M) * KCAP] = acc[q];
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) {
      const int old = atomicAdd(counters + it.counter, 1);
      lastf = (old == it.nchunk - 1) ? 1 : 0;
      if (lastf) atomicExch(counters + it.counter, 0);
    }
    __syncthreads();
    if (lastf) {
      __threadfence();
      const double* part0 = ws + it.part - (int64_t)it.chunk * (KCAP * KCAP);
      for (int e = tid; e < nout; e += NT_MM) {
        const int rr = e % M, cc = e / M;
        double sacc = 0.0;
        for (int ch = 0; ch < it.nchunk; ++ch) sacc += part0[(int64_t)ch * (KCAP * KCAP) + rr + cc * KCAP];
        double* cp = J.C + (int64_t)rr + (int64_t)cc * J.ldc;
        const double v = J.alpha * sacc;
        *cp = (J.beta == 0.0) ? v : v + J.beta * (*cp);
      }
    }
  }
  if (tid == 0) add_flops(J.flops, J.fc, 2.0 * M * N * it.kn);
}

}  // namespace hq

namespace hq {
template __global__ void k_mm_apply<16>(const MmJob*, const MmApply*, int, const double*, Opnd);
template __global__ void k_mm_apply<64>(const MmJob*, const MmApply*, int, const double*, Opnd);
}  // namespace hq

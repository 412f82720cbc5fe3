// Leaf QR of the stacked column with its compact WY factor (Alg. hQR at the
// lowest level; Alg. blockQR's T merge).
#include "kernels_common.h"
#include "kernels.h"

namespace hq {
// ------------------------------------------------------------------ leaf QR
// Blocked right-looking Householder QR of the stacked leaf column H (M x m,
// ld MAXSTACK) with its compact WY factor T, in 16-column panels.  A panel is
// factorised by one 1024-thread block, one wavefront per column, so every
// column reduction stays inside a wavefront.  Launch p (the "step") updates the
// trailing strips with panel p's reflectors; its first block updates panel
// p+1's columns and then factorises panel p+1 (look-ahead), while other blocks
// form the Gram blocks Y_i^T Y_p and the T block of panel p-1:
//   T[0:c_q, q] = -T[0:c_q, 0:c_q] (Y_{0:c_q}^T Y_q) T_qq     (eq. recqrcombined)
__device__ __forceinline__ int leaf_rows(const LeafJob& J) {
  int M = J.mr;
  for (int g = 0; g < J.ngroups; ++g) M += *J.g[g].rank;
  return M;
}

// H = [A_leaf; C_g1; ...] (one column per block)
// Leaf kernels: a launch covers nper blocks of each of its jobs, job first +
// blockIdx / nper (jobs of different factorisations of one batch).
__global__ void __launch_bounds__(NT_MM) k_leaf_gather(const LeafJob* __restrict__ jobs, int first,
                                                        int nper) {
  const LeafJob& J = jobs[first + blockIdx.x / nper];
  const LeafWs W = J.ws;
  int* err = J.err;
  const int c = blockIdx.x % nper;
  if (c >= J.m) return;
  const int M = leaf_rows(J);
  if (M > MAXSTACK) {
    if (c == 0 && threadIdx.x == 0) atomicOr(err, ERR_STACK);
    return;
  }
  const int mr = J.mr;  // rows of the leaf (its leading dimension)
  double* h = W.H + (int64_t)c * MAXSTACK;
  for (int r = threadIdx.x; r < mr; r += NT_MM) h[r] = J.D[r + (int64_t)c * mr];
  int off = mr;
  for (int g = 0; g < J.ngroups; ++g) {
    const int k = *J.g[g].rank;
    const double* V = J.g[g].V + J.g[g].row0 + c;
    const int ld = J.g[g].ld;
    for (int t = threadIdx.x; t < k; t += NT_MM) h[off + t] = V[(int64_t)t * ld];
    off += k;
  }
}

// LDS layout of the leaf kernels (doubles)

// acc += (Y^T B) over the staged rows: wavefront w takes 4-row steps w, w+16, ...
__device__ __forceinline__ d4_t leaf_ytb_acc(const double* Ys, const double* Bs, int rn, d4_t acc) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nk = (rn + 3) >> 2;
  for (int ks = w; ks < nk; ks += 16) {
    const int r = 4 * ks + (l >> 4);
    acc = mfma16(Ys[r + (l & 15) * LF_LD], Bs[r + (l & 15) * LF_LD], acc);
  }
  return acc;
}

// Sum the 16 wavefronts' 16 x 16 tiles into out: out[i + NB j] (TOUT = false)
// or its transpose out[j + NB i] (TOUT = true).  The partial tiles are stored
// row by row (element (i, j) at j + NB i), so that the lanes of a wavefront,
// whose j runs fastest, write consecutive doubles (column by column, the
// 16-double stride put 8 lanes on each bank pair).
template <bool TOUT = false>
__device__ __forceinline__ void leaf_reduce_tile(d4_t acc, double* part, double* out) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = 4 * e + (l >> 4), j = l & 15;
    part[w * 256 + j + NB * i] = acc[e];
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    double sacc = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) sacc += part[q * 256 + threadIdx.x];
    const int j = threadIdx.x & 15, i = threadIdx.x >> 4;
    out[TOUT ? threadIdx.x : i + NB * j] = sacc;
  }
  __syncthreads();
}

// Unblocked Householder QR of panel columns [c0, c0+pw) over rows [c0, M):
// wavefront w owns column c0 + w, lane l owns rows c0 + l + 64 t.  Step j: the
// owner forms reflector j and broadcasts it through LDS, the wavefronts of the
// later columns apply it, and the wavefronts of the finished columns i < j
// form the Gram entries G[i, j] = v_i^T v_j meanwhile.  T then follows from G
// by eq. recqrcombined (below).
template <int RPT>
__device__ __forceinline__ void leaf_panel_rows(LeafWs W, int c0, int pw, int M, double* sm) {
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int h = M - c0;
  double* taus = sm + LF_TAU;
  double* gram = sm + LF_GRAM;
  gdouble* col = gmem(W.H) + (int64_t)(c0 + w) * MAXSTACK + c0;
  double a[RPT];
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int r = lane + 64 * t;
    a[t] = (w < pw && r < h) ? col[r] : 0.0;
  }
  wait_loads();
  for (int j = 0; j < pw; ++j) {
    double* vb = sm + LF_VBUF + (j & 1) * MAXSTACK;
    if (w == j) {
      double ss0 = 0.0, ss1 = 0.0;
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const int r = lane + 64 * t;
        const double x = (r > j) ? a[t] : 0.0;
        if (t & 1) ss1 += x * x; else ss0 += x * x;
      }
      const double ss = gsumt<64>(ss0 + ss1);
      const double al = lane_read(a[0], j);  // row j < 16 sits in t = 0
      double tau, beta, scal;
      house_scalars(al, ss, beta, tau, scal);
      const double sc = (ss != 0.0) ? scal : 1.0;
      {  // t = 0 holds rows 0..63, the only ones that can be <= j
        const int r = lane;
        const double x = a[0];
        const double v = (r > j) ? x * sc : (r == j ? 1.0 : 0.0);
        a[0] = (r > j) ? x * sc : (r == j ? beta : x);
        vb[r] = v;
      }
#pragma unroll
      for (int t = 1; t < RPT; ++t) {
        a[t] *= sc;
        vb[lane + 64 * t] = a[t];
      }
      if (lane == 0) taus[j] = tau;
      __builtin_amdgcn_s_setprio(0);
    }
    __syncthreads();
    if (w > j && w < pw) {
      // The owner of the next column runs the critical chain (this update,
      // then its own reflector before the next barrier): it issues ahead of
      // the other wavefronts on its SIMD until its reflector is out.
      if (w == j + 1) __builtin_amdgcn_s_setprio(3);
      // tau and v in one round of LDS reads; tau = 0 (a column already zero
      // below its diagonal, v = e_j) gives f = 0 and leaves a unchanged
      const double tau = taus[j];
      double v[RPT];
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        v[t] = vb[lane + 64 * t];
        if (t & 1) d1 += v[t] * a[t]; else d0 += v[t] * a[t];
      }
      const double f = tau * gsumt<64>(d0 + d1);
#pragma unroll
      for (int t = 0; t < RPT; ++t) a[t] -= f * v[t];
    } else if (w < j) {
      // a finished column: G[w, j] = v_w^T v_j (the Gram matrix for T) while
      // the later columns take reflector j
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const int r = lane + 64 * t;
        const double y = r > w ? a[t] : (r == w ? 1.0 : 0.0);
        if (t & 1) d1 += vb[r] * y; else d0 += vb[r] * y;
      }
      const double d = gsumt<64>(d0 + d1);
      if (lane == 0) gram[w + NB * j] = d;
    }
  }
#pragma unroll
  for (int t = 0; t < RPT; ++t) {
    const int r = lane + 64 * t;
    if (w < pw && r < h) col[r] = a[t];
  }
  __syncthreads();  // the last column's Gram entries
  // T by eq. recqrcombined, doubling the block size: on blocks B1 = [2ab, 2ab+b)
  // and B2 = [2ab+b, 2ab+2b), T[B1, B2] = -T[B1, B1] (Y_B1^T Y_B2) T[B2, B2].
  // Wavefront 0 alone (at most 64 entries per step), ordered by wavefront fences.
  double* Tp = sm + LF_TP;
  double* Xt = sm + LF_W;
  if (tid < 64) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + 64 * e, i = idx % NB, j = idx / NB;
      Tp[idx] = (i == j && i < pw) ? taus[i] : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int b = 1; b < NB; b *= 2) {
      const int bb = b * b;
      const bool act = tid < (NB / (2 * b)) * bb;
      const int pa = tid / bb, rc = tid % bb, r = rc % b, c = rc / b;
      const int i = 2 * pa * b + r, j = 2 * pa * b + b + c;
      if (act) {
        double x = 0.0;
        for (int k = 2 * pa * b + b; k < 2 * pa * b + 2 * b; ++k) x += gram[i + NB * k] * Tp[k + NB * j];
        Xt[i + NB * j] = x;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (act) {
        double y = 0.0;
        for (int k = 2 * pa * b; k < 2 * pa * b + b; ++k) y += Tp[i + NB * k] * Xt[k + NB * j];
        Tp[i + NB * j] = -y;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + 64 * e, i = idx % NB, j = idx / NB;
      if (i < pw && j < pw) gmem(W.T)[(int64_t)(c0 + i) + (int64_t)(c0 + j) * MAXLEAF] = Tp[idx];
    }
  }
}

__device__ __forceinline__ void leaf_panel(LeafWs W, int c0, int pw, int M, double* sm) {
  const int h = M - c0;  // rows per lane: as few as the panel's height allows
  if (h <= 128)
    leaf_panel_rows<2>(W, c0, pw, M, sm);
  else if (h <= 192)
    leaf_panel_rows<3>(W, c0, pw, M, sm);
  else if (h <= 256)
    leaf_panel_rows<4>(W, c0, pw, M, sm);
  else if (h <= 320)
    leaf_panel_rows<5>(W, c0, pw, M, sm);
  else if (h <= 576)
    leaf_panel_rows<9>(W, c0, pw, M, sm);
  else
    leaf_panel_rows<16>(W, c0, pw, M, sm);
}

// Y_p(r, j), panel p starting at column/row c0, for rows r >= c0
__device__ __forceinline__ double leaf_y(const LeafWs& W, int c0, int r, int j) {
  const int rr = r - c0;
  return rr < j ? 0.0 : (rr == j ? 1.0 : W.H[(int64_t)r + (int64_t)(c0 + j) * MAXSTACK]);
}

// Stage rows [r0, r0 + rn) of Y_p (unit lower panel at c0) and of the B
// columns [cb, cb + bw) (unmasked) into LDS, zero-padded to LF_CH rows.  All
// loads of a thread are issued (from clamped, in-bounds addresses) before any
// LDS store, so the staging costs one round trip to memory.
__device__ __forceinline__ void leaf_stage(const LeafWs& W, int c0, int pw, int r0, int rn, int cb,
                                           int bw, double* Ys, double* Bs) {
  constexpr int PER = (LF_CH * NB + NT_LEAF - 1) / NT_LEAF;
  const gdouble* H = gmem(W.H);
  double y[PER], bv[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * NT_LEAF;
    const int rr = e % LF_CH, jj = e / LF_CH;
    const bool row_ok = rr < rn && jj < NB;
    const int r = row_ok ? r0 + rr : r0;
    const int rel = r - c0;
    const double yv = H[(int64_t)r + (int64_t)(c0 + (jj < pw ? jj : 0)) * MAXSTACK];
    const double bb = H[(int64_t)r + (int64_t)(cb + (jj < bw ? jj : 0)) * MAXSTACK];
    y[q] = (row_ok && jj < pw) ? (rel < jj ? 0.0 : (rel == jj ? 1.0 : yv)) : 0.0;
    bv[q] = (row_ok && jj < bw) ? bb : 0.0;
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * NT_LEAF;
    if (e < LF_CH * NB) {
      const int rr = e % LF_CH, jj = e / LF_CH;
      Ys[rr + jj * LF_LD] = y[q];
      Bs[rr + jj * LF_LD] = bv[q];
    }
  }
}

// S = Y_p^T B over rows [c0, M) into sm[LF_W] (16 x 16, ld NB).
__device__ __forceinline__ void leaf_ytb(const LeafWs& W, int c0, int pw, int M, int cb, int bw,
                                         double* sm) {
  double* Ys = sm + LF_A;
  double* Bs = Ys + LF_LD * NB;
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = c0; r0 < M; r0 += LF_CH) {
    const int rn = min(LF_CH, M - r0);
    leaf_stage(W, c0, pw, r0, rn, cb, bw, Ys, Bs);
    __syncthreads();
    acc = leaf_ytb_acc(Ys, Bs, rn, acc);
    __syncthreads();
  }
  leaf_reduce_tile(acc, sm + LF_PART, sm + LF_W);
}

// Strip [cs, cs+sw) -= Y_p T_pp^T (Y_p^T strip)  (the block reflector of panel p),
// all three products on FP64 MFMA.  W = Y^T strip is summed over the
// wavefronts through LDS; every wavefront then forms W2 = T^T W itself (four
// MFMAs), whose result registers are already the B operand of the update
// MFMA, and writes its updated rows straight to global memory.
__device__ __forceinline__ void leaf_strip(const LeafWs& W, int c0, int pw, int M, int cs, int sw,
                                           double* sm) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  double* Ys = sm + LF_A;
  double* Bs = Ys + LF_LD * NB;
  double* Wt = sm + LF_W;
  double* Tt = Wt + 2 * NB * NB;
  double tval = 0.0;  // T_pp tile (transposed: T(i, j) at j + NB i), loaded with the first staging
  if (tid < 256) {
    const int j = tid & 15, i = tid >> 4;
    tval = (i <= j && i < pw && j < pw) ? gmem(W.T)[(int64_t)(c0 + i) + (int64_t)(c0 + j) * MAXLEAF] : 0.0;
  }
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
  const bool one_chunk = (M - c0) <= LF_CH;
  for (int r0 = c0; r0 < M; r0 += LF_CH) {
    const int rn = min(LF_CH, M - r0);
    leaf_stage(W, c0, pw, r0, rn, cs, sw, Ys, Bs);
    __syncthreads();
    acc = leaf_ytb_acc(Ys, Bs, rn, acc);
    if (!one_chunk) __syncthreads();
  }
  if (tid < 256) Tt[tid] = tval;
  leaf_reduce_tile<true>(acc, sm + LF_PART, Wt);  // W transposed: W(i, j) at j + NB i
  // W2 = T^T W: A[i][k] = T[k][i], B[k][j] = W[k][j]; D[i][j] sits in lane
  // j + 16 (i % 4), element i / 4, i.e. element e of lane l is W2[4e + l/16][l%16]:
  // the B operand of k-step e of the update below.  Both tiles are stored
  // transposed, so the lanes (l % 16 fastest) read consecutive doubles.
  d4_t w2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < NB; k0 += 4)
    w2 = mfma16(Tt[(l & 15) + NB * (k0 + (l >> 4))], Wt[(l & 15) + NB * (k0 + (l >> 4))], w2);
  for (int r0 = c0; r0 < M; r0 += LF_CH) {
    const int rn = min(LF_CH, M - r0);
    if (!one_chunk) {
      leaf_stage(W, c0, pw, r0, rn, cs, sw, Ys, Bs);
      __syncthreads();
    }
    const int nt = (rn + 15) >> 4;
    for (int t = w; t < nt; t += 16) {
      d4_t d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int e = 0; e < 4; ++e)
        d = mfma16(Ys[(16 * t + (l & 15)) + (4 * e + (l >> 4)) * LF_LD], w2[e], d);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = 16 * t + 4 * e + (l >> 4), col = l & 15;
        if (row < rn && col < sw)
          gmem(W.H)[(int64_t)(r0 + row) + (int64_t)(cs + col) * MAXSTACK] = Bs[row + col * LF_LD] - d[e];
      }
    }
    if (!one_chunk) __syncthreads();
  }
}

constexpr size_t LEAF_PANEL_LDS = LEAF_LDS;

// One step of the blocked leaf QR (see the section comment).  p = -1 only
// factorises panel 0; p = np only forms the last T block.
__global__ void __launch_bounds__(NT_LEAF) k_leaf_step(const LeafJob* __restrict__ jobs, int first,
                                                        int nper, int p) {
  extern __shared__ double sm[];
  const LeafJob& J = jobs[first + blockIdx.x / nper];
  if (*J.err & ERR_STACK) return;
  const LeafWs W = J.ws;
  double* fc = J.flops;
  const int tid = threadIdx.x;
  const int m = J.m;
  const int np = (m + NB - 1) / NB;
  const int M = leaf_rows(J);
  if (p < 0) {
    // the whole leaf's flops (Householder QR of M x m, Table 1, plus forming T
    // by eq. recqrcombined) are credited to this kernel's first launch
    if (tid == 0) {
      const double Mr = M, n = m;
      add_flops(fc, FC_LEAF, 2.0 * Mr * n * n - 2.0 / 3.0 * n * n * n + Mr * n * n - n * n * n / 3.0);
    }
    leaf_panel(W, 0, min(NB, m), M, sm);
    return;
  }
  const int c0 = p * NB, pw = min(NB, m - c0);
  const int nstrip = (p < np) ? np - p - 1 : 0;
  const int ngram = (p < np) ? p : 0;
  int b = blockIdx.x % nper;
  if (b < nstrip) {
    const int s = p + 1 + b;
    const int cs = s * NB, sw = min(NB, m - cs);
    leaf_strip(W, c0, pw, M, cs, sw, sm);
    if (b == 0) {  // look-ahead: the next panel is ready, factorise it
      __threadfence_block();
      __syncthreads();
      leaf_panel(W, cs, sw, M, sm);
    }
    return;
  }
  b -= nstrip;
  if (b < ngram) {
    // G[16b : 16b+16, c0 : c0+pw] = Y_b^T Y_p over rows >= c0 (Y_b has no mask there)
    leaf_ytb(W, c0, pw, M, b * NB, NB, sm);
    // leaf_ytb computed Y_p^T Y_b; store its transpose
    if (tid < 256) {
      const int i = tid & 15, j = tid >> 4;  // (Y_p^T Y_b)[i][j] = G[b*16 + j][c0 + i]
      if (i < pw) gmem(W.G)[(int64_t)(b * NB + j) + (int64_t)(c0 + i) * MAXLEAF] = sm[LF_W + i + j * NB];
    }
    return;
  }
  b -= ngram;
  // T block of panel q = p - 1, row tile b: T[16b : 16b+16, cq : cq+qw]
  const int q = p - 1;
  const int cq = q * NB, qw = min(NB, m - cq);
  const int i0 = b * NB;
  const int w = tid >> 6, l = tid & 63;
  double* X = sm + LF_W;
  double* Tq = X + NB * NB;
  if (tid < 256) {
    const int i = tid & 15, j = tid >> 4;
    Tq[tid] = (i <= j && i < qw && j < qw) ? gmem(W.T)[(int64_t)(cq + i) + (int64_t)(cq + j) * MAXLEAF] : 0.0;
  }
  // X = T[i0:i0+16, i0:cq] G[i0:cq, cq:cq+16]  (T upper: zero left of its diagonal)
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
  const int nk = (cq - i0) >> 2;
  for (int ks = w; ks < nk; ks += 16) {
    const int row = i0 + (l & 15), colT = i0 + 4 * ks + (l >> 4);
    const double a = (colT >= row) ? gmem(W.T)[(int64_t)row + (int64_t)colT * MAXLEAF] : 0.0;
    // columns of G beyond panel q's width are not part of this leaf: zero them
    // (X's columns >= qw then stay zero instead of carrying stale values)
    const double g = (l & 15) < qw
                         ? gmem(W.G)[(int64_t)(i0 + 4 * ks + (l >> 4)) + (int64_t)(cq + (l & 15)) * MAXLEAF]
                         : 0.0;
    acc = mfma16(a, g, acc);
  }
  leaf_reduce_tile(acc, sm + LF_PART, X);
  if (tid < 256) {
    const int i = tid & 15, j = tid >> 4;
    double sacc = 0.0;
#pragma unroll
    for (int q2 = 0; q2 < NB; ++q2) sacc += X[i + NB * q2] * Tq[q2 + NB * j];
    if (j < qw) gmem(W.T)[(int64_t)(i0 + i) + (int64_t)(cq + j) * MAXLEAF] = -sacc;
  }
}

// R + Y back into the leaf, Y rows back into the ancestors' right factors, T out.
__global__ void __launch_bounds__(NT_MM) k_leaf_scatter(const LeafJob* __restrict__ jobs, int first,
                                                         int nper) {
  const LeafJob& J = jobs[first + blockIdx.x / nper];
  if (*J.err & ERR_STACK) return;
  const LeafWs W = J.ws;
  const int c = blockIdx.x % nper;
  if (c >= J.m) return;
  const int m = J.m, mr = J.mr;
  const double* h = W.H + (int64_t)c * MAXSTACK;
  for (int r = threadIdx.x; r < mr; r += NT_MM) J.D[r + (int64_t)c * mr] = h[r];
  for (int r = threadIdx.x; r < m; r += NT_MM) J.Tleaf[r + (int64_t)c * m] = (r <= c) ? W.T[r + (int64_t)c * MAXLEAF] : 0.0;
  int off = mr;
  for (int g = 0; g < J.ngroups; ++g) {
    const int k = *J.g[g].rank;
    double* V = J.g[g].V + J.g[g].row0 + c;
    const int ld = J.g[g].ld;
    for (int t = threadIdx.x; t < k; t += NT_MM) V[(int64_t)t * ld] = h[off + t];
    off += k;
  }
}

// ------------------------------------------------------------------ vectors
}  // namespace hq

// Device kernels of the HODLR QR library (gfx950, wave64, FP64 throughout).
//
// Paper: Kressner & Susnjara, "Fast QR decomposition of HODLR matrices".
//  * reg_qr / reg_formq : Householder QR of a register-resident tile (one
//    reflector per column, Sec. 3's n = 1 case) and its explicit Q factor.
//  * k_tr_qr / k_tr_form: recompression T_tau of Sec. 2.1.1 for a batch of
//    blocks.  Both factors are reduced by a tall-skinny QR tree (chunks of CH
//    rows, then stacked R factors), the last block of a job runs a one-sided
//    Jacobi SVD of R1 R2^T, and the second kernel forms Q1 U_k and R (R1^T U_k).
//  * k_tr_small: the same recompression for factors of at most four chunks in
//    one launch (for widths <= 8 a TSQR inside one block, in registers).
//  * k_mm_proj / k_mm_apply: HODLR matrix times a tall-skinny block (Table 1,
//    matrix-vector product) for a whole sub-HODLR: all blocks of all levels in
//    one launch per phase.
//  * k_gemm_tall / k_gemm_red: small dense products of the update step.
//  * k_leaf_*: blocked Householder QR with compact WY factor of the stacked
//    leaf column (Alg. hQR at the lowest level, Alg. blockQR's T merge).
#include "common.h"

#include <float.h>

namespace hq {

// ------------------------------------------------------------------ helpers
// Device memory reached through pointers held in job structs.  A generic
// pointer compiles to flat instructions, which also count against the LDS
// counter, so the compiler waits for outstanding loads and stores before
// later memory operations; a pointer in the global address space compiles to
// global instructions that do not.
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ gdouble* gmem(double* p) { return (gdouble*)p; }

// Wait until this thread's vector memory loads have returned (s_waitcnt with
// vmcnt 0, the other counters at their maxima).  Used after loads whose values
// are later stored under divergent control flow: the compiler cannot see that
// every path has consumed them, so it would otherwise put a vmcnt(0) wait in
// front of each conditional store, and each such wait also waits for the
// stores before it.
__device__ __forceinline__ void wait_loads() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Cross-lane moves of a double through DPP (VALU, a few cycles) instead of
// ds_bpermute round trips.  CTRL is a gfx9 DPP control word.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi2, lo2);
}

__device__ __forceinline__ double swz_xor16(double x) {  // lane ^ 16 within 32 lanes
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const int lo2 = __builtin_amdgcn_ds_swizzle(lo, 0x401F);
  const int hi2 = __builtin_amdgcn_ds_swizzle(hi, 0x401F);
  return __hiloint2double(hi2, lo2);
}

__device__ __forceinline__ double lane_read(double x, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
  return __hiloint2double(hi, lo);
}

// Sum over aligned groups of W lanes (W = 1, 2, ..., 64); every lane of the
// group receives the group sum.  The 64-lane case needs the whole wave active.
template <int W>
__device__ __forceinline__ double gsumt(double x) {
  if constexpr (W >= 2) x += dpp_mov<0xB1>(x);   // quad_perm [1,0,3,2]
  if constexpr (W >= 4) x += dpp_mov<0x4E>(x);   // quad_perm [2,3,0,1]
  if constexpr (W >= 8) x += dpp_mov<0x141>(x);  // row_half_mirror
  if constexpr (W >= 16) x += dpp_mov<0x140>(x); // row_mirror
  if constexpr (W == 32) {
    const double r0 = lane_read(x, 0), r1 = lane_read(x, 16), r2 = lane_read(x, 32), r3 = lane_read(x, 48);
    x = ((int)(__lane_id()) < 32) ? r0 + r1 : r2 + r3;
  }
  if constexpr (W >= 64) x = (lane_read(x, 0) + lane_read(x, 16)) + (lane_read(x, 32) + lane_read(x, 48));
  return x;
}

// 1/x and sqrt(x) from the hardware estimates refined by Newton steps (a few
// ulp), much shorter dependency chains than the correctly rounded sequences.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ double sqrt_nr(double x) {  // x > 0
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  const double sq = x * y;
  return fma(0.5 * y, fma(-sq, sq, x), sq);
}

// Householder reflector of x = [alpha; x2] from alpha and ss = |x2|^2:
// beta = -sign(alpha) |x|, tau = (beta - alpha)/beta, scal = 1/(alpha - beta).
__device__ __forceinline__ void house_scalars(double al, double ss, double& beta, double& tau,
                                              double& scal) {
  if (ss == 0.0) {
    beta = al;
    tau = 0.0;
    scal = 0.0;
    return;
  }
  const double nrm = sqrt_nr(al * al + ss);
  beta = (al >= 0.0) ? -nrm : nrm;
  const double d = beta - al;  // never 0: |beta| >= |alpha| and opposite sign
  tau = d * rcp_nr(beta);
  scal = -rcp_nr(d);
}

typedef double d4_t __attribute__((ext_vector_type(4)));
// D += A B for A 16x4, B 4x16 (FP64 MFMA).  Lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; D[i][j] lives in lane j + 16*(i%4), element i/4.
__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double gsum(double x, int width) {
  switch (width) {
    case 1: return x;
    case 2: return gsumt<2>(x);
    case 4: return gsumt<4>(x);
    case 8: return gsumt<8>(x);
    case 16: return gsumt<16>(x);
    case 32: return gsumt<32>(x);
    default: return gsumt<64>(x);
  }
}

__device__ __forceinline__ int seg_n(const Seg& s) {
  return s.p ? (s.ncols_dev ? *s.ncols_dev : s.ncols) : 0;
}

__device__ __forceinline__ int rel_node(int u, int v) {
  const int du = 31 - __clz(u), dv = 31 - __clz(v);
  const int d = du - dv;
  return (1 << d) - 1 + (u - (v << d));
}

__device__ __forceinline__ void add_flops(double* fc, int cat, double f) {
  // striped by block so that thousands of blocks do not queue on one address
  if (fc && f != 0.0) atomicAdd(fc + cat * FC_STRIPE + (blockIdx.x % FC_STRIPE), f);
}

__device__ __forceinline__ int tier_of(int w) {
  return w <= 8 ? 8 : w <= 16 ? 16 : w <= 32 ? 32 : w <= 64 ? 64 : 128;
}

// Householder QR of a tile held in registers.  Thread (c, sub) owns column c
// and rows r = sub + TPC*i (i < RPT) of a (TPC*RPT) x W tile; the valid part
// is h x w (rows >= h are zero).  Reflector convention: for x = [alpha; x2]
// with x2 != 0, beta = -sign(alpha)|x|, tau = (beta - alpha)/beta,
// v = [1; x2/(alpha - beta)]; tau = 0 (identity) when x2 = 0.  On exit the
// tile holds R on and above the diagonal and v below it, taus[j] = tau_j.
// When `gram` is set, gram[c + j*gld] = v_c . v_j for c < j (used for T).
template <int TPC, int RPT>
__device__ __forceinline__ void reg_qr(double (&a)[RPT], int c, int sub, int h, int w, double* vbuf,
                       double* taus, double* gram, int gld) {
  constexpr int CHR = TPC * RPT;
  const int jmax = min(h, w);
  for (int j = 0; j < jmax; ++j) {
    double* vb = vbuf + (j & 1) * CHR;
    if (c == j) {
      double ss = 0.0, al = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = sub + TPC * i;
        if (r > j) ss += a[i] * a[i];
        if (r == j) al = a[i];
      }
      ss = gsumt<TPC>(ss);
      al = gsumt<TPC>(al);
      double tau, beta, scal;
      house_scalars(al, ss, beta, tau, scal);
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = sub + TPC * i;
        if (r > j) {
          if (ss != 0.0) a[i] *= scal;
          vb[r] = a[i];
        } else if (r == j) {
          a[i] = beta;
          vb[r] = 1.0;
        } else {
          vb[r] = 0.0;
        }
      }
      if (sub == 0) taus[j] = tau;
    }
    __syncthreads();
    const double tau = taus[j];
    if (tau != 0.0 && c > j && c < w) {
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) d += vb[sub + TPC * i] * a[i];
      d = gsumt<TPC>(d);
      const double f = tau * d;
      asm volatile("" ::: "memory");  // re-read v from LDS instead of holding it in registers
#pragma unroll
      for (int i = 0; i < RPT; ++i) a[i] -= f * vb[sub + TPC * i];
    }
    if (gram != nullptr && c < j) {
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) d += vb[sub + TPC * i] * a[i];
      d = gsumt<TPC>(d);
      if (sub == 0) gram[c + j * gld] = d;
    }
  }
}

// Explicit Q = H_0 H_1 ... H_{jmax-1} [I; 0] (h x w) from reg_qr's output,
// accumulated backwards; column c only changes under reflectors j <= c.
template <int TPC, int RPT>
__device__ __forceinline__ void reg_formq(const double (&a)[RPT], double (&q)[RPT], int c, int sub, int h, int w,
                          double* vbuf, const double* taus) {
  constexpr int CHR = TPC * RPT;
  const int jmax = min(h, w);
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = sub + TPC * i;
    q[i] = (r == c && r < h && c < w) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = jmax - 1; j >= 0; --j) {
    double* vb = vbuf + (j & 1) * CHR;
    if (c == j) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = sub + TPC * i;
        vb[r] = (r < j) ? 0.0 : (r == j ? 1.0 : a[i]);
      }
    }
    __syncthreads();
    const double tau = taus[j];
    if (tau != 0.0 && c >= j && c < w) {
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) d += vb[sub + TPC * i] * q[i];
      d = gsumt<TPC>(d);
      const double f = tau * d;
      asm volatile("" ::: "memory");
#pragma unroll
      for (int i = 0; i < RPT; ++i) q[i] -= f * vb[sub + TPC * i];
    }
  }
}

// As reg_formq, but the reflectors are read back from a column-major copy
// (ld CH) in global memory instead of the owners' registers (widest tier).
template <int TPC, int RPT>
__device__ __forceinline__ void reg_formq_g(const double* Va, double (&q)[RPT], int c, int sub, int h, int w,
                            double* vbuf, const double* taus) {
  constexpr int CHR = TPC * RPT;
  const int jmax = min(h, w);
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = sub + TPC * i;
    q[i] = (r == c && r < h && c < w) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = jmax - 1; j >= 0; --j) {
    double* vb = vbuf + (j & 1) * CHR;
    if (c == j) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = sub + TPC * i;
        vb[r] = (r < j) ? 0.0 : (r == j ? 1.0 : (r < h ? Va[r + (int64_t)j * CH] : 0.0));
      }
    }
    __syncthreads();
    const double tau = taus[j];
    if (tau != 0.0 && c >= j && c < w) {
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) d += vb[sub + TPC * i] * q[i];
      d = gsumt<TPC>(d);
      const double f = tau * d;
      asm volatile("" ::: "memory");
#pragma unroll
      for (int i = 0; i < RPT; ++i) q[i] -= f * vb[sub + TPC * i];
    }
  }
}

// ------------------------------------------------------------------ recompression
// LDS layout of k_tr_qr (doubles)
constexpr int TRS_VBUF = 0;
constexpr int TRS_TAU = 2 * CH;
constexpr int TRS_FLAG = TRS_TAU + WMAX;      // 16 doubles of int flags
constexpr int TRS_X = TRS_FLAG + 16;
constexpr int TRS_TOTAL = TRS_X + WMAX * WMAX + 2 * WMAX;   // X (+V for W<=64) + sig + perm
constexpr size_t TR_QR_LDS = sizeof(double) * (size_t)TRS_TOTAL;

__device__ __forceinline__ int tr_root_slot(int p0, int G) {
  int s = 0, cnt = p0;
  while (cnt > 1) {
    s += cnt;
    cnt = (cnt + G - 1) / G;
  }
  return s;
}

// Rotation of one-sided Jacobi for a column pair with a = |x_i|^2, b = |x_j|^2,
// g = x_i . x_j: false when |g| <= tol sqrt(a b) (tested squared); otherwise
// the (cs, sn) that makes the rotated pair orthogonal, the smaller angle with
// tan(2 theta) = 2g / (b - a) (the rotation of jacobi()).  Short dependency
// chain: with d = b - a and g2 = 2g scaled by a power of two (squares neither
// overflow nor underflow), r = |(d, g2)|, s = r + |d| and q = 1/sqrt(2 r s),
// cs = s q and sn = sign(d) g2 q (cs^2 + sn^2 = (s^2 + g2^2) / (2 r s) = 1).
__device__ __forceinline__ bool jac_rot_fast(double al, double be, double ga, double tol2, double& cs,
                                             double& sn) {
  if (!(ga != 0.0 && ga * ga > tol2 * (al * be))) return false;
  double d = be - al, g = 2.0 * ga;
  const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(d), fabs(g)));
  d = __builtin_ldexp(d, -e);
  g = __builtin_ldexp(g, -e);
  const double h2 = fma(d, d, g * g);  // in [1/4, 2]
  double y = __builtin_amdgcn_rsq(h2);
  y = y * fma(-0.5 * h2 * y, y, 1.5);
  y = y * fma(-0.5 * h2 * y, y, 1.5);
  const double r = h2 * y;
  const double s = r + fabs(d);
  const double u = 2.0 * r * s;
  double q = __builtin_amdgcn_rsq(u);
  q = q * fma(-0.5 * u * q, q, 1.5);
  q = q * fma(-0.5 * u * q, q, 1.5);
  cs = s * q;
  sn = (d >= 0.0 ? g : -g) * q;
  return true;
}

// One-sided Jacobi on the columns of X (w x w, ld lx), accumulating the
// rotations in V (ld lv).  Round-robin pairing; one pair per group of TPP
// lanes; a sweep ends when no pair needed a rotation.
__device__ __forceinline__ void jacobi(double* X, int lx, double* V, int lv, int w, int* sflag) {
  const int tid = threadIdx.x;
  const int n = w + (w & 1);
  if (n < 2) return;
  const int P = n / 2;
  int Pp = 1;
  while (Pp < P) Pp <<= 1;
  int TPP = NT_TR / Pp;
  if (TPP > 64) TPP = 64;
  const int p = tid / TPP, sub = tid % TPP;
  const double tol = (double)w * DBL_EPSILON;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) *sflag = 0;
    __syncthreads();
    for (int r = 0; r < n - 1; ++r) {
      if (p < P) {
        int i, j;
        if (p == 0) {
          i = r;
          j = n - 1;
        } else {
          i = (r + p) % (n - 1);
          j = (r - p + n - 1) % (n - 1);
        }
        if (i > j) {
          const int t = i;
          i = j;
          j = t;
        }
        const bool valid = j < w;
        double al = 0.0, be = 0.0, ga = 0.0;
        if (valid) {
          for (int row = sub; row < w; row += TPP) {
            const double xi = X[row + i * lx], xj = X[row + j * lx];
            al += xi * xi;
            be += xj * xj;
            ga += xi * xj;
          }
        }
        al = gsum(al, TPP);
        be = gsum(be, TPP);
        ga = gsum(ga, TPP);
        double cs, sn;
        if (valid && jac_rot_fast(al, be, ga, tol * tol, cs, sn)) {
          for (int row = sub; row < w; row += TPP) {
            const double xi = X[row + i * lx], xj = X[row + j * lx];
            X[row + i * lx] = cs * xi - sn * xj;
            X[row + j * lx] = sn * xi + cs * xj;
            const double vi = V[row + i * lv], vj = V[row + j * lv];
            V[row + i * lv] = cs * vi - sn * vj;
            V[row + j * lv] = sn * vi + cs * vj;
          }
          if (sub == 0) *sflag = 1;
        }
      }
      __syncthreads();
    }
    const int f = *sflag;
    __syncthreads();
    if (f == 0) break;
  }
}

// The same one-sided Jacobi for w <= WS (WS = 8 or 16) inside one wavefront.
// X (and V = X + WS*WS) are WS x WS in LDS with leading dimension WS, rows and
// columns beyond w zero (rotations keep them zero), so a lane loads, rotates and
// stores whole padded columns without branches.  Lane p rotates pair p of the
// round-robin schedule; a round costs no block barrier and no cross-lane
// reduction; the sweep test is a wavefront vote.  Same rotation and threshold as
// jacobi() (|g| > tol sqrt(a b) is tested squared).  All threads of the block
// call it; it ends with a block barrier.
template <int WS>
__device__ __forceinline__ void jacobi_small(double* X, int w) {
  double* V = X + WS * WS;
  const int tid = threadIdx.x;
  const int n = w + (w & 1);
  if (n >= 2 && tid < 64) {
    const int P = n / 2;
    const double tol = (double)w * DBL_EPSILON;
    const double tol2 = tol * tol;
    for (int sweep = 0; sweep < 40; ++sweep) {
      int rot = 0;
      for (int r = 0; r < n - 1; ++r) {
        int i = 0, j = 0;
        if (tid == 0) {
          i = r;
          j = n - 1;
        } else {
          i = (r + tid) % (n - 1);
          j = (r - tid + n - 1) % (n - 1);
        }
        if (i > j) {
          const int t = i;
          i = j;
          j = t;
        }
        if (tid < P && j < w) {
          double* xi = X + i * WS;
          double* xj = X + j * WS;
          double* vi = V + i * WS;
          double* vj = V + j * WS;
          double a[WS], b[WS], c[WS], d[WS];
#pragma unroll
          for (int row = 0; row < WS; ++row) {
            a[row] = xi[row];
            b[row] = xj[row];
            c[row] = vi[row];
            d[row] = vj[row];
          }
          double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
          for (int row = 0; row < WS; ++row) {
            al = fma(a[row], a[row], al);
            be = fma(b[row], b[row], be);
            ga = fma(a[row], b[row], ga);
          }
          double cs, sn;
          if (jac_rot_fast(al, be, ga, tol2, cs, sn)) {
#pragma unroll
            for (int row = 0; row < WS; ++row) {
              xi[row] = cs * a[row] - sn * b[row];
              xj[row] = sn * a[row] + cs * b[row];
              vi[row] = cs * c[row] - sn * d[row];
              vj[row] = sn * c[row] + cs * d[row];
            }
            rot = 1;
          }
        }
        // the next round reads columns other lanes of this wavefront wrote
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
      if (__ballot(rot) == 0) break;
    }
  }
  __syncthreads();
}

// Flops of one recompression (the oracle's counting: Householder QR of both
// factors, the product of the R factors, the SVD as 21 p^3, forming the factors).
__device__ __forceinline__ double qr_flops(double m, double n) {
  const double pp = fmin(m, n);
  return m >= n ? 2.0 * m * n * pp - 2.0 / 3.0 * pp * pp * pp : 2.0 * n * m * m - 2.0 / 3.0 * m * m * m;
}

__device__ __forceinline__ double tr_flops_full(int m0, int m1, int w, int k) {
  const double p1 = min(m0, w), p2 = min(m1, w);
  const double mp = fmax(p1, p2);
  return qr_flops(m0, w) + qr_flops(m1, w) + 2.0 * p1 * p2 * w + 21.0 * mp * mp * mp +
         4.0 * (double)m0 * p1 * k + 2.0 * (double)m1 * w * k;
}

__device__ __forceinline__ double tr_flops_orth(int m0, int m1, int w) {
  const double pq = (double)min(m0, w);
  return 2.0 * (2.0 * (double)m0 * w * pq - 2.0 / 3.0 * pq * pq * pq) + 2.0 * (double)w * w * m1;
}

// Last block of a job: SVD of R1 R2^T and the small factors U_k, P = R1^T U_k.
template <int W>
__device__ __forceinline__ void tr_svd(const TrJob& J, double* ws, int w, int n0a, int n0b, double* smem, int* err,
                       double* fc) {
  const int tid = threadIdx.x;
  constexpr int G = CH / W;
  double* hdr = ws + J.hdr;
  double* Uk = hdr + 8;
  double* P = Uk + WMAX * WMAX;
  const double* R1 = ws + J.side[0].node0 + (int64_t)tr_root_slot(J.side[0].p0, G) * TR_NODE;
  int* sflag = (int*)(smem + TRS_FLAG);
  const int m0 = J.side[0].m, m1 = J.side[1].m;
  const double tau = *J.tau;
  const int capk = J.cap, fcat = J.fc;
  int k;
  if (J.flags & TR_ORTH) {
    k = min(m0, w);
    for (int e = tid; e < w * k; e += NT_TR) {
      const int r = e % w, p = e / w;
      Uk[r + p * WMAX] = (r == p) ? 1.0 : 0.0;
      P[r + p * WMAX] = R1[p + r * WMAX];
    }
    if (tid == 0) add_flops(fc, fcat, tr_flops_orth(m0, m1, w));
  } else {
    const double* R2 = ws + J.side[1].node0 + (int64_t)tr_root_slot(J.side[1].p0, G) * TR_NODE;
    // w <= 16: X and V padded to WS x WS (zeros beyond w) for jacobi_small
    const int WSs = w <= 8 ? 8 : (w <= 16 ? 16 : 0);
    const int LX = WSs ? WSs : w;
    double* X = smem + TRS_X;
    double* V;
    int LV;
    if (WSs) {
      V = X + LX * LX;
      LV = LX;
    } else if (2 * w * w <= WMAX * WMAX) {  // X and V both in LDS
      V = X + w * w;
      LV = w;
    } else {
      V = hdr + 8 + 2 * WMAX * WMAX;
      LV = WMAX;
    }
    double* sig = smem + TRS_X + WMAX * WMAX;
    int* perm = (int*)(sig + WMAX);
    // stage R1 and R2 in LDS when they fit next to X and V
    const double* R1s = R1;
    const double* R2s = R2;
    int lr = WMAX;
    if (4 * LX * LX <= WMAX * WMAX) {
      double* r1 = X + 2 * LX * LX;
      double* r2 = r1 + w * w;
      for (int e = tid; e < w * w; e += NT_TR) {
        const int i = e % w, j = e / w;
        r1[e] = R1[i + j * WMAX];
        r2[e] = R2[i + j * WMAX];
      }
      R1s = r1;
      R2s = r2;
      lr = w;
      __syncthreads();
    }
    // X = R2 R1^T  (both upper triangular, w x w; zero padding up to LX)
    const int wx = WSs ? LX : w;
    for (int e = tid; e < wx * wx; e += NT_TR) {
      const int i = e % wx, j = e / wx;
      double sacc = 0.0;
      if (i < w && j < w)
        for (int l = max(i, j); l < w; ++l) sacc += R2s[i + l * lr] * R1s[j + l * lr];
      X[i + j * LX] = sacc;
      V[i + j * LV] = (i == j && i < w) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (WSs == 8)
      jacobi_small<8>(X, w);
    else if (WSs == 16)
      jacobi_small<16>(X, w);
    else
      jacobi(X, LX, V, LV, w, sflag);
    for (int cc = tid; cc < w; cc += NT_TR) {
      double sacc = 0.0;
      for (int r = 0; r < w; ++r) sacc += X[r + cc * LX] * X[r + cc * LX];
      sig[cc] = sqrt(sacc);
    }
    __syncthreads();
    for (int cc = tid; cc < w; cc += NT_TR) {
      int pos = 0;
      const double sc = sig[cc];
      for (int j = 0; j < w; ++j) {
        const double sj = sig[j];
        pos += (sj > sc || (sj == sc && j < cc)) ? 1 : 0;
      }
      perm[pos] = cc;
    }
    __syncthreads();
    k = 0;
    for (int j = 0; j < w; ++j) k += (sig[j] > tau) ? 1 : 0;
    if (k > capk) {
      if (tid == 0) atomicOr(err, ERR_CAPACITY);
      k = capk;
    }
    for (int e = tid; e < w * k; e += NT_TR) {
      const int r = e % w, p = e / w;
      const int pc = perm[p];
      Uk[r + p * WMAX] = V[r + pc * LV];
      double sacc = 0.0;
      for (int l = 0; l <= r; ++l) sacc += R1s[l + r * lr] * V[l + pc * LV];
      P[r + p * WMAX] = sacc;
    }
    if (tid == 0) add_flops(fc, fcat, tr_flops_full(m0, m1, w, k));
  }
  if (tid == 0) {
    hdr[0] = (double)w;
    hdr[1] = (double)k;
    hdr[2] = (double)n0a;
    hdr[3] = (double)n0b;
  }
}

template <int W>
// Returns true in the block that ran the SVD (the job's last block).
__device__ __forceinline__ bool tr_chunk(const TrJob& J, int side, int chunk, double* ws, int* counters, int* err,
                         double* fc, double* smem, int w, int n0a, int n0b) {
  constexpr int TPC = NT_TR / W;
  constexpr int RPT = CH / TPC;
  constexpr int G = CH / W;
  const int tid = threadIdx.x, c = tid / TPC, sub = tid % TPC;
  double* vbuf = smem + TRS_VBUF;
  double* taus = smem + TRS_TAU;
  int* sflag = (int*)(smem + TRS_FLAG);
  const TrSide S = J.side[side];
  const int n0 = side == 0 ? n0a : n0b;
  const Seg s0 = J.seg[side][0], s1 = J.seg[side][1];

  double a[RPT];
  int idx = chunk, count = S.p0;
  int64_t base = 0;  // first slot of the current level
  int row0 = (int)((int64_t)idx * S.m / S.p0);
  int h = (int)((int64_t)(idx + 1) * S.m / S.p0) - row0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = sub + TPC * i;
    double x = 0.0;
    if (r < h && c < w) {
      const int64_t gr = row0 + r;
      x = (c < n0) ? s0.scale * s0.p[gr + (int64_t)c * s0.ld]
                   : s1.scale * s1.p[gr + (int64_t)(c - n0) * s1.ld];
    }
    a[i] = x;
  }
  int64_t slot = idx;
  while (true) {
    reg_qr<TPC, RPT>(a, c, sub, h, w, vbuf, taus, nullptr, 0);
    double* node = ws + S.node0 + slot * TR_NODE;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = sub + TPC * i;
      if (c < w && r < w) node[r + c * WMAX] = (r <= c && r < h) ? a[i] : 0.0;
    }
    if (side == 0) {
      double q[RPT];
      double* Qa = node + WMAX * WMAX;
      if constexpr (W <= 32) {
        __syncthreads();
        reg_formq<TPC, RPT>(a, q, c, sub, h, w, vbuf, taus);
      } else {
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int r = sub + TPC * i;
          if (r < h && c < w) Qa[r + c * CH] = a[i];
        }
        __threadfence_block();
        __syncthreads();
        reg_formq_g<TPC, RPT>(Qa, q, c, sub, h, w, vbuf, taus);
      }
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = sub + TPC * i;
        if (r < h && c < w) Qa[r + c * CH] = q[i];
      }
    }
    if (count == 1) break;
    const int pidx = idx / G;
    const int pcount = (count + G - 1) / G;
    const int nchild = min(G, count - pidx * G);
    const int64_t pbase = base + count;
    const int64_t pslot = pbase + pidx;
    __threadfence();
    __syncthreads();
    if (tid == 0) {
      int* cnt = counters + S.cnt0 + (int)(pslot - S.p0);
      const int old = atomicAdd(cnt, 1);
      const int last = (old == nchild - 1) ? 1 : 0;
      if (last) atomicExch(cnt, 0);
      sflag[0] = last;
    }
    __syncthreads();
    const int last = sflag[0];
    __syncthreads();
    if (!last) return false;
    __threadfence();
    // become the parent: stack the children's R factors
    const int64_t cbase = base;
    const int cfirst = pidx * G;
    base = pbase;
    idx = pidx;
    count = pcount;
    slot = pslot;
    h = nchild * w;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = sub + TPC * i;
      double x = 0.0;
      if (r < h && c < w) {
        const int ch = r / w, rr = r % w;
        x = ws[S.node0 + (cbase + cfirst + ch) * TR_NODE + rr + c * WMAX];
      }
      a[i] = x;
    }
  }
  // this side is reduced; join the two sides
  if (!(J.flags & TR_ORTH)) {
    __threadfence();
    __syncthreads();
    if (tid == 0) {
      int* cnt = counters + J.jcounter;
      const int old = atomicAdd(cnt, 1);
      const int last = (old == 1) ? 1 : 0;
      if (last) atomicExch(cnt, 0);
      sflag[0] = last;
    }
    __syncthreads();
    const int last = sflag[0];
    __syncthreads();
    if (!last) return false;
    __threadfence();
  }
  tr_svd<W>(J, ws, w, n0a, n0b, smem, err, fc);
  return true;
}

// WTOP: widest tier compiled into this instantiation (the host picks it from
// the rank capacity: a recompression is at most twice as wide as a block).
template <int WTOP>
__global__ void __launch_bounds__(NT_TR) k_tr_qr(const TrJob* __restrict__ jobs,
                                                  const TrChunk* __restrict__ items, int first,
                                                  double* ws, int* counters) {
  extern __shared__ double smem[];
  const TrChunk it = items[first + blockIdx.x];
  const TrJob& J = jobs[it.job];
  int* err = J.err;
  double* fc = J.flops;
  const int n0a = seg_n(J.seg[0][0]);
  const int w = n0a + seg_n(J.seg[0][1]);
  const int n0b = seg_n(J.seg[1][0]);
  if (w == 0 || w > WTOP) {
    if (it.side == 0 && it.chunk == 0 && threadIdx.x == 0) {
      double* hdr = ws + J.hdr;
      hdr[0] = 0.0;
      hdr[1] = 0.0;
      if (w > WTOP) atomicOr(err, ERR_WIDTH);
    }
    return;
  }
  const int t = tier_of(w);
  if (t == 8) {
    tr_chunk<8>(J, it.side, it.chunk, ws, counters, err, fc, smem, w, n0a, n0b);
  } else if (t == 16) {
    if constexpr (WTOP >= 16) tr_chunk<16>(J, it.side, it.chunk, ws, counters, err, fc, smem, w, n0a, n0b);
  } else if (t == 32) {
    if constexpr (WTOP >= 32) tr_chunk<32>(J, it.side, it.chunk, ws, counters, err, fc, smem, w, n0a, n0b);
  } else if (t == 64) {
    if constexpr (WTOP >= 64) tr_chunk<64>(J, it.side, it.chunk, ws, counters, err, fc, smem, w, n0a, n0b);
  } else {
    if constexpr (WTOP >= 128) tr_chunk<128>(J, it.side, it.chunk, ws, counters, err, fc, smem, w, n0a, n0b);
  }
}

constexpr size_t TR_FORM_LDS = sizeof(double) * (size_t)WMAX * WMAX;

// out[r, p] = sum_c A(r, c) B[c + p*ldb] for r < rows, p < k; thread = row
// (NT threads), 16 output columns at a time in registers.  A(r, c) = a[r + c*lda].
template <int NT = NT_MM>
__device__ __forceinline__ void rows_times_small(const double* a, int64_t lda, int rows, int w,
                                                 const double* B, int ldb, int k, double* out,
                                                 int64_t ldo) {
  const int tid = threadIdx.x;
  for (int r = tid; r < rows; r += NT) {
    for (int p0 = 0; p0 < k; p0 += 16) {
      double acc[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = 0.0;
#pragma unroll 4
      for (int c = 0; c < w; ++c) {
        const double x = a[r + (int64_t)c * lda];
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (p0 + q < k) acc[q] += x * B[c + (p0 + q) * ldb];
      }
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (p0 + q < k) out[r + (int64_t)(p0 + q) * ldo] = acc[q];
    }
  }
}

__global__ void __launch_bounds__(NT_MM) k_tr_form(const TrJob* __restrict__ jobs,
                                                    const TrForm* __restrict__ items, int first,
                                                    const double* __restrict__ ws) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const TrForm it = items[first + blockIdx.x];
  const TrJob& J = jobs[it.job];
  const double* hdr = ws + J.hdr;
  const int w = (int)hdr[0], k = (int)hdr[1];
  // the header is written by k_tr_qr for every job; refuse anything else
  if (w < 0 || w > WMAX || k < 0 || k > w || k > J.cap) return;
  if (it.leader && tid == 0) *J.out_rank = k;
  if (w == 0 || k == 0) return;
  const double* Uk = hdr + 8;
  const double* P = Uk + WMAX * WMAX;
  const int G = CH / tier_of(w);
  if (it.side == 0) {
    const TrSide S = J.side[0];
    double* out = J.out[0];
    const int ldo = J.ldout[0];
    // path of tree indices from the chunk to the root
    int idxs[16], bases[16];
    int lvl = 0, idx = it.chunk, count = S.p0, base = 0;
    idxs[0] = idx;
    bases[0] = 0;
    while (count > 1) {
      base += count;
      idx /= G;
      count = (count + G - 1) / G;
      ++lvl;
      idxs[lvl] = idx;
      bases[lvl] = base;
    }
    // Z = U_k (w x k, ld w), then Z <- Q_node[slot rows] Z down the path
    double* Z = smem;
    double* Zn = smem + w * k;
    const bool fits = 2 * w * k <= WMAX * WMAX;
    for (int e = tid; e < w * k; e += NT_MM) Z[e] = Uk[(e % w) + (e / w) * WMAX];
    __syncthreads();
    for (int l = lvl; l >= 1; --l) {
      const int cslot = idxs[l - 1] - idxs[l] * G;
      const double* Qn = ws + S.node0 + (int64_t)(bases[l] + idxs[l]) * TR_NODE + WMAX * WMAX + cslot * w;
      if (fits) {
        rows_times_small(Qn, CH, w, w, Z, w, k, Zn, w);
        __syncthreads();
        for (int e = tid; e < w * k; e += NT_MM) Z[e] = Zn[e];
        __syncthreads();
      } else {
        // wide case: one column of Z at a time through registers
        for (int p = 0; p < k; ++p) {
          double zr = 0.0;
          if (tid < w)
            for (int c = 0; c < w; ++c) zr += Qn[tid + (int64_t)c * CH] * Z[c + p * w];
          __syncthreads();
          if (tid < w) Z[tid + p * w] = zr;
          __syncthreads();
        }
      }
    }
    const int row0 = (int)((int64_t)it.chunk * S.m / S.p0);
    const int h = (int)((int64_t)(it.chunk + 1) * S.m / S.p0) - row0;
    const double* Qc = ws + S.node0 + (int64_t)it.chunk * TR_NODE + WMAX * WMAX;
    rows_times_small(Qc, CH, h, w, Z, w, k, out + row0, ldo);
  } else {
    const int n0 = (int)hdr[3];
    const Seg s0 = J.seg[1][0], s1 = J.seg[1][1];
    double* out = J.out[1];
    const int ldo = J.ldout[1];
    double* In = smem;                 // rows x w, ld 64
    double* Ps = smem + 64 * w;        // w x k, ld w
    const bool fits = 64 * w + w * k <= WMAX * WMAX;
    const int rows = it.rows;
    for (int e = tid; e < rows * w; e += NT_MM) {
      const int r = e % rows, cc = e / rows;
      const int64_t gr = it.row0 + r;
      In[r + cc * 64] = (cc < n0) ? s0.scale * s0.p[gr + (int64_t)cc * s0.ld]
                                  : s1.scale * s1.p[gr + (int64_t)(cc - n0) * s1.ld];
    }
    if (fits)
      for (int e = tid; e < w * k; e += NT_MM) Ps[e] = P[(e % w) + (e / w) * WMAX];
    __syncthreads();
    if (fits)
      rows_times_small(In, 64, rows, w, Ps, w, k, out + it.row0, ldo);
    else
      rows_times_small(In, 64, rows, w, P, WMAX, k, out + it.row0, ldo);
  }
}

// ------------------------------------------------------------------ one-block recompression
// A recompression whose two factors have at most TRS_MAXCH chunks each (rows
// split evenly, at most CH per chunk) in one launch, without the tree in
// global memory or the forming kernel.  Width w <= 8: a TSQR inside one block.
// Wavefront c < 4 factorises chunk c of L and wavefront 4 + c chunk c of R in
// registers (wave_qr); wavefronts 4 and 5 factorise the stacked chunk R
// factors; wavefront 4 runs the SVD of R2 R1^T (jacobi_wave) and applies the
// stacked Q factor of L to [U_k; 0]; then wavefront c applies its chunk's Q to
// its rows of that product (L' = Q1 U_k) and wavefront 4 + c forms its rows of
// R (R1^T U_k).  Wider jobs run the chunk code of k_tr_qr in one block per
// chunk and the block that ran the SVD forms both factors.
constexpr int TRS_MAXCH = 4;

// Load rows [r0, r0 + h) of the factor [seg0 | seg1] (n0 columns in seg0)
// into a wavefront's tile: lane l holds rows r0 + l + 64 i, columns < WT (zero
// beyond w and h).
template <int WT>
__device__ __forceinline__ void wave_load(double (&a)[4][WT], const Seg& s0, const Seg& s1, int n0, int r0,
                                          int h, int w) {
  const int lane = threadIdx.x & 63;
  if (h <= 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < WT; ++c) a[i][c] = 0.0;
    return;
  }
  // every load is issued (elements outside the tile read the factor's first
  // element, which exists for w >= 1 and h >= 1) before any is used
  const double* base = (n0 > 0) ? s0.p : s1.p;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = lane + 64 * i;
    const int64_t gr = r0 + r;
#pragma unroll
    for (int c = 0; c < WT; ++c) {
      const bool ok = r < h && c < w;
      const double* src = (c < n0) ? s0.p + gr + (int64_t)c * s0.ld : s1.p + gr + (int64_t)(c - n0) * s1.ld;
      a[i][c] = *(ok ? src : base);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = lane + 64 * i;
#pragma unroll
    for (int c = 0; c < WT; ++c) a[i][c] = (r < h && c < w) ? ((c < n0) ? s0.scale : s1.scale) * a[i][c] : 0.0;
  }
}

// Householder QR of the h x w tile of one wavefront (w <= WT, h <= 256), the
// reflector convention of reg_qr.  On exit R is on and above the diagonal, v
// below it, tau[j] in registers (0 past min(h, w)).  The products with the
// later columns are independent and run interleaved (columns past w are zero
// and stay zero).
template <int WT>
__device__ __forceinline__ void wave_qr(double (&a)[4][WT], int h, int w, double (&tau)[WT]) {
  const int lane = threadIdx.x & 63;
  const int jmax = min(h, w);
#pragma unroll
  for (int j = 0; j < WT; ++j) {
    tau[j] = 0.0;
    if (j < jmax) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double x = (lane + 64 * i > j) ? a[i][j] : 0.0;
        if (i & 1) s1 += x * x; else s0 += x * x;
      }
      const double ss = gsumt<64>(s0 + s1);
      const double al = lane_read(a[0][j], j);
      double tj, beta, scal;
      house_scalars(al, ss, beta, tj, scal);
      const double sc = (ss != 0.0) ? scal : 1.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = lane + 64 * i;
        a[i][j] = (r > j) ? a[i][j] * sc : (r == j ? beta : a[i][j]);
      }
      tau[j] = tj;
      if (tj != 0.0) {
        double f[WT];
#pragma unroll
        for (int c = j + 1; c < WT; ++c) {
          double d0 = 0.0, d1 = 0.0;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double v = (lane + 64 * i > j) ? a[i][j] : 0.0;
            if (i & 1) d1 += v * a[i][c]; else d0 += v * a[i][c];
          }
          f[c] = tj * (gsumt<64>(d0 + d1) + lane_read(a[0][c], j));
        }
#pragma unroll
        for (int c = j + 1; c < WT; ++c) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = lane + 64 * i;
            const double v = (r > j) ? a[i][j] : (r == j ? 1.0 : 0.0);
            a[i][c] -= f[c] * v;
          }
        }
      }
    }
  }
}

// Z <- H_0 H_1 ... H_{jmax-1} Z for the reflectors of wave_qr (columns of a)
// on the wavefront's tile Z (columns < WT).
template <int WT>
__device__ __forceinline__ void wave_apply_q(const double (&a)[4][WT], const double (&tau)[WT], int jmax,
                                             double (&z)[4][WT]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = WT - 1; j >= 0; --j) {
    if (j < jmax && tau[j] != 0.0) {
      double f[WT];
#pragma unroll
      for (int c = 0; c < WT; ++c) {
        double d0 = 0.0, d1 = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = lane + 64 * i;
          const double v = (r > j) ? a[i][j] : (r == j ? 1.0 : 0.0);
          if (i & 1) d1 += v * z[i][c]; else d0 += v * z[i][c];
        }
        f[c] = tau[j] * gsumt<64>(d0 + d1);
      }
#pragma unroll
      for (int c = 0; c < WT; ++c) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int r = lane + 64 * i;
          const double v = (r > j) ? a[i][j] : (r == j ? 1.0 : 0.0);
          z[i][c] -= f[c] * v;
        }
      }
    }
  }
}

// One-sided Jacobi (rotation and threshold of jacobi_small) on the w <= WT
// columns of X (WT x WT, ld WT, zero beyond w), rotations accumulated in V, by
// one wavefront: lane (p, r) = (lane / WT, lane % WT) holds row r of column
// pair p of the round-robin schedule and the pair's sums are WT-lane reductions.
template <int WT>
__device__ __forceinline__ void jacobi_wave(double* X, double* V, int w) {
  const int lane = threadIdx.x & 63;
  const int n = w + (w & 1);
  if (n < 2) return;
  const int P = n / 2;
  const int p = lane / WT, r = lane % WT;
  const double tol = (double)w * DBL_EPSILON;
  const double tol2 = tol * tol;
  for (int sweep = 0; sweep < 40; ++sweep) {
    int rot = 0;
    for (int rd = 0; rd < n - 1; ++rd) {
      int i = 0, j = 0;
      if (p == 0) {
        i = rd;
        j = n - 1;
      } else {  // (rd + p) mod (n - 1) and (rd - p) mod (n - 1), p < n/2
        i = rd + p;
        if (i >= n - 1) i -= n - 1;
        j = rd - p;
        if (j < 0) j += n - 1;
      }
      if (i > j) {
        const int t = i;
        i = j;
        j = t;
      }
      const bool live = p < P;
      double xi = 0.0, xj = 0.0, vi = 0.0, vj = 0.0;
      if (live) {
        xi = X[r + i * WT];
        xj = X[r + j * WT];
        vi = V[r + i * WT];
        vj = V[r + j * WT];
      }
      const double al = gsumt<WT>(xi * xi), be = gsumt<WT>(xj * xj), ga = gsumt<WT>(xi * xj);
      double cs, sn;
      if (live && j < w && jac_rot_fast(al, be, ga, tol2, cs, sn)) {
        X[r + i * WT] = cs * xi - sn * xj;
        X[r + j * WT] = sn * xi + cs * xj;
        V[r + i * WT] = cs * vi - sn * vj;
        V[r + j * WT] = sn * vi + cs * vj;
        rot = 1;
      }
      // the next round reads columns that other lanes wrote
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    if (__ballot(rot) == 0) break;
  }
}

// LDS layout of the narrow path (doubles): the stacked chunk R factors of
// both sides (TRS_MAXCH*WT x WT, ld 32), the stacked product Q_top [U_k; 0]
// (ld 32), R1, R2, X, V, U_k, P (WT x WT, ld WT), then ints.
constexpr int TSM_S0 = 0, TSM_S1 = 256, TSM_Z = 512, TSM_R1 = 768, TSM_R2 = 832, TSM_X = 896, TSM_V = 960,
              TSM_U = 1024, TSM_P = 1088, TSM_INT = 1152;
constexpr int TSM_LD = 32;

// chunk c of nc over m rows: [row0, row0 + h)
__device__ __forceinline__ void tr_chunk_rows(int m, int nc, int c, int& row0, int& h) {
  row0 = (int)((int64_t)c * m / nc);
  h = (int)((int64_t)(c + 1) * m / nc) - row0;
}

template <int WT>
__device__ __forceinline__ void tr_small_narrow(const TrJob& J, int w, int n0a, int n0b, double* sm) {
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const bool orth = (J.flags & TR_ORTH) != 0;
  const int m0 = J.side[0].m, m1 = J.side[1].m;
  const int nc0 = max(1, (m0 + CH - 1) / CH), nc1 = max(1, (m1 + CH - 1) / CH);
  double* S0 = sm + TSM_S0;
  double* S1 = sm + TSM_S1;
  double* Zt = sm + TSM_Z;
  double* R1 = sm + TSM_R1;
  double* R2 = sm + TSM_R2;
  double* X = sm + TSM_X;
  double* V = sm + TSM_V;
  double* Uk = sm + TSM_U;
  double* P = sm + TSM_P;
  int* perm = (int*)(sm + TSM_INT);
  const int side = wv >> 2, c = wv & 3;  // this wavefront's chunk
  int row0 = 0, h = 0;
  if (side == 0 && c < nc0) tr_chunk_rows(m0, nc0, c, row0, h);
  if (side == 1 && c < nc1) tr_chunk_rows(m1, nc1, c, row0, h);
  double a[4][WT];  // the chunk's tile; wavefronts 4, 5 then the stacked R factors
  double tau[WT];
#pragma unroll
  for (int j = 0; j < WT; ++j) tau[j] = 0.0;
  // chunk QRs; their R factors stacked in LDS
  if (side == 0 ? c < nc0 : (!orth && c < nc1)) {
    if (side == 0)
      wave_load<WT>(a, J.seg[0][0], J.seg[0][1], n0a, row0, h, w);
    else
      wave_load<WT>(a, J.seg[1][0], J.seg[1][1], n0b, row0, h, w);
    wave_qr<WT>(a, h, w, tau);
    double* S = side == 0 ? S0 : S1;
    if (lane < WT) {
#pragma unroll
      for (int q = 0; q < WT; ++q) S[c * WT + lane + q * TSM_LD] = (lane <= q) ? a[0][q] : 0.0;
    }
  }
  __syncthreads();
  // R1 (wavefront 4) and R2 (wavefront 5): QR of the stacked chunk factors
  // (their own chunk's reflectors are no longer needed)
  const int ncs = (wv == 4) ? nc0 : nc1;
  if (wv == 4 || (wv == 5 && !orth)) {
    const double* S = (wv == 4) ? S0 : S1;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < WT; ++q) a[i][q] = (i == 0 && lane < ncs * WT) ? S[lane + q * TSM_LD] : 0.0;
#pragma unroll
    for (int j = 0; j < WT; ++j) tau[j] = 0.0;
    if (ncs > 1) wave_qr<WT>(a, ncs * WT, w, tau);
    double* R = (wv == 4) ? R1 : R2;
    if (lane < WT) {
#pragma unroll
      for (int q = 0; q < WT; ++q) R[lane + q * WT] = (lane <= q) ? a[0][q] : 0.0;
    }
  }
  __syncthreads();
  int k = 0;
  if (wv == 4) {
    const double thr = *J.tau;
    if (orth) {
      k = min(m0, w);
      if (lane < WT * WT) {
        const int rr = lane % WT, pp = lane / WT;
        Uk[lane] = (rr == pp && pp < k) ? 1.0 : 0.0;
        P[lane] = (pp < k) ? R1[pp + rr * WT] : 0.0;  // P = R1^T [I_k; 0]
      }
    } else {
      // X = R2 R1^T (upper triangular factors, zero beyond w), V = I
      if (lane < WT * WT) {
        const int ii = lane % WT, jj = lane / WT;
        double s = 0.0;
        for (int l = max(ii, jj); l < w; ++l) s += R2[ii + l * WT] * R1[jj + l * WT];
        X[lane] = s;
        V[lane] = (ii == jj && ii < w) ? 1.0 : 0.0;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      jacobi_wave<WT>(X, V, w);
      // singular values (column norms), their descending order, and k (sig > tau)
      double sg = -1.0;
      if (lane < w) {
        double s = 0.0;
        for (int rr = 0; rr < WT; ++rr) s += X[rr + lane * WT] * X[rr + lane * WT];
        sg = sqrt(s);
      }
      int pos = 0;
#pragma unroll
      for (int jj = 0; jj < WT; ++jj) {
        const double sj = lane_read(sg, jj);
        pos += (jj < w && (sj > sg || (sj == sg && jj < lane))) ? 1 : 0;
      }
      if (lane < w) perm[pos] = lane;
      k = __popcll(__ballot(lane < w && sg > thr));
      if (k > J.cap) {
        if (lane == 0) atomicOr(J.err, ERR_CAPACITY);
        k = J.cap;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // U_k = V[:, perm[:k]], P = R1^T U_k
      if (lane < WT * WT) {
        const int rr = lane % WT, pp = lane / WT;
        Uk[lane] = (pp < k && rr < w) ? V[rr + perm[pp] * WT] : 0.0;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (lane < WT * WT) {
        const int rr = lane % WT, pp = lane / WT;
        double s = 0.0;
        for (int l = 0; l <= rr; ++l) s += R1[l + rr * WT] * Uk[l + pp * WT];
        P[lane] = (pp < k && rr < w) ? s : 0.0;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // Zt = Q_top [U_k; 0] (stacked rows; Q_top = I for one chunk)
    double z[4][WT];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < WT; ++q) z[i][q] = (i == 0 && lane < WT) ? Uk[lane + q * WT] : 0.0;
    if (nc0 > 1) wave_apply_q<WT>(a, tau, w, z);
    if (lane < nc0 * WT) {
#pragma unroll
      for (int q = 0; q < WT; ++q) Zt[lane + q * TSM_LD] = z[0][q];
    }
    if (lane == 0) {
      *J.out_rank = k;
      perm[WT] = k;  // for the other wavefronts
      add_flops(J.flops, J.fc, orth ? tr_flops_orth(m0, m1, w) : tr_flops_full(m0, m1, w, k));
    }
  }
  __syncthreads();
  k = perm[WT];
  if (side == 0 && c < nc0) {
    // rows of L' = Q_c [Zt rows of chunk c; 0] (rows past min(h, w) are zero)
    double z[4][WT];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = lane + 64 * i;
#pragma unroll
      for (int q = 0; q < WT; ++q) z[i][q] = (i == 0 && r < WT && r < h) ? Zt[c * WT + r + q * TSM_LD] : 0.0;
    }
    wave_apply_q<WT>(a, tau, min(h, w), z);
    double* out = J.out[0];
    const int ld = J.ldout[0];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = lane + 64 * i;
#pragma unroll
      for (int q = 0; q < WT; ++q)
        if (r < h && q < k) out[row0 + r + (int64_t)q * ld] = z[i][q];
    }
  } else if (side == 1 && c < nc1) {
    // rows of R' = R P (R read again: it is cached)
    double b[4][WT];
    wave_load<WT>(b, J.seg[1][0], J.seg[1][1], n0b, row0, h, w);
    double* out = J.out[1];
    const int ld = J.ldout[1];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = lane + 64 * i;
#pragma unroll
      for (int q = 0; q < WT; ++q) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < WT; ++l) s += b[i][l] * P[l + q * WT];
        if (r < h && q < k) out[row0 + r + (int64_t)q * ld] = s;
      }
    }
  }
}

// Forming step inside the block that ran the SVD (k_tr_form for a tree of
// at most one combine level): L' = Q_chunk (Q_root rows of the chunk) U_k for
// each chunk of side 0, and R' = R P, from the header tr_svd wrote.
__device__ __forceinline__ void tr_small_form(const TrJob& J, const double* ws, double* sm) {
  const int tid = threadIdx.x;
  const double* hdr = ws + J.hdr;
  const int w = (int)hdr[0], k = (int)hdr[1];
  if (w < 0 || w > WMAX || k < 0 || k > w || k > J.cap) return;
  if (tid == 0) *J.out_rank = k;
  if (w == 0 || k == 0) return;
  const double* Uk = hdr + 8;
  const double* P = Uk + WMAX * WMAX;
  const TrSide S = J.side[0];
  double* Z = sm;           // U_k (w x k, ld w)
  double* Zc = sm + w * k;  // Q_root rows of a chunk times U_k
  for (int e = tid; e < w * k; e += NT_TR) Z[e] = Uk[(e % w) + (e / w) * WMAX];
  __syncthreads();
  for (int c = 0; c < S.p0; ++c) {
    int row0, h;
    tr_chunk_rows(S.m, S.p0, c, row0, h);
    const double* Zuse = Z;
    if (S.p0 > 1) {
      const double* Qn = ws + S.node0 + (int64_t)S.p0 * TR_NODE + WMAX * WMAX + c * w;
      rows_times_small<NT_TR>(Qn, CH, w, w, Z, w, k, Zc, w);
      __syncthreads();
      Zuse = Zc;
    }
    const double* Qc = ws + S.node0 + (int64_t)c * TR_NODE + WMAX * WMAX;
    rows_times_small<NT_TR>(Qc, CH, h, w, Zuse, w, k, J.out[0] + row0, J.ldout[0]);
    __syncthreads();
  }
  // R' = R P.  R' may overwrite R in place (row r of R' over row r of R), so a
  // thread computes all k outputs of its row before it writes them: with
  // k <= 16 it reads its row straight from the segments (coalesced over the
  // threads), otherwise 64-row pieces of R are staged in LDS first.
  const int n0 = (int)hdr[3];
  const Seg s0 = J.seg[1][0], s1 = J.seg[1][1];
  if (k <= 16) {
    double* Ps = sm;  // w x k, ld w
    for (int e = tid; e < w * k; e += NT_TR) Ps[e] = P[(e % w) + (e / w) * WMAX];
    __syncthreads();
    for (int r = tid; r < J.side[1].m; r += NT_TR) {
      double acc[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] = 0.0;
      for (int c = 0; c < w; ++c) {
        const double x = (c < n0) ? s0.scale * s0.p[r + (int64_t)c * s0.ld]
                                  : s1.scale * s1.p[r + (int64_t)(c - n0) * s1.ld];
#pragma unroll
        for (int q = 0; q < 16; ++q)
          if (q < k) acc[q] += x * Ps[c + q * w];
      }
#pragma unroll
      for (int q = 0; q < 16; ++q)
        if (q < k) J.out[1][r + (int64_t)q * J.ldout[1]] = acc[q];
    }
    return;
  }
  double* In = sm;           // rows x w, ld 64
  double* Ps = sm + 64 * w;  // w x k, ld w
  const bool fits = 64 * w + w * k <= WMAX * WMAX;
  if (fits)
    for (int e = tid; e < w * k; e += NT_TR) Ps[e] = P[(e % w) + (e / w) * WMAX];
  for (int r0 = 0; r0 < J.side[1].m; r0 += 64) {
    const int rows = min(64, J.side[1].m - r0);
    for (int e = tid; e < rows * w; e += NT_TR) {
      const int r = e % rows, cc = e / rows;
      const int64_t gr = r0 + r;
      In[r + cc * 64] = (cc < n0) ? s0.scale * s0.p[gr + (int64_t)cc * s0.ld]
                                  : s1.scale * s1.p[gr + (int64_t)(cc - n0) * s1.ld];
    }
    __syncthreads();
    if (fits)
      rows_times_small<NT_TR>(In, 64, rows, w, Ps, w, k, J.out[1] + r0, J.ldout[1]);
    else
      rows_times_small<NT_TR>(In, 64, rows, w, P, WMAX, k, J.out[1] + r0, J.ldout[1]);
    __syncthreads();
  }
}

// Wider jobs: the chunk code of k_tr_qr, one block per chunk (the chunks
// and sides join through the job's counters); the block that ran the SVD
// then forms both factors.
template <int WTOP>
__device__ __forceinline__ void tr_small_wide(const TrJob& J, int side, int chunk, int w, int n0a, int n0b,
                                              double* ws, int* counters, double* smem) {
  const int t = tier_of(w);
  bool last = false;
  if (t == 16) {
    if constexpr (WTOP >= 16) last = tr_chunk<16>(J, side, chunk, ws, counters, J.err, J.flops, smem, w, n0a, n0b);
  } else if (t == 32) {
    if constexpr (WTOP >= 32) last = tr_chunk<32>(J, side, chunk, ws, counters, J.err, J.flops, smem, w, n0a, n0b);
  } else if (t == 64) {
    if constexpr (WTOP >= 64) last = tr_chunk<64>(J, side, chunk, ws, counters, J.err, J.flops, smem, w, n0a, n0b);
  } else {
    if constexpr (WTOP >= 128)
      last = tr_chunk<128>(J, side, chunk, ws, counters, J.err, J.flops, smem, w, n0a, n0b);
  }
  if (!last) return;
  __threadfence_block();
  __syncthreads();
  tr_small_form(J, ws, smem);
}

// One block per chunk of each side (the items of k_tr_qr).  Width <= 8: the
// block of side 0, chunk 0 does the whole job and the others return.  The
// host sends a job here only when each side has at most TRS_MAXCH chunks and
// at most CH / WTOP of them (so that a wide job's tree has one combine level).
template <int WTOP>
__global__ void __launch_bounds__(NT_TR) k_tr_small(const TrJob* __restrict__ jobs,
                                                     const TrChunk* __restrict__ items, int first,
                                                     double* ws, int* counters) {
  extern __shared__ double smem[];
  const TrChunk it = items[first + blockIdx.x];
  const TrJob& J = jobs[it.job];
  const int n0a = seg_n(J.seg[0][0]);
  const int w = n0a + seg_n(J.seg[0][1]);
  const int n0b = seg_n(J.seg[1][0]);
  const bool lead = it.side == 0 && it.chunk == 0;
  if (w == 0 || w > WTOP) {
    if (lead && threadIdx.x == 0) {
      *J.out_rank = 0;
      if (w > WTOP) atomicOr(J.err, ERR_WIDTH);
    }
    return;
  }
  if (w <= 8) {
    if (!lead) return;
    if (max(J.side[0].m, J.side[1].m) > TRS_MAXCH * CH) {  // not sent here by the host
      if (threadIdx.x == 0) atomicOr(J.err, ERR_WIDTH);
      return;
    }
    if (w <= 4)
      tr_small_narrow<4>(J, w, n0a, n0b, smem);
    else
      tr_small_narrow<8>(J, w, n0a, n0b, smem);
    return;
  }
  tr_small_wide<WTOP>(J, it.side, it.chunk, w, n0a, n0b, ws, counters, smem);
}

// ------------------------------------------------------------------ HODLR x tall-skinny
__device__ __forceinline__ int mm_s(const MmJob& J) { return J.s_dev ? *J.s_dev : J.s; }

// Phase A: projections P_b = F_b^T X (F = V for op N, U for op T) of every
// block of the sub-HODLR, MM_CH rows per block of threads.  Thread t takes
// output e = t % nout (nout = k s) and every Q-th row of the chunk
// (Q = NT_MM / nout groups), so all loads of a block are in flight together;
// the Q partial sums are added in a fixed order.  A block of one chunk writes
// its projection directly, longer blocks write per-chunk partials that
// k_mm_red sums (a separate launch: no cross-block fences).
__global__ void __launch_bounds__(NT_MM) k_mm_proj(const MmJob* __restrict__ jobs,
                                                    const MmProj* __restrict__ items, int first,
                                                    double* ws) {
  __shared__ double part_s[NT_MM];
  const int tid = threadIdx.x;
  const MmProj it = items[first + blockIdx.x];
  const MmJob& J = jobs[it.job];
  const int s = mm_s(J);
  const HBlk b = (it.kind == 0 ? J.M.up : J.M.lo)[it.node];
  const int k = *b.rank;
  if (k == 0 || s == 0) return;
  const int trans = J.trans;
  const int len = trans ? b.rows : b.cols;
  const double* F = trans ? b.U : b.V;
  const int ldF = trans ? b.ldU : b.ldV;
  const double* X = J.X + ((trans ? b.r0 : b.c0) - J.row0);
  const int ldX = J.ldX;
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
      dst[(tid % k) + (tid / k) * KCAP] = sacc;
    }
  } else {
    for (int e = tid; e < nout; e += NT_MM) {
      const int j = e % k, c = e / k;
      const double* f = F + c0 + (int64_t)j * ldF;
      const double* x = X + c0 + (int64_t)c * ldX;
      double acc = 0.0;
      for (int r = 0; r < cn; ++r) acc += f[r] * x[r];
      dst[j + c * KCAP] = acc;
    }
  }
  if (tid == 0) add_flops(J.flops, FC_HMAT, 2.0 * k * cn * s);
}

// Sum the per-chunk partials of one block projection (chunk order fixed).
__global__ void __launch_bounds__(NT_MM) k_mm_red(const MmJob* __restrict__ jobs,
                                                   const MmProj* __restrict__ items, int first,
                                                   double* ws) {
  const MmProj it = items[first + blockIdx.x];
  const MmJob& J = jobs[it.job];
  const int s = mm_s(J);
  const HBlk b = (it.kind == 0 ? J.M.up : J.M.lo)[it.node];
  const int k = *b.rank;
  const double* part0 = ws + it.part;
  double* red = ws + J.red0 + (int64_t)(2 * rel_node(it.node, J.v) + it.kind) * (KCAP * SMAX);
  for (int e = threadIdx.x; e < k * s; e += NT_MM) {
    const int off = (e % k) + (e / k) * KCAP;
    double acc = 0.0;
    for (int ch = 0; ch < it.nchunk; ++ch) acc += part0[(int64_t)ch * (KCAP * SMAX) + off];
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
constexpr int MA_LD = 17;
constexpr int DT_LD = 65;  // transposed leaf tile, padded row

__host__ __device__ constexpr size_t mm_apply_lds(int mleaf) {
  return sizeof(double) * (size_t)MA_LD * (size_t)(mleaf > 256 ? mleaf : 256);
}

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
                                              double* shm, double* Dt, int s) {
  constexpr int G = NT_MM / RT;
  constexpr int DMAX = RT == 16 ? MAXLEAF / G : 1;
  const int tid = threadIdx.x;
  const int r = tid % RT, g = tid / RT;
  const HLeaf lf = J.M.leaf[it.leaf];
  const int kind = J.M.leaf_kind;
  const int trans = J.trans;
  const int m = lf.m;
  const int R = it.row0 + r;  // row of this thread within the leaf
  const bool live = r < it.rows;
  double dv[DMAX];
  if constexpr (RT == 16) {
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
          aF[a] = (trans ? b.V : b.U) + (lf.r0 + R - (trans ? b.c0 : b.r0));
          aR[a] = ws + J.red0 + (int64_t)(2 * rel_node(u, J.v) + bk) * (KCAP * SMAX);
        }
      }
    }
  }
  const double* xl = J.X + (lf.r0 - J.row0);
  double* Xs = shm;
  for (int c0 = 0; c0 < s; c0 += CW) {
    const int cn = min(CW, s - c0);
    for (int e = tid; e < m * CW; e += NT_MM) {
      const int kk = e % m, c = e / m;
      Xs[kk * MA_LD + c] = (c < cn) ? xl[kk + (int64_t)(c0 + c) * J.ldX] : 0.0;
    }
    __syncthreads();
    double acc[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) acc[c] = 0.0;
    if constexpr (RT == 16) {
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
        const double* red = aR[a] + (int64_t)c0 * KCAP;
        for (int j = 0; j < akb[a]; ++j) {
          const double fv = live ? aF[a][(int64_t)j * ald[a]] : 0.0;
#pragma unroll
          for (int c = 0; c < CW; ++c)
            if (c < cn) acc[c] += fv * red[j + c * KCAP];
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
          const double* red = ws + J.red0 + (int64_t)(2 * rel_node(u, J.v) + bk) * (KCAP * SMAX) +
                              (int64_t)c0 * KCAP;
          const double* F = trans ? b.V : b.U;
          const int ldF = trans ? b.ldV : b.ldU;
          const int64_t frow = lf.r0 + R - (trans ? b.c0 : b.r0);
          for (int j = 0; j < kb; ++j) {
            const double fv = live ? F[frow + (int64_t)j * ldF] : 0.0;
#pragma unroll
            for (int c = 0; c < CW; ++c)
              if (c < cn) acc[c] += fv * red[j + c * KCAP];
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
        double* zp = J.Z + (lf.r0 - J.row0 + it.row0 + rr) + (int64_t)(c0 + c) * J.ldZ;
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
                                                     const double* __restrict__ ws) {
  extern __shared__ double shm[];
  double* Dt = nullptr;  // transposed leaf tile (RT = 64 only)
  if constexpr (RT == 64) {
    __shared__ double dtile[64 * DT_LD];
    Dt = dtile;
  }
  const MmApply it = items[first + blockIdx.x];
  const MmJob& J = jobs[it.job];
  const int s = mm_s(J);
  if (s == 0) return;
  if (s <= 4)
    mm_apply_rows<RT, 4>(J, it, ws, shm, Dt, s);
  else
    mm_apply_rows<RT, 16>(J, it, ws, shm, Dt, s);
  if (threadIdx.x == 0) {
    const HLeaf lf = J.M.leaf[it.leaf];
    const int trans = J.trans;
    const int hleaf = (1 << J.M.levels) + it.leaf;
    double flops = 2.0 * it.rows * lf.m * s * (J.tri ? 0.5 : 1.0);
    int child2 = hleaf, u2 = hleaf >> 1;
    while (child2 != J.v && u2 >= 1) {
      const bool left = (child2 == 2 * u2);
      const int bk = trans ? (left ? 1 : 0) : (left ? 0 : 1);
      const HBlk* arr = bk == 0 ? J.M.up : J.M.lo;
      if (arr != nullptr) flops += 2.0 * it.rows * (*arr[u2].rank) * s;
      child2 = u2;
      u2 >>= 1;
    }
    add_flops(J.flops, FC_HMAT, flops);
  }
}

// ------------------------------------------------------------------ small GEMMs
__device__ __forceinline__ double gA(const GemmJob& J, int r, int kk) {
  return J.ta ? J.A[kk + (int64_t)r * J.lda] : J.A[r + (int64_t)kk * J.lda];
}
__device__ __forceinline__ double gB(const GemmJob& J, int kk, int c) {
  return J.tb ? J.B[c + (int64_t)kk * J.ldb] : J.B[kk + (int64_t)c * J.ldb];
}

__global__ void __launch_bounds__(NT_MM) k_gemm_tall(const GemmJob* __restrict__ jobs,
                                                      const GemmTile* __restrict__ items, int first) {
  __shared__ double At[64][33];
  __shared__ double Bt[32][65];
  const int tid = threadIdx.x;
  const GemmTile it = items[first + blockIdx.x];
  const GemmJob J = jobs[it.job];
  const int M = J.Md ? *J.Md : J.M, N = J.Nd ? *J.Nd : J.N, K = J.Kd ? *J.Kd : J.K;
  if (it.row0 >= M || it.col0 >= N) return;
  const int mr = min(64, M - it.row0), nc = min(64, N - it.col0);
  const int r = tid & 63, cg = tid >> 6;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
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
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int cc = cg + 4 * q;
      if (cc < nc) {  // uniform in the wavefront (cg is its index): skips empty columns
        double sacc = acc[q];
#pragma unroll 8
        for (int kk = 0; kk < 32; ++kk) sacc += At[r][kk] * Bt[kk][cc];
        acc[q] = sacc;
      }
    }
    __syncthreads();
  }
  if (r < mr) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int cc = cg + 4 * q;
      if (cc < nc) {
        double* cp = J.C + (int64_t)(it.row0 + r) + (int64_t)(it.col0 + cc) * J.ldc;
        const double v = J.alpha * acc[q];
        *cp = (J.beta == 0.0) ? v : v + J.beta * (*cp);
      }
    }
  }
  if (tid == 0) add_flops(J.flops, J.fc, 2.0 * mr * nc * K);
}

// C (M x N, both <= KCAP) from a long K, split into chunks; the last chunk sums.
__global__ void __launch_bounds__(NT_MM) k_gemm_red(const GemmJob* __restrict__ jobs,
                                                     const GemmRed* __restrict__ items, int first,
                                                     double* ws, int* counters) {
  __shared__ double At[32][KCAP + 1];
  __shared__ double Bt[32][KCAP + 1];
  __shared__ int lastf;
  const int tid = threadIdx.x;
  const GemmRed it = items[first + blockIdx.x];
  const GemmJob J = jobs[it.job];
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
  int M = J.m;
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
  const int m = J.m;
  double* h = W.H + (int64_t)c * MAXSTACK;
  for (int r = threadIdx.x; r < m; r += NT_MM) h[r] = J.D[r + (int64_t)c * m];
  int off = m;
  for (int g = 0; g < J.ngroups; ++g) {
    const int k = *J.g[g].rank;
    const double* V = J.g[g].V + J.g[g].row0 + c;
    const int ld = J.g[g].ld;
    for (int t = threadIdx.x; t < k; t += NT_MM) h[off + t] = V[(int64_t)t * ld];
    off += k;
  }
}

// LDS layout of the leaf kernels (doubles)
constexpr int LF_VBUF = 0;                       // 2 x MAXSTACK reflector broadcast
constexpr int LF_TAU = 2 * MAXSTACK;             // NB
constexpr int LF_GRAM = LF_TAU + NB;             // NB x NB
constexpr int LF_TP = LF_GRAM + NB * NB;         // NB x NB
constexpr int LF_CH = 320;                       // rows per staged strip chunk
constexpr int LF_LD = LF_CH + 4;                 // leading dimension of staged strips
constexpr int LF_A = LF_TP + NB * NB;            // staged Y_p and strip: 2 x LF_LD x NB
constexpr int LF_PART = LF_A + 2 * LF_LD * NB;   // 16 wave partial tiles (16 x 256)
constexpr int LF_W = LF_PART + 16 * NB * NB;     // 3 tiles of NB x NB
constexpr int LF_TOTAL = LF_W + 3 * NB * NB;
constexpr size_t LEAF_LDS = sizeof(double) * (size_t)LF_TOTAL;

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

// Sum the 16 wavefronts' 16 x 16 tiles into out (ld NB).
__device__ __forceinline__ void leaf_reduce_tile(d4_t acc, double* part, double* out) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = 4 * e + (l >> 4), j = l & 15;
    part[w * 256 + i + NB * j] = acc[e];
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    double sacc = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) sacc += part[q * 256 + threadIdx.x];
    out[threadIdx.x] = sacc;
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
    }
    __syncthreads();
    if (w > j && w < pw) {
      const double tau = taus[j];
      if (tau != 0.0) {
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
      }
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
  double tval = 0.0;  // T_pp tile, loaded together with the first staging
  if (tid < 256) {
    const int i = tid & 15, j = tid >> 4;
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
  leaf_reduce_tile(acc, sm + LF_PART, Wt);
  // W2 = T^T W: A[i][k] = T[k][i], B[k][j] = W[k][j]; D[i][j] sits in lane
  // j + 16 (i % 4), element i / 4, i.e. element e of lane l is W2[4e + l/16][l%16]:
  // the B operand of k-step e of the update below
  d4_t w2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < NB; k0 += 4)
    w2 = mfma16(Tt[(k0 + (l >> 4)) + NB * (l & 15)], Wt[(k0 + (l >> 4)) + NB * (l & 15)], w2);
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
    const double g = gmem(W.G)[(int64_t)(i0 + 4 * ks + (l >> 4)) + (int64_t)(cq + (l & 15)) * MAXLEAF];
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
  const int m = J.m;
  const double* h = W.H + (int64_t)c * MAXSTACK;
  for (int r = threadIdx.x; r < m; r += NT_MM) {
    J.D[r + (int64_t)c * m] = h[r];
    J.Tleaf[r + (int64_t)c * m] = (r <= c) ? W.T[r + (int64_t)c * MAXLEAF] : 0.0;
  }
  int off = m;
  for (int g = 0; g < J.ngroups; ++g) {
    const int k = *J.g[g].rank;
    double* V = J.g[g].V + J.g[g].row0 + c;
    const int ld = J.g[g].ld;
    for (int t = threadIdx.x; t < k; t += NT_MM) V[(int64_t)t * ld] = h[off + t];
    off += k;
  }
}

// ------------------------------------------------------------------ vectors
// x <- z / |z|, out[0] = |z|  (one block per item; x or out may be null)
__global__ void __launch_bounds__(1024) k_normalize(const VecJob* __restrict__ items, int first) {
  __shared__ double red[16];
  const VecJob it = items[first + blockIdx.x];
  const double* z = it.z;
  const int64_t n = it.n;
  // sixteen loads in flight per thread (a plain loop waits for every load)
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 15 * 1024 < n; i += 16 * 1024) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = z[i + u * 1024];
#pragma unroll
    for (int u = 0; u < 16; u += 4) {
      s0 += v[u] * v[u];
      s1 += v[u + 1] * v[u + 1];
      s2 += v[u + 2] * v[u + 2];
      s3 += v[u + 3] * v[u + 3];
    }
  }
  for (; i < n; i += 1024) s0 += z[i] * z[i];
  double s = (s0 + s1) + (s2 + s3);
  s = gsum(s, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < 16; ++i) t += red[i];
  const double nrm = sqrt(t);
  if (it.x != nullptr) {
    const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
    int64_t j = threadIdx.x;
    for (; j + 15 * 1024 < n; j += 16 * 1024) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = z[j + u * 1024];
#pragma unroll
      for (int u = 0; u < 16; ++u) it.x[j + u * 1024] = v[u] * inv;
    }
    for (; j < n; j += 1024) it.x[j] = z[j] * inv;
  }
  if (threadIdx.x == 0 && it.out != nullptr) it.out[0] = nrm;
}

// thresholds of one factorisation: x = [|A|_2, eps*|A|_2, eps] with eps = d0 and
// |A|_2 = d1 if d1 > 0, else the estimate already in x[0]  (one thread per item)
__global__ void k_set_scal(const VecJob* __restrict__ items, int first, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const VecJob it = items[first + i];
  const double a = it.d1 > 0.0 ? it.d1 : it.x[0];
  it.x[0] = a;
  it.x[1] = it.d0 * a;
  it.x[2] = it.d0;
}

// x[0:n] = d0, one block per item
__global__ void k_fill_items(const VecJob* __restrict__ items, int first) {
  const VecJob it = items[first + blockIdx.x];
  for (int64_t i = threadIdx.x; i < it.n; i += blockDim.x) it.x[i] = it.d0;
}

__global__ void k_fill(double* x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// Back substitution with one upper triangular leaf: X <- R^{-1} X (m x nrhs).
__global__ void __launch_bounds__(NT_MM) k_leaf_trsm(const double* __restrict__ D, int m, int ld,
                                                      double* X, int ldx, int nrhs) {
  __shared__ double xs[MAXLEAF];
  __shared__ double red[4];
  const int c = blockIdx.x;  // one column per block
  if (c >= nrhs) return;
  double* x = X + (int64_t)c * ldx;
  for (int r = threadIdx.x; r < m; r += NT_MM) xs[r] = x[r];
  __syncthreads();
  for (int i = m - 1; i >= 0; --i) {
    double s = 0.0;
    for (int j = i + 1 + threadIdx.x; j < m; j += NT_MM) s += D[i + (int64_t)j * ld] * xs[j];
    s = gsum(s, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) xs[i] = (xs[i] - (red[0] + red[1] + red[2] + red[3])) / D[i + (int64_t)i * ld];
    __syncthreads();
  }
  for (int r = threadIdx.x; r < m; r += NT_MM) x[r] = xs[r];
}

}  // namespace hq

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
// ds_bpermute round trips.  CTRL is a gfx9 DPP control word whose source lane
// lies in the same row for every lane (quad permutes, row mirrors): with all
// rows and banks enabled every lane takes the moved value, so no old value has
// to be set up (bound_ctrl), which saves two moves per step.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xF, 0xF, true);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi2, lo2);
}

// x[l] + x[l ^ 16] (ROWS = 16) or x[l] + x[l ^ 32] (ROWS = 32) in every lane l,
// from the gfx950 permlane swaps: with both operands equal to x, the two
// results hold x of the even and of the odd row group of each pair, so their
// sum is the same (commutative) addition on every lane of the pair.
template <int ROWS>
__device__ __forceinline__ double swap_add(double x) {
  const unsigned lo = __double2loint(x), hi = __double2hiint(x);
  if constexpr (ROWS == 16) {
    const auto l2 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h2 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return __hiloint2double(h2[0], l2[0]) + __hiloint2double(h2[1], l2[1]);
  } else {
    const auto l2 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h2 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double(h2[0], l2[0]) + __hiloint2double(h2[1], l2[1]);
  }
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
  // rows of 16 lanes: (r0 + r1) and (r2 + r3), then their sum, on VALU only
  if constexpr (W >= 32) x = swap_add<16>(x);
  if constexpr (W >= 64) x = swap_add<32>(x);
  return x;
}

// 1/x, 1/sqrt(x) and sqrt(x) from the hardware estimates (relative error about
// 2^-24 on gfx950) with one correction by the series of the residual
// e = 1 - x r (resp. 1 - x y^2) up to its second-order term:
//   1/x = r (1 + e + e^2 + ...),  1/sqrt(x) = y (1 + e/2 + 3e^2/8 + ...),
// so the truncation error is of order e^3 (about 2^-72) and the result is off
// by rounding only (an ulp or two), with a dependency chain of three or four
// operations after the estimate instead of two Newton steps.
__device__ __forceinline__ double rcp_nr(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

__device__ __forceinline__ double rsq_nr(double x) {  // x > 0
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

__device__ __forceinline__ double sqrt_nr(double x) {  // x > 0: x y (1 + e/2 + 3e^2/8)
  const double y = __builtin_amdgcn_rsq(x);
  const double t = x * y;
  const double e = fma(-t, y, 1.0);
  return fma(t * e, fma(e, 0.375, 0.5), t);
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

}  // namespace hq

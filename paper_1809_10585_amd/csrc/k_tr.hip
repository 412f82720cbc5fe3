// Recompression T_tau of Sec. 2.1.1 (k_tr_qr, k_tr_form, k_tr_small).
#include "kernels_common.h"
#include "kernels.h"

namespace hq {

// ------------------------------------------------------------------ recompression
// The kept rank k of a job (and, when the job carries a log entry, its input
// width w next to k).
__device__ __forceinline__ void tr_set_rank(const TrJob& J, int w, int k) {
  *J.out_rank = k;
  if (J.log != nullptr) {
    J.log[0] = w;
    J.log[1] = k;
  }
}

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
  const double r = sqrt_nr(h2);
  const double s = r + fabs(d);
  const double q = rsq_nr(2.0 * r * s);
  cs = s * q;
  sn = (d >= 0.0 ? g : -g) * q;
  return true;
}

// The rotation of jac_rot_fast without the power-of-two scaling of (d, g),
// computed whether or not the pair needs one (no branch), for columns scaled
// so that the squared Frobenius norm of the whole matrix is below 1 and the
// squared norm of every rotated pair above 1e-40 (the caller's eta2): then
// d^2 + g^2 neither overflows nor underflows whenever a rotation is due
// (|g|^2 > tol2 a b with max(a, b) > 1e-40).  Same formula, three dependent
// operations shorter.
__device__ __forceinline__ void jac_rot_unit(double al, double be, double ga, double& cs, double& sn) {
  const double d = be - al, g = 2.0 * ga;
  const double h2 = fma(d, d, g * g);
  const double r = sqrt_nr(h2);
  const double s = r + fabs(d);
  const double q = rsq_nr((2.0 * r) * s);
  cs = s * q;
  sn = (d >= 0.0 ? g : -g) * q;
}

// One-sided Jacobi on the columns of X (w x w, ld lx), accumulating the
// rotations in V (ld lv) unless V is null.  Round-robin pairing; one pair per
// group of TPP lanes; a sweep ends when no pair needed a rotation.  Pairs of two
// columns whose squared norms are both <= eta2 are left alone (columns at the
// roundoff level of the matrix, which the caller discards).
__device__ __forceinline__ void jacobi(double* X, int lx, double* V, int lv, int w, int* sflag,
                                       double eta2 = 0.0) {
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
        if (valid && (al > eta2 || be > eta2) && jac_rot_fast(al, be, ga, tol * tol, cs, sn)) {
          for (int row = sub; row < w; row += TPP) {
            const double xi = X[row + i * lx], xj = X[row + j * lx];
            X[row + i * lx] = cs * xi - sn * xj;
            X[row + j * lx] = sn * xi + cs * xj;
          }
          if (V != nullptr) {
            for (int row = sub; row < w; row += TPP) {
              const double vi = V[row + i * lv], vj = V[row + j * lv];
              V[row + i * lv] = cs * vi - sn * vj;
              V[row + j * lv] = sn * vi + cs * vj;
            }
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

// jacobi() without V and without branches in its rounds, for 16 < w <= 128.
// X holds n = w + (w & 1) columns of TPP * RPL >= w rows (ld lx >= TPP * RPL),
// zero beyond row w and in column w when w is odd (rotations keep them zero,
// so every lane loads and stores its rows unconditionally).  Pair p of a round
// is taken by TPP lanes, each holding RPL rows of both columns in registers
// between the dot products and the rotation; a pair that needs no rotation is
// stored back unchanged (cs = 1, sn = 0).  X is scaled as jac_rot_unit
// requires, and eta2 >= 1e-40.
template <int TPP, int RPL>
__device__ __forceinline__ void jacobi_pad(double* X, int lx, int w, int* sflag, double eta2) {
  const int tid = threadIdx.x;
  const int n = w + (w & 1), nm1 = n - 1;
  const int P = n / 2;
  const int p = tid / TPP, sub = tid % TPP;
  const double tol = (double)w * DBL_EPSILON;
  const double tol2 = tol * tol;
  constexpr int NA = RPL >= 8 ? 4 : (RPL >= 4 ? 2 : 1);
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) *sflag = 0;
    __syncthreads();
    for (int r = 0; r < nm1; ++r) {
      if (p < P) {
        int i = r + p;
        i = i >= nm1 ? i - nm1 : i;
        int j = r - p;
        j = j < 0 ? j + nm1 : j;
        j = p == 0 ? nm1 : j;
        double* ci = X + min(i, j) * lx + sub;
        double* cj = X + max(i, j) * lx + sub;
        double xi[RPL], xj[RPL];
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          xi[t] = ci[t * TPP];
          xj[t] = cj[t * TPP];
        }
        double pa[NA], pb[NA], pg[NA];
#pragma unroll
        for (int q = 0; q < NA; ++q) pa[q] = pb[q] = pg[q] = 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          pa[t % NA] += xi[t] * xi[t];
          pb[t % NA] += xj[t] * xj[t];
          pg[t % NA] += xi[t] * xj[t];
        }
#pragma unroll
        for (int h = NA / 2; h >= 1; h /= 2)
#pragma unroll
          for (int q = 0; q < h; ++q) {
            pa[q] += pa[q + h];
            pb[q] += pb[q + h];
            pg[q] += pg[q + h];
          }
        const double al = gsumt<TPP>(pa[0]);
        const double be = gsumt<TPP>(pb[0]);
        const double ga = gsumt<TPP>(pg[0]);
        const bool rot = (al > eta2 || be > eta2) && ga != 0.0 && ga * ga > tol2 * (al * be);
        double cr, sr;
        jac_rot_unit(al, be, ga, cr, sr);
        const double cs = rot ? cr : 1.0, sn = rot ? sr : 0.0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
          ci[t * TPP] = cs * xi[t] - sn * xj[t];
          cj[t * TPP] = sn * xi[t] + cs * xj[t];
        }
        if (rot && sub == 0) *sflag = 1;
      }
      __syncthreads();
    }
    const int f = *sflag;
    __syncthreads();
    if (f == 0) break;
  }
}

// Lanes per pair and rows per lane of jacobi_pad for a width 16 < w <= 128.
__device__ __forceinline__ void jacobi_pad_shape(int w, int& tpp, int& rpl) {
  if (w <= 32) {
    tpp = 32;
    rpl = 1;
  } else if (w <= 64) {
    tpp = 16;
    rpl = w <= 48 ? 3 : 4;
  } else {
    tpp = 8;
    rpl = w <= 80 ? 10 : (w <= 96 ? 12 : (w <= 112 ? 14 : 16));
  }
}

__device__ __forceinline__ void jacobi_noacc(double* X, int lx, int w, int* sflag, double eta2) {
  if (w <= 32)
    jacobi_pad<32, 1>(X, lx, w, sflag, eta2);
  else if (w <= 48)
    jacobi_pad<16, 3>(X, lx, w, sflag, eta2);
  else if (w <= 64)
    jacobi_pad<16, 4>(X, lx, w, sflag, eta2);
  else if (w <= 80)
    jacobi_pad<8, 10>(X, lx, w, sflag, eta2);
  else if (w <= 96)
    jacobi_pad<8, 12>(X, lx, w, sflag, eta2);
  else if (w <= 112)
    jacobi_pad<8, 14>(X, lx, w, sflag, eta2);
  else
    jacobi_pad<8, 16>(X, lx, w, sflag, eta2);
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

// Householder QR of X (w x w in LDS, ld w) by the whole block, in place: R in
// the upper triangle on return (the reflectors below it are not kept).  Column
// j's reflector is formed by wavefront 0; the later columns take it TPC
// threads each.  tau_slot: one double of LDS.
__device__ __forceinline__ void block_qr_r(double* X, int w, int lx, double* tau_slot) {
  const int tid = threadIdx.x;
  for (int j = 0; j < w - 1; ++j) {
    if (tid < 64) {
      double ss = 0.0;
      for (int r = j + 1 + tid; r < w; r += 64) {
        const double x = X[r + j * lx];
        ss += x * x;
      }
      ss = gsumt<64>(ss);
      double beta, tau, sc;
      house_scalars(X[j + j * lx], ss, beta, tau, sc);
      if (tau != 0.0)
        for (int r = j + 1 + tid; r < w; r += 64) X[r + j * lx] *= sc;
      if (tid == 0) {
        X[j + j * lx] = beta;
        *tau_slot = tau;
      }
    }
    __syncthreads();
    const double tau = *tau_slot;
    const int nc = w - 1 - j;  // columns j+1 .. w-1
    if (tau != 0.0) {
      int Pp = 1;
      while (Pp < nc) Pp <<= 1;
      int TPC = NT_TR / Pp;
      if (TPC > 64) TPC = 64;
      if (TPC < 1) TPC = 1;
      const int ci = tid / TPC, sub = tid % TPC;
      const bool live = ci < nc;
      const int c = j + 1 + ci;
      double d = 0.0;
      if (live) {
        if (sub == 0) d = X[j + c * lx];
        for (int r = j + 1 + sub; r < w; r += TPC) d += X[r + j * lx] * X[r + c * lx];
      }
      d = gsum(d, TPC);
      if (live) {
        const double f = tau * d;
        if (sub == 0) X[j + c * lx] -= f;
        for (int r = j + 1 + sub; r < w; r += TPC) X[r + c * lx] -= f * X[r + j * lx];
      }
    }
    __syncthreads();
  }
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
    double* sig = smem + TRS_X + TRS_XSZ;
    int* perm = (int*)(sig + WMAX);
    double* X = smem + TRS_X;
    const double* R1s = R1;
    int lr = WMAX;
    if (w <= 16) {
      // X = R2 R1^T and V padded to WS x WS (zeros beyond w) for jacobi_small;
      // the right singular vectors of X (accumulated in V) are U of R1 R2^T
      const int LX = w <= 8 ? 8 : 16;
      double* V = X + LX * LX;
      const double* R2s = R2;
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
      for (int e = tid; e < LX * LX; e += NT_TR) {
        const int i = e % LX, j = e / LX;
        double sacc = 0.0;
        if (i < w && j < w)
          for (int l = max(i, j); l < w; ++l) sacc += R2s[i + l * lr] * R1s[j + l * lr];
        X[i + j * LX] = sacc;
        V[i + j * LX] = (i == j && i < w) ? 1.0 : 0.0;
      }
      __syncthreads();
      if (LX == 8)
        jacobi_small<8>(X, w);
      else
        jacobi_small<16>(X, w);
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
        Uk[r + p * WMAX] = V[r + pc * LX];
        double sacc = 0.0;
        for (int l = 0; l <= r; ++l) sacc += R1s[l + r * lr] * V[l + pc * LX];
        P[r + p * WMAX] = sacc;
      }
    } else {
      // X = R2 R1^T = M^T (w x w), M = R1 R2^T.  When every column that can be
      // kept lies far above the roundoff level of M (tau^2 > 1e6 eta^2): the
      // Householder QR M^T = Q' R' first, then one-sided Jacobi on the columns
      // of R'^T without accumulating rotations: R'^T W = V' S with V' the right
      // singular vectors of R', which are those of M^T, i.e. U of M, so the
      // columns over their norms are U (orthonormal to the relative tolerance
      // once every kept pair has converged).  The triangular preconditioning
      // cuts the sweeps several-fold against Jacobi on M itself.  Otherwise
      // (tau at or near roundoff, e.g. tau = 0) the Jacobi runs on M^T and
      // accumulates the rotations V, whose columns are U and stay orthonormal
      // however far the roundoff columns converge.
      // X: nc = w + (w & 1) columns of the Jacobi's padded height, odd leading
      // dimension (LDS banks of the column pairs)
      int tpp, rpl;
      jacobi_pad_shape(w, tpp, rpl);
      const int lx = tpp * rpl + 1, nc = w + (w & 1);
      const double* R2s = R2;
      if (lx * nc + 2 * w * w <= TRS_XSZ) {
        double* r1 = X + lx * nc;
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
      for (int e = tid; e < w * w; e += NT_TR) {
        const int i = e % w, j = e / w;
        double sacc = 0.0;
        for (int l = max(i, j); l < w; ++l) sacc += R2s[i + l * lr] * R1s[j + l * lr];
        X[i + j * lx] = sacc;
      }
      __syncthreads();
      for (int cc = tid; cc < w; cc += NT_TR) {
        double sacc = 0.0;
        for (int r = 0; r < w; ++r) sacc += X[r + cc * lx] * X[r + cc * lx];
        sig[cc] = sacc;
      }
      __syncthreads();
      double fro2 = 0.0;
      for (int cc = 0; cc < w; ++cc) fro2 += sig[cc];
      const double eta2 = (double)w * DBL_EPSILON * DBL_EPSILON * fro2;
      const bool fast = 1e6 * eta2 < tau * tau;
      __syncthreads();
      double* V = nullptr;
      int LV = 0;
      int scl = 0;  // X = 2^scl (matrix whose column norms are the singular values)
      if (fast) {
        block_qr_r(X, w, lx, smem + TRS_TAU);
        // X <- 2^-e R'^T (lower triangular) with |X|_F^2 = 2^-2e fro2 in [1/4, 1):
        // the unit scale of jac_rot_unit (the rotations are those of the
        // unscaled matrix; only k's threshold is scaled the same way below)
        const int ex = __builtin_amdgcn_frexp_exp(sqrt(fro2));
        for (int e = tid; e < w * w; e += NT_TR) {
          const int i = e % w, j = e / w;
          if (i < j) {
            X[j + i * lx] = __builtin_ldexp(X[i + j * lx], -ex);
            X[i + j * lx] = 0.0;
          } else if (i == j) {
            X[i + i * lx] = __builtin_ldexp(X[i + i * lx], -ex);
          }
        }
        const int hp = lx - 1;  // zero padding: rows w.. of every column, column w
        for (int e = tid; e < hp * nc; e += NT_TR) {
          const int i = e % hp, j = e / hp;
          if (i >= w || j >= w) X[i + j * lx] = 0.0;
        }
        scl = -ex;
        __syncthreads();
        jacobi_noacc(X, lx, w, sflag, fmax(__builtin_ldexp(eta2, -2 * ex), 1e-40));
      } else {
        R1s = R1;  // V takes the staging space
        lr = WMAX;
        if (lx * nc + w * w <= TRS_XSZ) {
          V = X + lx * nc;
          LV = w;
        } else {
          V = hdr + 8 + 2 * WMAX * WMAX;
          LV = WMAX;
        }
        __syncthreads();
        for (int e = tid; e < w * w; e += NT_TR) {
          const int i = e % w, j = e / w;
          V[i + j * LV] = (i == j) ? 1.0 : 0.0;
        }
        __syncthreads();
        jacobi(X, lx, V, LV, w, sflag);
      }
      for (int cc = tid; cc < w; cc += NT_TR) {
        double sacc = 0.0;
        for (int r = 0; r < w; ++r) sacc += X[r + cc * lx] * X[r + cc * lx];
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
      const double tau_s = __builtin_ldexp(tau, scl);
      for (int j = 0; j < w; ++j) k += (sig[j] > tau_s) ? 1 : 0;
      if (k > capk) {
        if (tid == 0) atomicOr(err, ERR_CAPACITY);
        k = capk;
      }
      for (int e = tid; e < w * k; e += NT_TR) {
        const int r = e % w, p = e / w;
        const int pc = perm[p];
        const double* u = fast ? X + (int64_t)pc * lx : V + (int64_t)pc * LV;
        const double inv = fast ? 1.0 / sig[pc] : 1.0;
        Uk[r + p * WMAX] = u[r] * inv;
        double sacc = 0.0;
        for (int l = 0; l <= r; ++l) sacc += R1s[l + r * lr] * u[l];
        P[r + p * WMAX] = sacc * inv;
      }
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

// Returns true in the block that ran the SVD (the job's last block).  LOCAL:
// every chunk of the job runs in this block (one after another), so the
// hand-offs between chunks need only block-scope fences.
template <int W, bool LOCAL>
__device__ __forceinline__ bool tr_chunk2p(const TrJob& J, int side, int chunk, double* ws, int* counters, int* err,
                                           double* fc, double* smem, int w, int n0a, int n0b);

template <int W, bool LOCAL = false>
__device__ __forceinline__ bool tr_chunk(const TrJob& J, int side, int chunk, double* ws, int* counters, int* err,
                         double* fc, double* smem, int w, int n0a, int n0b) {
  if constexpr (W >= 64) return tr_chunk2p<W, LOCAL>(J, side, chunk, ws, counters, err, fc, smem, w, n0a, n0b);
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
    if constexpr (LOCAL) __threadfence_block(); else __threadfence();
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
    if constexpr (LOCAL) __threadfence_block(); else __threadfence();
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
    if constexpr (LOCAL) __threadfence_block(); else __threadfence();
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
    if constexpr (LOCAL) __threadfence_block(); else __threadfence();
  }
  tr_svd<W>(J, ws, w, n0a, n0b, smem, err, fc);
  return true;
}

// ---- the 64- and 128-column tiers: a tile of h <= 256 rows and PW < w <= 2 PW
// columns (PW = W / 2) as two panels of PW columns, each in the register layout
// of the PW-column tier (thread (c, sub) = (tid / TPC, tid % TPC), TPC =
// NT_TR / PW, holds rows sub + TPC i, i < CH / TPC, of panel column c).  One
// 256 x W tile in registers holds twice the rows per thread, and at W = 128 it
// did not fit beside the rest of the kernel (spilled to scratch: about six
// times the time per column of the 64-column tier); and a panel keeps every
// thread busy on its columns instead of idling the threads of the finished
// ones.  Panel A (columns 0..PW-1) is factorised; its reflectors go to LDS and
// are applied, one after another, to panel B (columns PW..w-1), whose rows
// PW.. are then factorised: the Householder QR of the whole tile, column by
// column.  R goes to node (ld WMAX); with wantq, the explicit Q (h x w, ld CH)
// to Qa, formed as H_A (H_B [I; 0]) with the reflectors read back from Qa.
template <int PW, class LD>
__device__ __forceinline__ void qr2_tile(const LD& ld, int h, int w, bool wantq, double* node, double* Qa,
                                         double* smem) {
  constexpr int T2_TPC = NT_TR / PW, T2_RPT = CH / T2_TPC;
  const int tid = threadIdx.x, c = tid / T2_TPC, sub = tid % T2_TPC;
  double* vbuf = smem + TRS_VBUF;
  double* taus = smem + TRS_TAU;  // panel A: taus[0..PW-1], panel B: taus[PW..]
  double* Vs = smem + TRS_X;      // panel A's columns (ld CH), later Q's first PW columns
  const int wB = w - PW, hB = max(h - PW, 0);
  const bool liveB = c < wB;
  {
    double a[T2_RPT];
#pragma unroll
    for (int i = 0; i < T2_RPT; ++i) {
      const int r = sub + T2_TPC * i;
      a[i] = (r < h) ? ld(r, c) : 0.0;
    }
    reg_qr<T2_TPC, T2_RPT>(a, c, sub, h, PW, vbuf, taus, nullptr, 0);
#pragma unroll
    for (int i = 0; i < T2_RPT; ++i) {
      const int r = sub + T2_TPC * i;
      if (r < w) node[r + c * WMAX] = (r <= c && r < h) ? a[i] : 0.0;
      Vs[r + c * CH] = (r < h) ? a[i] : 0.0;
      if (wantq && r < h) Qa[r + c * CH] = a[i];
    }
  }
  __syncthreads();
  const int jA = min(h, PW);
  double b[T2_RPT];
#pragma unroll
  for (int i = 0; i < T2_RPT; ++i) {
    const int r = sub + T2_TPC * i;
    b[i] = (liveB && r < h) ? ld(r, PW + c) : 0.0;
  }
  if (liveB) {  // whole 8-lane groups: the sums stay inside the group
    for (int j = 0; j < jA; ++j) {
      const double tau = taus[j];
      if (tau == 0.0) continue;
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < T2_RPT; ++i) {
        const int r = sub + T2_TPC * i;
        const double v = r < j ? 0.0 : (r == j ? 1.0 : Vs[r + j * CH]);
        d += v * b[i];
      }
      const double f = tau * gsumt<T2_TPC>(d);
#pragma unroll
      for (int i = 0; i < T2_RPT; ++i) {
        const int r = sub + T2_TPC * i;
        const double v = r < j ? 0.0 : (r == j ? 1.0 : Vs[r + j * CH]);
        b[i] -= f * v;
      }
    }
  }
  // rows 0..PW-1 of panel B are R's; rows PW.. are factorised
  constexpr int RA = PW / T2_TPC;  // register rows of a thread above row PW
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    const int r = sub + T2_TPC * i;
    if (liveB) node[r + (PW + c) * WMAX] = (r < h) ? b[i] : 0.0;
  }
  constexpr int RB = T2_RPT - RA;
  double bb[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) bb[i] = b[RA + i];
  reg_qr<T2_TPC, RB>(bb, c, sub, hB, wB, vbuf, taus + PW, nullptr, 0);
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    const int r = sub + T2_TPC * i;  // row PW + r of the tile
    if (liveB && PW + r < w) node[(PW + r) + (PW + c) * WMAX] = (r <= c && r < hB) ? bb[i] : 0.0;
    if (wantq && liveB && r < hB) Qa[(PW + r) + (PW + c) * CH] = bb[i];
  }
  if (!wantq) return;
  __threadfence_block();
  __syncthreads();
  // Q's columns 0..PW-1: H_A [e_c] (panel B's reflectors act on rows >= PW only)
  {
    double q[T2_RPT];
    reg_formq_g<T2_TPC, T2_RPT>(Qa, q, c, sub, h, PW, vbuf, taus);
#pragma unroll
    for (int i = 0; i < T2_RPT; ++i) {
      const int r = sub + T2_TPC * i;
      Vs[r + c * CH] = q[i];
    }
  }
  // Q's columns PW..w-1: H_B [e_c] on rows PW.., then H_A on all rows
  double q2[T2_RPT];
  {
    double qb[RB];
    reg_formq_g<T2_TPC, RB>(Qa + PW + PW * (int64_t)CH, qb, c, sub, hB, wB, vbuf, taus + PW);
#pragma unroll
    for (int i = 0; i < T2_RPT; ++i) q2[i] = (i < RA) ? 0.0 : qb[i - RA];
  }
  for (int j = jA - 1; j >= 0; --j) {
    double* vb = vbuf + (j & 1) * CH;
    if (c == j) {
#pragma unroll
      for (int i = 0; i < T2_RPT; ++i) {
        const int r = sub + T2_TPC * i;
        vb[r] = r < j ? 0.0 : (r == j ? 1.0 : (r < h ? Qa[r + (int64_t)j * CH] : 0.0));
      }
    }
    __syncthreads();
    const double tau = taus[j];
    if (tau != 0.0 && liveB) {
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < T2_RPT; ++i) d += vb[sub + T2_TPC * i] * q2[i];
      const double f = tau * gsumt<T2_TPC>(d);
#pragma unroll
      for (int i = 0; i < T2_RPT; ++i) q2[i] -= f * vb[sub + T2_TPC * i];
    }
  }
  __syncthreads();  // every read of the reflectors in Qa is done
#pragma unroll
  for (int i = 0; i < T2_RPT; ++i) {
    const int r = sub + T2_TPC * i;
    if (r < h) {
      Qa[r + c * CH] = Vs[r + c * CH];
      if (liveB) Qa[r + (PW + c) * CH] = q2[i];
    }
  }
}

// tr_chunk for the 64- and 128-column tiers (the same tree, joins and SVD)
// with the tile factorised by qr2_tile.
template <int W, bool LOCAL>
__device__ __forceinline__ bool tr_chunk2p(const TrJob& J, int side, int chunk, double* ws, int* counters, int* err,
                                           double* fc, double* smem, int w, int n0a, int n0b) {
  constexpr int G = CH / W;
  const int tid = threadIdx.x;
  int* sflag = (int*)(smem + TRS_FLAG);
  const TrSide S = J.side[side];
  const int n0 = side == 0 ? n0a : n0b;
  const Seg s0 = J.seg[side][0], s1 = J.seg[side][1];
  int idx = chunk, count = S.p0;
  int64_t base = 0;  // first slot of the current level
  const int row0 = (int)((int64_t)idx * S.m / S.p0);
  int h = (int)((int64_t)(idx + 1) * S.m / S.p0) - row0;
  int64_t slot = idx;
  int64_t cbase = 0;
  int cfirst = 0;
  bool leaf = true;
  while (true) {
    double* node = ws + S.node0 + slot * TR_NODE;
    double* Qa = node + WMAX * WMAX;
    if (leaf) {
      auto ld = [&](int r, int col) -> double {
        const int64_t gr = row0 + r;
        return col < n0 ? s0.scale * s0.p[gr + (int64_t)col * s0.ld]
                        : s1.scale * s1.p[gr + (int64_t)(col - n0) * s1.ld];
      };
      qr2_tile<W / 2>(ld, h, w, side == 0, node, Qa, smem);
    } else {
      const double* kids = ws + S.node0 + (cbase + cfirst) * TR_NODE;
      auto ld = [&](int r, int col) -> double {
        const int ch = r / w, rr = r % w;
        return kids[(int64_t)ch * TR_NODE + rr + col * WMAX];
      };
      qr2_tile<W / 2>(ld, h, w, side == 0, node, Qa, smem);
    }
    if (count == 1) break;
    const int pidx = idx / G;
    const int pcount = (count + G - 1) / G;
    const int nchild = min(G, count - pidx * G);
    const int64_t pbase = base + count;
    const int64_t pslot = pbase + pidx;
    if constexpr (LOCAL) __threadfence_block(); else __threadfence();
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
    if constexpr (LOCAL) __threadfence_block(); else __threadfence();
    // become the parent: the children's R factors stacked
    cbase = base;
    cfirst = pidx * G;
    base = pbase;
    idx = pidx;
    count = pcount;
    slot = pslot;
    h = nchild * w;
    leaf = false;
  }
  // this side is reduced; join the two sides
  if (!(J.flags & TR_ORTH)) {
    if constexpr (LOCAL) __threadfence_block(); else __threadfence();
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
    if constexpr (LOCAL) __threadfence_block(); else __threadfence();
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


// out[r, p] = sum_c A(r, c) B[c + p*ldb] for r < rows, p < k <= 128 by NT
// threads: thread (tr, g) keeps the 4 x 8 outputs of rows tr + TR i (i < 4) and
// columns 8g + j (j < 8) in registers, TR = NT / (the number of 8-column groups
// rounded up to a power of two), so each A element it loads serves 8 products
// and each B element 4; row blocks of 4 TR rows.  A(r, c) = aload(r, c) for
// r < rows (rows and columns past the ends are clamped, computed and dropped).
// With sync, every thread has read its rows of a row block before any output
// of that block is stored (out may overwrite A in place, row by row).
template <int NT, class AL>
__device__ __forceinline__ void tile_times_small(const AL& aload, int rows, int w, const double* B, int ldb,
                                                 int k, double* out, int64_t ldo, bool sync) {
  const int tid = threadIdx.x;
  const int G = (k + 7) >> 3;
  int Gp = 1;
  while (Gp < G) Gp <<= 1;
  const int TR = NT / Gp;
  const int tr = tid % TR, g = tid / TR;
  const bool live = g < G;
  const int q0 = 8 * g;
  int qq[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) qq[j] = min(q0 + j, k - 1) * ldb;
  for (int rb = 0; rb < rows; rb += 4 * TR) {
    double acc[4][8];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[i][j] = 0.0;
    if (live) {
      int rr[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) rr[i] = min(rb + tr + TR * i, rows - 1);
#pragma unroll 4
      for (int c = 0; c < w; ++c) {
        double av[4], bv[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) av[i] = aload(rr[i], c);
#pragma unroll
        for (int j = 0; j < 8; ++j) bv[j] = B[c + qq[j]];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 8; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
      }
    }
    if (sync) __syncthreads();
    if (live) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = rb + tr + TR * i;
        if (r < rows)
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (q0 + j < k) out[r + (int64_t)(q0 + j) * ldo] = acc[i][j];
      }
    }
  }
}

// A(r, c) = a[r + c*lda]
struct ALoadPlain {
  const double* a;
  int64_t lda;
  __device__ __forceinline__ double operator()(int r, int c) const { return a[r + (int64_t)c * lda]; }
};

// A(r, c): the two scaled segments of a recompression side, side by side
struct ALoadSegs {
  Seg s0, s1;
  int n0;
  int64_t row0;
  __device__ __forceinline__ double operator()(int r, int c) const {
    const int64_t gr = row0 + r;
    return c < n0 ? s0.scale * s0.p[gr + (int64_t)c * s0.ld] : s1.scale * s1.p[gr + (int64_t)(c - n0) * s1.ld];
  }
};

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
  if (it.leader && tid == 0) tr_set_rank(J, w, k);
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
        tile_times_small<NT_MM>(ALoadPlain{Qn, CH}, w, w, Z, w, k, Zn, w, false);
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
    tile_times_small<NT_MM>(ALoadPlain{Qc, CH}, h, w, Z, w, k, out + row0, ldo, false);
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
      tile_times_small<NT_MM>(ALoadPlain{In, 64}, rows, w, Ps, w, k, out + it.row0, ldo, false);
    else
      tile_times_small<NT_MM>(ALoadPlain{In, 64}, rows, w, P, WMAX, k, out + it.row0, ldo, false);
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
      tr_set_rank(J, w, k);
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
  if (tid == 0) tr_set_rank(J, w, k);
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
      tile_times_small<NT_TR>(ALoadPlain{Qn, CH}, w, w, Z, w, k, Zc, w, false);
      __syncthreads();
      Zuse = Zc;
    }
    const double* Qc = ws + S.node0 + (int64_t)c * TR_NODE + WMAX * WMAX;
    tile_times_small<NT_TR>(ALoadPlain{Qc, CH}, h, w, Zuse, w, k, J.out[0] + row0, J.ldout[0], false);
    __syncthreads();
  }
  // R' = R P.  R' may overwrite R in place (row r of R' over row r of R): every
  // thread reads its rows of a row block before any of them is stored.
  const int n0 = (int)hdr[3];
  double* Ps = sm;  // w x k, ld w
  for (int e = tid; e < w * k; e += NT_TR) Ps[e] = P[(e % w) + (e / w) * WMAX];
  __syncthreads();
  tile_times_small<NT_TR>(ALoadSegs{J.seg[1][0], J.seg[1][1], n0, 0}, J.side[1].m, w, Ps, w, k, J.out[1],
                          J.ldout[1], true);
}

// Wider jobs: the chunk code of k_tr_qr, one block per chunk (the chunks
// and sides join through the job's counters); the block that ran the SVD
// then forms both factors.
template <int WTOP, bool LOCAL = false>
__device__ __forceinline__ void tr_small_wide(const TrJob& J, int side, int chunk, int w, int n0a, int n0b,
                                              double* ws, int* counters, double* smem) {
  const int t = tier_of(w);
  bool last = false;
  if (t == 16) {
    if constexpr (WTOP >= 16) last = tr_chunk<16, LOCAL>(J, side, chunk, ws, counters, J.err, J.flops, smem, w, n0a, n0b);
  } else if (t == 32) {
    if constexpr (WTOP >= 32) last = tr_chunk<32, LOCAL>(J, side, chunk, ws, counters, J.err, J.flops, smem, w, n0a, n0b);
  } else if (t == 64) {
    if constexpr (WTOP >= 64) last = tr_chunk<64, LOCAL>(J, side, chunk, ws, counters, J.err, J.flops, smem, w, n0a, n0b);
  } else {
    if constexpr (WTOP >= 128)
      last = tr_chunk<128, LOCAL>(J, side, chunk, ws, counters, J.err, J.flops, smem, w, n0a, n0b);
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
      tr_set_rank(J, w, 0);
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

// A chain of recompressions in one block: jobs it.job .. it.job + it.chunk - 1
// in order, each reading the previous one's output (the term-by-term sums of
// Sec. 4: every added term is recompressed at once).  A step runs as k_tr_small
// runs a job: narrow (w <= 8) as one block does; wider, its chunks one after
// another in this block, the last one running the SVD and forming both
// factors.  The steps share the chain's workspace and counters; each step's
// outputs and rank are visible to the next after a block-scope fence (one
// block, one L2: no device-scope write-back and invalidation between steps).
// A wide step of a chain: its chunks one after another (out of line, so that
// the narrow steps keep the register allocation of k_tr_small).
template <int WTOP>
__device__ __noinline__ void tr_chain_wide(const TrJob& J, int w, int n0a, int n0b, double* ws, int* counters,
                                           double* smem) {
  for (int side = 0; side < 2; ++side)
    for (int c = 0; c < J.side[side].p0; ++c) {
      tr_small_wide<WTOP, true>(J, side, c, w, n0a, n0b, ws, counters, smem);
      __syncthreads();
    }
}

template <int WTOP>
__global__ void __launch_bounds__(NT_TR) k_tr_chain(const TrJob* __restrict__ jobs,
                                                     const TrChunk* __restrict__ items, int first,
                                                     double* ws, int* counters) {
  extern __shared__ double smem[];
  const TrChunk it = items[first + blockIdx.x];
#pragma unroll 1
  for (int s = 0; s < it.chunk; ++s) {
    const TrJob& J = jobs[it.job + s];
    const int n0a = seg_n(J.seg[0][0]);
    const int w = n0a + seg_n(J.seg[0][1]);
    const int n0b = seg_n(J.seg[1][0]);
    if (w == 0 || w > WTOP || max(J.side[0].m, J.side[1].m) > TRS_MAXCH * CH) {
      if (threadIdx.x == 0) {
        tr_set_rank(J, w, 0);
        if (w > 0) atomicOr(J.err, ERR_WIDTH);
      }
    } else if (w <= 4) {
      tr_small_narrow<4>(J, w, n0a, n0b, smem);
    } else if (w <= 8) {
      tr_small_narrow<8>(J, w, n0a, n0b, smem);
    } else {
      tr_chain_wide<WTOP>(J, w, n0a, n0b, ws, counters, smem);
    }
    __threadfence_block();
    __syncthreads();
  }
}
}  // namespace hq

namespace hq {
template __global__ void k_tr_qr<16>(const TrJob*, const TrChunk*, int, double*, int*);
template __global__ void k_tr_qr<32>(const TrJob*, const TrChunk*, int, double*, int*);
template __global__ void k_tr_qr<64>(const TrJob*, const TrChunk*, int, double*, int*);
template __global__ void k_tr_qr<128>(const TrJob*, const TrChunk*, int, double*, int*);
template __global__ void k_tr_chain<16>(const TrJob*, const TrChunk*, int, double*, int*);
template __global__ void k_tr_chain<32>(const TrJob*, const TrChunk*, int, double*, int*);
template __global__ void k_tr_small<16>(const TrJob*, const TrChunk*, int, double*, int*);
template __global__ void k_tr_small<32>(const TrJob*, const TrChunk*, int, double*, int*);
template __global__ void k_tr_small<64>(const TrJob*, const TrChunk*, int, double*, int*);
template __global__ void k_tr_small<128>(const TrJob*, const TrChunk*, int, double*, int*);
}  // namespace hq

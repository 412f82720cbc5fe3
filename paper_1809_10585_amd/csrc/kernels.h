// Kernel declarations and launch constants of the HODLR QR library, shared by
// the host scheduler (hodlr.cpp) and the kernel translation units (k_*.hip).
// Each kernel family is compiled on its own; the host launches them through
// these declarations.
#pragma once
#include "common.h"

namespace hq {

// ---------------------------------------------------------------- recompression (k_tr.hip)
// LDS layout of k_tr_qr / k_tr_small (doubles)
constexpr int TRS_VBUF = 0;
constexpr int TRS_TAU = 2 * CH;
constexpr int TRS_FLAG = TRS_TAU + WMAX;      // 16 doubles of int flags
constexpr int TRS_X = TRS_FLAG + 16;
constexpr int TRS_XSZ = WMAX * (WMAX + 1);                  // X (ld up to WMAX + 1), staging, V
constexpr int TRS_TOTAL = TRS_X + TRS_XSZ + 2 * WMAX;           // + sig + perm
constexpr size_t TR_QR_LDS = sizeof(double) * (size_t)TRS_TOTAL;
constexpr size_t TR_FORM_LDS = sizeof(double) * (size_t)WMAX * WMAX;
// k_tr_small takes factors of at most this many CH-row chunks per side
constexpr int TRS_MAXCH = 4;

template <int WTOP>
__global__ void k_tr_qr(const TrJob* __restrict__ jobs, const TrChunk* __restrict__ items, int first,
                        double* ws, int* counters);
template <int WTOP>
__global__ void k_tr_chain(const TrJob* __restrict__ jobs, const TrChunk* __restrict__ items, int first,
                           double* ws, int* counters);
template <int WTOP>
__global__ void k_tr_small(const TrJob* __restrict__ jobs, const TrChunk* __restrict__ items, int first,
                           double* ws, int* counters);
__global__ void k_tr_form(const TrJob* __restrict__ jobs, const TrForm* __restrict__ items, int first,
                          const double* __restrict__ ws);

// ---------------------------------------------------------------- products (k_mm.hip)
constexpr int MA_LD = 17;
constexpr int DT_LD = 65;  // transposed leaf tile, padded row
// dynamic LDS of k_mm_apply: max(m_leaf, 256) * MA_LD doubles (staged X, then
// the groups' partial rows) and the wavefronts' 16 x 16 MFMA partial tiles
__host__ __device__ constexpr size_t mm_apply_lds(int mleaf) {
  return sizeof(double) * ((size_t)MA_LD * (size_t)(mleaf > 256 ? mleaf : 256) + (size_t)(NT_MM / 64) * 256);
}

__global__ void k_mm_proj(const MmJob* __restrict__ jobs, const MmProj* __restrict__ items, int first,
                          double* ws, Opnd op);
__global__ void k_mm_red(const MmJob* __restrict__ jobs, const MmProj* __restrict__ items, int first,
                         double* ws, Opnd op);
template <int RT>
__global__ void k_mm_apply(const MmJob* __restrict__ jobs, const MmApply* __restrict__ items, int first,
                           const double* __restrict__ ws, Opnd op);
__global__ void k_gemm_tall(const GemmJob* __restrict__ jobs, const GemmTile* __restrict__ items, int first,
                            Opnd op);
__global__ void k_gemm_red(const GemmJob* __restrict__ jobs, const GemmRed* __restrict__ items, int first,
                           double* ws, int* counters, Opnd op);

// ---------------------------------------------------------------- leaf QR (k_leaf.hip)
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

__global__ void k_leaf_gather(const LeafJob* __restrict__ jobs, int first, int nper);
__global__ void k_leaf_step(const LeafJob* __restrict__ jobs, int first, int nper, int p);
__global__ void k_leaf_scatter(const LeafJob* __restrict__ jobs, int first, int nper);

// ---------------------------------------------------------------- vectors (k_vec.hip)
__global__ void k_normalize(const VecJob* __restrict__ items, int first);
__global__ void k_set_scal(const VecJob* __restrict__ items, int first, int count);
__global__ void k_fill_items(const VecJob* __restrict__ items, int first);
__global__ void k_fill(double* x, int64_t n, double v);
__global__ void k_zero_i32(int* x, int n);
__global__ void k_rows(const RowJob* __restrict__ items, int first);
__global__ void k_pivot_rows(const int* __restrict__ runs, int nrun, const double* B, int ldb, double* X, int ldx,
                             int ncols);
__global__ void k_leaf_trsm(const double* __restrict__ D, int m, int ld, double* X, int ldx, int nrhs);

}  // namespace hq

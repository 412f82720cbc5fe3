// Shared host/device definitions of the HODLR QR library: the work
// descriptors the host scheduler writes once per factorisation and the
// kernels read.  Everything is FP64; sizes that depend on truncation ranks
// are read on the device through `const int*` pointers, so a whole
// factorisation can be queued (or captured) without host round trips.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hq {

constexpr int CH = 256;        // rows of one tall-skinny QR chunk (TSQR leaf)
constexpr int MM_CH = 1024;    // rows of one projection chunk of a HODLR product
constexpr int WMAX = 128;      // widest recompression handled on the device
constexpr int SMAX = 64;       // widest tall-skinny operand of a HODLR product
constexpr int KCAP = 64;       // largest rank capacity of a stored block
constexpr int NT_TR = 512;     // threads of the recompression kernels
constexpr int NT_MM = 256;     // threads of the product / GEMM / leaf kernels
constexpr int NB = 16;         // leaf QR panel width (one wavefront per column)
constexpr int NT_LEAF = 1024;  // threads of the leaf QR kernels (16 wavefronts)
constexpr int MAXLEAF = 512;   // largest leaf order
constexpr int MAXSTACK = 1024; // largest stacked leaf column (leaf + group rows)
constexpr int MAXGROUPS = 24;

// size (doubles) of one TSQR tree node's storage: R (WMAX x WMAX) + Q (CH x WMAX)
constexpr int64_t TR_NODE = (int64_t)WMAX * WMAX + (int64_t)CH * WMAX;
// size (doubles) of a recompression job header: 8 scalars + U_k + P (+ V scratch)
constexpr int64_t TR_HDR = 8 + 3 * (int64_t)WMAX * WMAX;

// device-side error bits
enum : int { ERR_CAPACITY = 1, ERR_WIDTH = 2, ERR_STACK = 4 };

// flop counter categories (same counting conventions as the CPU oracle).  The
// factorisation's total sums the first FC_N; FC_NORM (the |A|_2 power
// iteration, which the oracle does not count) is kept apart.
enum : int { FC_LEAF = 0, FC_HMAT = 1, FC_TRUNC = 2, FC_DENSE = 3, FC_UPDATE = 4, FC_ORTH = 5,
             FC_N = 6, FC_NORM = 6 };
// flop counters: FC_N categories x FC_STRIPE stripes (summed on the host)
constexpr int FC_STRIPE = 64;
constexpr int FC_SIZE = 8 * FC_STRIPE;

// Operands bound per call of a cached launch sequence (apply Q, solve,
// products): jobs that name a slot >= 0 read pointer p[slot] + their offset and
// leading dimension ld[slot]; a job whose width is not fixed uses s columns.
// Passed to the kernels by value, so a cached sequence is reused with new
// operands without touching device memory.
struct Opnd {
  double* p[4];
  int ld[4];
  int s;
};

// Columns [0, ncols) of a column-major array, scaled by `scale`.  ncols is
// *ncols_dev when that pointer is set.  p == nullptr means an empty segment.
struct Seg {
  const double* p;
  int ld;
  int ncols;
  const int* ncols_dev;
  double scale;
};

// ---------------------------------------------------------------- recompression
// One recompression T_tau: block = L R^T with L = [seg[0][0] | seg[0][1]]
// (m[0] rows) and R = [seg[1][0] | seg[1][1]] (m[1] rows).  Output
// L' = Q1 U_k (orthonormal) into out[0], R' = R (R1^T U_k) into out[1],
// k into *out_rank.  flags & TR_ORTH: left-orthogonalisation only (k = w,
// U = I); side 1 is then not factorised.
enum : int { TR_ORTH = 1 };

struct TrSide {
  int m;            // rows
  int p0;           // level-0 chunks (rows split evenly, each >= CH/2 when p0 > 1)
  int64_t node0;    // storage of node slot 0 (chunks, then combine nodes), TR_NODE each
  int cnt0;         // first counter of this side (one per combine slot)
};

struct TrJob {
  Seg seg[2][2];
  TrSide side[2];
  const double* tau;  // threshold (device scalar: eps*|A|_2 or eps)
  int flags;
  double* out[2];
  int ldout[2];
  int cap;          // columns available in out[*]
  int* out_rank;
  int jcounter;     // counter joining the two sides
  int fc;           // flop category
  int64_t hdr;      // offset (doubles) of the job header in the workspace
  int* err;         // error word of the factorisation the job belongs to
  double* flops;    // flop counters of that factorisation
  int* log;         // rank log entry (input width, kept rank) or nullptr
};

struct TrChunk {    // one block of the first recompression kernel
  int job, side, chunk;  // (k_tr_chain: jobs job .. job + chunk - 1 in order; side unused)
};

struct TrForm {     // one block of the second recompression kernel
  int job, side;
  int chunk;        // side 0: TSQR chunk
  int row0, rows;   // side 1: output rows
  int leader;       // writes *out_rank
};

// ---------------------------------------------------------------- HODLR views
struct HBlk {       // A(r0:r0+rows, c0:c0+cols) = U V^T, rank *rank
  double* U;
  double* V;
  int ldU, ldV;
  int* rank;
  int64_t r0, c0;
  int rows, cols;
};

struct HLeaf {       // D(0:m, 0:n) of the rows from r0 and the columns from c0
  double* D;
  int ld;
  int64_t r0;
  int m;             // rows
  int64_t c0;
  int n;             // columns (a leaf of a rectangular HODLR matrix has m >= n)
};

enum : int { LEAF_FULL = 0, LEAF_UNIT_LOWER = 1, LEAF_UPPER = 2 };

// A HODLR matrix as seen by the product kernels.  up/lo are indexed by the
// heap number of the internal node (nullptr: blocks of that kind are zero).
struct HView {
  int levels;
  const HBlk* up;
  const HBlk* lo;
  const HLeaf* leaf;   // indexed by leaf number j (heap node 2^levels + j)
  int leaf_kind;
};

// Z = alpha * op(M_v) X + beta * Z  for the sub-HODLR rooted at heap node v.
// X (Z) is operand slot xs (zs) + xoff (zoff) when xs (zs) >= 0.  Width: *s_dev
// if set, else s if > 0, else the call's Opnd::s.
struct MmJob {
  HView M;
  int v;
  int trans;
  const double* X;
  int ldX;
  int s;
  const int* s_dev;
  double* Z;
  int ldZ;
  double alpha, beta;
  int64_t row0;        // global row index of row 0 of the row-space operand (Z; X when trans)
  int64_t col0;        // global column index of row 0 of the column-space operand (X; Z when trans)
  int64_t red0;        // reduced projection of node u, kind t at
                       // red0 + (2*(rel(u)) + t) * rld*SMAX
  int rld;             // leading dimension of a projection (>= every block rank)
  int tri;             // triangular operand (halves the leaf flop count)
  int fc;              // flop category
  int xs, zs;
  int64_t xoff, zoff;
  double* flops;
};

struct MmProj {      // phase A: one row chunk of one block projection
  int job;
  int node;
  int kind;          // 0 = upper block, 1 = lower block
  int chunk, nchunk;
  int64_t part;      // this chunk's partial (rld x SMAX, ld rld); for k_mm_red
                     // items the first chunk's partial
};

struct MmApply {     // phase B: rows of one leaf of the output
  int job;
  int leaf;
  int row0, rows;    // rows within the leaf
};

// ---------------------------------------------------------------- small GEMMs
// C = beta*C + alpha * op(A) op(B); op(A) is M x K, op(B) is K x N.  A, B, C
// are operand slot as_, bs_, cs_ + their offset when the slot is >= 0 (leading
// dimension from the slot unless lda/ldb/ldc > 0).  N: *Nd if set, else N if
// > 0, else the call's Opnd::s.
struct GemmJob {
  int ta, tb;
  int M, N, K;
  const int *Md, *Nd, *Kd;
  const double* A;
  int lda;
  const double* B;
  int ldb;
  double* C;
  int ldc;
  double alpha, beta;
  int fc;
  int as_, bs_, cs_;
  int64_t aoff, boff, coff;
  double* flops;
};

struct GemmTile {    // 64 x 64 output tile of a tall GEMM
  int job, row0, col0;
};

struct GemmRed {     // K chunk of a reduction GEMM (M, N <= KCAP)
  int job, k0, kn, nchunk, chunk;
  int64_t part;
  int counter;
};

// ---------------------------------------------------------------- leaf QR
// Stacked leaf column [A_leaf; C_g1; ...; C_gq] (Sec. 4.1, eq. compressedcol):
// the rows below the leaf are the current right factors of the lower blocks
// of the ancestors whose left subtree holds the leaf, nearest first, stored
// transposed (leaf column c of group g is row c of V_g).
struct LeafGroup {
  double* V;
  int ld;
  int row0;
  const int* rank;
};

struct LeafWs {     // workspace of one leaf QR (one per factorisation: its leaves run in turn)
  double* H;        // stacked matrix, ld MAXSTACK
  double* T;        // T (MAXLEAF x MAXLEAF, ld MAXLEAF)
  double* G;        // Y^T Y blocks above the panel diagonal (ld MAXLEAF)
};
struct LeafJob {
  double* D;        // leaf (mr x m, ld mr): A on input, R + Y on output
  int m;            // columns
  int mr;           // rows of D (m for a square matrix, m_j >= n_j in Sec. 6)
  double* Tleaf;    // T leaf output (m x m, ld m)
  LeafWs ws;
  int* err;
  double* flops;
  int ngroups;
  LeafGroup g[MAXGROUPS];
};
struct RowJob {     // copy rows [src_r0, src_r0 + rows) of a column-major array to dst_r0..
  const double* src;
  int lds;
  double* dst;
  int ldd;
  int src_r0, dst_r0, rows;
  const int* ncols_dev;  // columns: *ncols_dev when set, else ncols
  int ncols;
};
struct VecJob {     // one vector of a batched fill / normalise / threshold op
  const double* z;
  double* x;
  int64_t n;
  double* out;
  double d0, d1;
};



}  // namespace hq

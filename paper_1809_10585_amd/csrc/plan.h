// Host-side structures of the HODLR QR library: device memory (through the
// caller's allocator when one is installed), the tree of a partition, the
// factor storage sets, and the flat launch plan that the scheduler compiles
// Algorithm hQR (Kressner & Susnjara, Sec. 4) into.  Shared by the scheduler
// and C ABI (hodlr.cpp) and the plan's hazard checker (check.cpp).
#pragma once
#include "kernels.h"

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "hodlr.h"

namespace hqh {

using namespace hq;

// ------------------------------------------------------------------ errors
hodlr_status fail(hodlr_status s, const std::string& m);
extern thread_local std::string g_err;

#define HIPCHK(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess) {                                                             \
      ::hqh::g_err = std::string(#x) + ": " + hipGetErrorString(e_);                    \
      return e_ == hipErrorOutOfMemory ? HODLR_ENOMEM : HODLR_EDEVICE;                  \
    }                                                                                   \
  } while (0)

#define TRY(x)                       \
  do {                               \
    hodlr_status s_ = (x);           \
    if (s_ != HODLR_OK) return s_;   \
  } while (0)

// ------------------------------------------------------------------ device memory
// The caller's allocator (hodlr_set_allocator); null members: hipMalloc / hipFree.
struct AllocHook {
  void* (*alloc)(size_t, void*, void*) = nullptr;
  void (*release)(void*, void*, void*) = nullptr;
  void* ctx = nullptr;
};
AllocHook current_hook();

// Planning without a device (the hazard checker): allocations hand out
// distinct fake addresses, copies and fills are skipped.  Thread-local.
extern thread_local bool g_virtual;
void* virtual_alloc(size_t bytes);

// Memory owned by one handle.  Every allocation goes through the allocator
// hook captured at the first allocation (or hipMalloc), on `stream`, and is
// released the same way when the DMem dies.
struct DMem {
  struct Blk {
    void* p;
    size_t bytes;
  };
  std::vector<Blk> ptrs;
  size_t bytes = 0;
  AllocHook hook;
  bool hooked = false;
  bool virt = false;
  hipStream_t stream = nullptr;
  // when set, every allocation is zero-filled on `stream` (capacity padding of
  // factors and temporaries then holds zeros, never recycled garbage)
  bool zero = false;
  DMem() = default;
  DMem(const DMem&) = delete;
  DMem& operator=(const DMem&) = delete;
  ~DMem();
  hodlr_status raw(void** out, size_t bytes);
  template <class T>
  hodlr_status alloc(T** out, size_t count) {
    void* p = nullptr;
    TRY(raw(&p, (count == 0 ? 1 : count) * sizeof(T)));
    *out = static_cast<T*>(p);
    return HODLR_OK;
  }
};

// Memory of one call (apply Q, solve, products): taken from the caller's
// allocator on the call's stream, else hipMallocAsync; released in stream
// order when the call has queued its work.
struct CallMem {
  struct Blk {
    void* p;
    bool async;
  };
  std::vector<Blk> ptrs;
  AllocHook hook;
  hipStream_t stream;
  explicit CallMem(hipStream_t st);
  CallMem(const CallMem&) = delete;
  CallMem& operator=(const CallMem&) = delete;
  ~CallMem();
  hodlr_status raw(void** out, size_t bytes);
  template <class T>
  hodlr_status alloc(T** out, size_t count) {
    void* p = nullptr;
    TRY(raw(&p, (count == 0 ? 1 : count) * sizeof(T)));
    *out = static_cast<T*>(p);
    return HODLR_OK;
  }
};

// asynchronous host-to-device copy and zero fill (no-ops while planning virtually)
hodlr_status h2d(void* dst, const void* src, size_t bytes, hipStream_t st);
hodlr_status dzero(void* dst, size_t bytes, hipStream_t st);

template <class T>
hodlr_status upload(DMem& mem, T** d, const std::vector<T>& h, hipStream_t st) {
  TRY(mem.alloc(d, h.size()));
  if (!h.empty()) TRY(h2d(*d, h.data(), h.size() * sizeof(T), st));
  return HODLR_OK;
}

// ------------------------------------------------------------------ tree
// The partition of a HODLR matrix: columns [lo[v], hi[v]) and rows
// [rlo[v], rhi[v]) of heap node v (the same for a square matrix; a rectangular
// one, Sec. 6, has m_j >= n_j rows per leaf).
struct Tree {
  int L = 0;
  int64_t n = 0;                  // columns
  int64_t nr = 0;                 // rows
  std::vector<int64_t> lo, hi;    // column ranges, heap numbering 1 .. 2^(L+1)-1
  std::vector<int64_t> rlo, rhi;  // row ranges
  int nleaf() const { return 1 << L; }
  bool is_leaf(int v) const { return v >= (1 << L); }
  int64_t m(int v) const { return hi[v] - lo[v]; }     // columns of node v
  int64_t mr(int v) const { return rhi[v] - rlo[v]; }  // rows of node v
  bool rect() const { return nr != n || rlo != lo; }
  static void fill(int L, const int64_t* off, std::vector<int64_t>& lo, std::vector<int64_t>& hi) {
    lo.assign(2 << L, 0);
    hi.assign(2 << L, 0);
    for (int j = 0; j < (1 << L); ++j) {
      lo[(1 << L) + j] = off[j];
      hi[(1 << L) + j] = off[j + 1];
    }
    for (int v = (1 << L) - 1; v >= 1; --v) {
      lo[v] = lo[2 * v];
      hi[v] = hi[2 * v + 1];
    }
  }
  void init(int levels, const int64_t* off, const int64_t* row_off = nullptr) {
    L = levels;
    n = off[1 << L];
    fill(L, off, lo, hi);
    if (row_off == nullptr) row_off = off;
    nr = row_off[1 << L];
    fill(L, row_off, rlo, rhi);
  }
  // the square tree on the column partition (T, and R on its pivot rows)
  Tree square() const {
    Tree q = *this;
    q.nr = n;
    q.rlo = lo;
    q.rhi = hi;
    return q;
  }
  void subtree_internal(int v, std::vector<int>& out) const {
    if (is_leaf(v)) return;
    out.push_back(v);
    subtree_internal(2 * v, out);
    subtree_internal(2 * v + 1, out);
  }
  void subtree_leaves(int v, std::vector<int>& out) const {
    if (is_leaf(v)) {
      out.push_back(v - (1 << L));
      return;
    }
    subtree_leaves(2 * v, out);
    subtree_leaves(2 * v + 1, out);
  }
  int subtree_size(int v) const {  // nodes in the subtree (heap-relative numbering bound)
    int d = 31 - __builtin_clz(v);
    return (2 << (L - d)) - 1;
  }
};

// One family of off-diagonal blocks (upper, lower or T's upper) with rank
// capacity `cap` per block.
struct BlockSet {
  double* U = nullptr;
  double* V = nullptr;
  std::vector<int64_t> uoff, voff;
  int64_t usz = 0, vsz = 0;
  int* rank = nullptr;  // device, indexed by node
  HBlk* dview = nullptr;
  std::vector<HBlk> hview;
};

enum BKind { BK_UP = 0, BK_LO = 1 };
hodlr_status make_blocks(DMem& mem, const Tree& t, int cap, BKind kind, int* rank, BlockSet& B);

struct LeafSet {
  double* D = nullptr;
  std::vector<int64_t> off;
  int64_t size = 0;
  HLeaf* dview = nullptr;
  std::vector<HLeaf> hview;
};
hodlr_status make_leaves(DMem& mem, const Tree& t, LeafSet& S);

// ------------------------------------------------------------------ schedule
enum OpType {
  OP_TRQR, OP_TRFORM, OP_MMPROJ, OP_MMAPPLY, OP_GTALL, OP_GRED, OP_LGATHER, OP_LPANEL,
  OP_LUPDATE, OP_LSCATTER, OP_FILL, OP_NORMALIZE, OP_TRSM, OP_SETSCAL,
  OP_MMRED, OP_TRSMALL,
  OP_ROWS,    // row runs between arrays (k_rows)
  OP_TRCHAIN, // chains of recompressions, one block per chain (k_tr_chain)
  OP_SIGNAL,  // record event a0 on the op's lane (no kernel)
  OP_WAIT,    // the op's lane waits for event a0 (no kernel)
  OP_NTYPES
};
extern const char* const OP_NAMES[OP_NTYPES];

struct Op {
  int type;
  int first, count;  // item range (grid = count blocks)
  int a0;            // leaf job / panel / misc
  int a1;
  const double* p0;
  double* p1;
  double d0;
  int64_t n;
  double* pout;
  double d1;
  int lane = 0;      // 0: main chain, 1: the T-factor chain (runs beside it)
  int xs = -1;       // OP_TRSM: operand slot of the right-hand sides (grid: the call's s)
  int64_t xoff = 0;
};

// does the op launch a kernel (SIGNAL / WAIT and empty ops do not)
inline bool op_launches(const Op& o) {
  if (o.type == OP_SIGNAL || o.type == OP_WAIT) return false;
  return o.count > 0 || (o.type == OP_TRSM && o.xs >= 0);
}

struct TrSpec {
  Seg seg[2][2];
  int m[2];
  const double* tau;
  int flags;
  double* out[2];
  int ldout[2];
  int cap;
  int* out_rank;
  int fc;
  int* err;
  double* flops;
  int* log = nullptr;
};

struct MmSpec {
  HView M;
  bool has_up, has_lo;
  int v, trans;
  const double* X;
  int ldX;
  int s;
  const int* s_dev;
  double* Z;
  int ldZ;
  double alpha, beta;
  int tri;
  int rld = KCAP;  // rank capacity of M's blocks
  int fc = FC_HMAT;
  int xs = -1, zs = -1;
  int64_t xoff = 0, zoff = 0;
  double* flops = nullptr;
};

struct GSpec {  // gemm job with host-side capacities for tiling
  GemmJob J;
  int Mcap, Ncap, Kstat;
};

inline Seg mkseg(const double* p, int ld, const int* ncols_dev, double scale = 1.0, int ncols = 0) {
  Seg s;
  s.p = p;
  s.ld = ld;
  s.ncols = ncols;
  s.ncols_dev = ncols_dev;
  s.scale = scale;
  return s;
}
inline Seg noseg() { return mkseg(nullptr, 1, nullptr); }

// Launch-shape choices of the schedule builder, taken from the measured table
// (tune_table.h) for the problem's order and rank capacity unless overridden:
// product launches over at least mm_rt64_rows output rows take 64 rows per
// block (else 16); recompressions of at most tr_small_chunks row chunks per
// factor (rank capacity <= 32) run in one k_tr_small launch, larger ones in
// k_tr_qr + k_tr_form.
struct Tuning {
  int mm_rt64_rows = 32768;
  int tr_small_chunks = 4;
};
Tuning tuning_for(int64_t n, int cap);

struct Plan {
  std::vector<TrJob> trj;
  std::vector<TrChunk> trc;
  std::vector<TrForm> trf;
  std::vector<MmJob> mmj;
  std::vector<MmProj> mmp;
  std::vector<MmApply> mma;
  std::vector<GemmJob> gj;
  std::vector<GemmTile> gt;
  std::vector<GemmRed> gr;
  std::vector<LeafJob> lj;
  std::vector<VecJob> vj;
  std::vector<RowJob> rj;
  std::vector<Op> ops;
  // Workspace and counters are reused by consecutive ops of one lane; the two
  // lanes get disjoint regions because their ops may run at the same time.
  int64_t ws_lane[2] = {0, 0};
  int cnt_lane[2] = {1, 1};
  int lane = 0;  // lane of the ops being added
  int n_events = 0;
  int64_t ws_need() const { return ws_lane[0] + ws_lane[1]; }
  int cnt_need() const { return cnt_lane[0] + cnt_lane[1]; }
  int64_t ws_off(int l) const { return l == 0 ? 0 : ws_lane[0]; }
  int cnt_off(int l) const { return l == 0 ? 0 : cnt_lane[0]; }
  bool uses_counters() const;
  void push(Op o) {
    o.lane = lane;
    ops.push_back(o);
  }
  int signal() {
    Op o{OP_SIGNAL};
    o.a0 = n_events++;
    push(o);
    return o.a0;
  }
  void wait(int ev) {
    Op o{OP_WAIT};
    o.a0 = ev;
    push(o);
  }
  // one launch over vector items (fill / normalise / thresholds)
  void vec(int type, const std::vector<VecJob>& items) {
    const int first = (int)vj.size();
    vj.insert(vj.end(), items.begin(), items.end());
    push(Op{type, first, (int)items.size()});
  }
  int64_t n_trunc = 0;
  int wtop = WMAX;  // widest recompression this plan can produce
  Tuning tune;      // launch shapes (set by the builder from tuning_for)
  int mleaf = 0;    // largest leaf any product of this plan touches
  // device copies
  TrJob* d_trj = nullptr;
  TrChunk* d_trc = nullptr;
  TrForm* d_trf = nullptr;
  MmJob* d_mmj = nullptr;
  MmProj* d_mmp = nullptr;
  MmApply* d_mma = nullptr;
  GemmJob* d_gj = nullptr;
  GemmTile* d_gt = nullptr;
  GemmRed* d_gr = nullptr;
  LeafJob* d_lj = nullptr;
  VecJob* d_vj = nullptr;
  RowJob* d_rj = nullptr;

  std::vector<char> staged;  // host image of the descriptors (kept until the copy is done)

  void trunc(const std::vector<TrSpec>& specs);
  // steps[s][b]: step s of chain b (step s + 1 reads step s's output); one
  // launch when every step fits one block, else one trunc() per step
  void trunc_chain(const std::vector<std::vector<TrSpec>>& steps);
  TrJob make_trjob(const TrSpec& sp, int64_t& off, int& cnt) const;
  void mm(const Tree& t, const std::vector<MmSpec>& specs);
  void gemm_tall(const std::vector<GSpec>& specs);
  void gemm_red(const std::vector<GSpec>& specs);
  hodlr_status upload_all(DMem& mem, hipStream_t st);
};

// Workspace + counters + error word + flop counters shared by a handle's plans.
struct Work {
  double* ws = nullptr;
  int64_t ws_size = 0;
  int* counters = nullptr;
  int cnt_size = 0;
  int* err = nullptr;
  double* fc = nullptr;
  LeafWs leaf{};
};

// ------------------------------------------------------------------ hazard check
// What the checker needs besides the plan: the host copies of the block and
// leaf views the plan's products read (keyed by their device address), the
// rank capacity of the blocks, and the workspace the plan ran with.
struct CheckCtx {
  std::map<const void*, const std::vector<HBlk>*> blocks;
  std::map<const void*, const std::vector<HLeaf>*> leaves;
  int cap = KCAP;
  const Work* work = nullptr;
};
struct CheckResult {
  int64_t ops = 0, lane1_ops = 0, pairs = 0, conflicts = 0, intra_conflicts = 0;
  std::string first;
};
// Every pair of ops that two streams may run at the same time (lane order plus
// the plan's signal / wait events) and every pair of jobs inside one launch is
// tested for a write that overlaps a read or write of the other.
CheckResult check_plan(const Plan& P, const CheckCtx& C);

}  // namespace hqh

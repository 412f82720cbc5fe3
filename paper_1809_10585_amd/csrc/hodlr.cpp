// Host side of the HODLR QR library: device-resident HODLR storage, the
// depth-first schedule of Algorithm hQR (Kressner & Susnjara, Sec. 4)
// compiled into a flat list of batched kernel launches, its execution
// (directly or as a captured HIP graph), the cached launch sequences of
// apply-Q, solve and the products, and the C ABI of include/hodlr.h.
//
// Storage of the factors (all on A's partition):
//  * leaf j        : R (upper triangle) and Y (strictly lower, unit diagonal
//                    implied) share the leaf array; T has its own leaf array.
//  * upper block v : A12 on input; the recompressed block of R afterwards.
//  * lower block v : A21 = U V^T on input.  U is made orthonormal up front and
//                    stays the left factor of Y's lower block; V is
//                    overwritten by Y~_B^T slice by slice as the leaves below
//                    node v's left child are factorised (Y_B = B_L Y~_B).
//  * T block v     : T12 = -T1 T~12 T2 in factored form.
#include "plan.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

namespace hqh {

thread_local std::string g_err;

hodlr_status fail(hodlr_status s, const std::string& m) {
  g_err = m;
  return s;
}

const char* const OP_NAMES[OP_NTYPES] = {
  "tr_qr", "tr_form", "mm_proj", "mm_apply", "gemm_tall", "gemm_red", "leaf_gather", "leaf_panel",
  "leaf_update", "leaf_scatter", "fill", "normalize", "leaf_trsm", "set_scal", "mm_red", "tr_small",
  "rows", "tr_chain", "signal", "wait"};

// ------------------------------------------------------------------ memory
namespace {
std::mutex g_hook_mu;
AllocHook g_hook;
// hipMallocAsync: -1 not tried yet, 1 works, 0 not supported (hipMalloc then)
std::atomic<int> g_async_ok{-1};
}  // namespace

AllocHook current_hook() {
  std::lock_guard<std::mutex> lk(g_hook_mu);
  return g_hook;
}

thread_local bool g_virtual = false;

void* virtual_alloc(size_t bytes) {
  static std::atomic<uint64_t> next{(uint64_t)1 << 44};
  bytes = (bytes + 255) & ~(size_t)255;
  return (void*)(uintptr_t)next.fetch_add(bytes + 256);  // a gap after every block
}

DMem::~DMem() {
  if (virt) return;
  for (const Blk& b : ptrs) {
    if (hook.release != nullptr)
      hook.release(b.p, stream, hook.ctx);
    else
      (void)hipFree(b.p);
  }
}

hodlr_status DMem::raw(void** out, size_t nbytes) {
  *out = nullptr;
  if (g_virtual) {
    virt = true;
    void* p = virtual_alloc(nbytes);
    ptrs.push_back({p, nbytes});
    bytes += nbytes;
    *out = p;
    return HODLR_OK;
  }
  if (!hooked) {
    hook = current_hook();
    hooked = true;
  }
  void* p = nullptr;
  if (hook.alloc != nullptr) {
    p = hook.alloc(nbytes, stream, hook.ctx);
    if (p == nullptr)
      return fail(HODLR_ENOMEM, "the installed allocator returned NULL for " + std::to_string(nbytes) + " bytes");
  } else {
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(HODLR_ENOMEM, "hipMalloc of " + std::to_string(nbytes) + " bytes failed");
    }
  }
  ptrs.push_back({p, nbytes});
  bytes += nbytes;
  *out = p;
  if (zero) TRY(dzero(p, nbytes, stream));
  return HODLR_OK;
}

CallMem::CallMem(hipStream_t st) : hook(current_hook()), stream(st) {}

CallMem::~CallMem() {
  for (const Blk& b : ptrs) {
    if (hook.release != nullptr) {
      hook.release(b.p, stream, hook.ctx);
    } else if (b.async) {
      (void)hipFreeAsync(b.p, stream);
    } else {
      (void)hipStreamSynchronize(stream);
      (void)hipFree(b.p);
    }
  }
}

hodlr_status CallMem::raw(void** out, size_t nbytes) {
  *out = nullptr;
  void* p = nullptr;
  if (hook.alloc != nullptr) {
    p = hook.alloc(nbytes, stream, hook.ctx);
    if (p == nullptr)
      return fail(HODLR_ENOMEM, "the installed allocator returned NULL for " + std::to_string(nbytes) + " bytes");
    ptrs.push_back({p, false});
    *out = p;
    return HODLR_OK;
  }
  if (g_async_ok.load() != 0) {
    hipError_t e = hipMallocAsync(&p, nbytes, stream);
    if (e == hipSuccess) {
      g_async_ok.store(1);
      ptrs.push_back({p, true});
      *out = p;
      return HODLR_OK;
    }
    (void)hipGetLastError();
    if (e == hipErrorOutOfMemory) return fail(HODLR_ENOMEM, "hipMallocAsync failed");
    g_async_ok.store(0);
  }
  hipError_t e = hipMalloc(&p, nbytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(HODLR_ENOMEM, "hipMalloc of " + std::to_string(nbytes) + " bytes failed");
  }
  ptrs.push_back({p, false});
  *out = p;
  return HODLR_OK;
}

hodlr_status h2d(void* dst, const void* src, size_t nbytes, hipStream_t st) {
  if (g_virtual || nbytes == 0) return HODLR_OK;
  HIPCHK(hipMemcpyAsync(dst, src, nbytes, hipMemcpyHostToDevice, st));
  return HODLR_OK;
}

hodlr_status dzero(void* dst, size_t nbytes, hipStream_t st) {
  if (g_virtual || nbytes == 0) return HODLR_OK;
  HIPCHK(hipMemsetAsync(dst, 0, nbytes, st));
  return HODLR_OK;
}

// ------------------------------------------------------------------ storage
hodlr_status make_blocks(DMem& mem, const Tree& t, int cap, BKind kind, int* rank, BlockSet& B) {
  const int nn = 1 << t.L;
  B.uoff.assign(nn, 0);
  B.voff.assign(nn, 0);
  B.usz = B.vsz = 0;
  for (int v = 1; v < nn; ++v) {
    const int64_t rows = kind == BK_UP ? t.mr(2 * v) : t.mr(2 * v + 1);
    const int64_t cols = kind == BK_UP ? t.m(2 * v + 1) : t.m(2 * v);
    B.uoff[v] = B.usz;
    B.voff[v] = B.vsz;
    B.usz += rows * cap;
    B.vsz += cols * cap;
  }
  TRY(mem.alloc(&B.U, (size_t)B.usz));
  TRY(mem.alloc(&B.V, (size_t)B.vsz));
  B.rank = rank;
  B.hview.assign(nn, HBlk{});
  for (int v = 1; v < nn; ++v) {
    HBlk& b = B.hview[v];
    const bool up = kind == BK_UP;
    b.rows = (int)(up ? t.mr(2 * v) : t.mr(2 * v + 1));
    b.cols = (int)(up ? t.m(2 * v + 1) : t.m(2 * v));
    b.r0 = up ? t.rlo[2 * v] : t.rlo[2 * v + 1];
    b.c0 = up ? t.lo[2 * v + 1] : t.lo[2 * v];
    b.U = B.U + B.uoff[v];
    b.V = B.V + B.voff[v];
    b.ldU = b.rows;
    b.ldV = b.cols;
    b.rank = rank + v;
  }
  return HODLR_OK;
}

hodlr_status make_leaves(DMem& mem, const Tree& t, LeafSet& S) {
  const int nl = t.nleaf();
  S.off.assign(nl, 0);
  S.size = 0;
  for (int j = 0; j < nl; ++j) {
    S.off[j] = S.size;
    S.size += t.mr(nl + j) * t.m(nl + j);
  }
  TRY(mem.alloc(&S.D, (size_t)S.size));
  S.hview.assign(nl, HLeaf{});
  for (int j = 0; j < nl; ++j) {
    const int64_t mr = t.mr(nl + j), n = t.m(nl + j);
    S.hview[j] = HLeaf{S.D + S.off[j], (int)mr, t.rlo[nl + j], (int)mr, t.lo[nl + j], (int)n};
  }
  return HODLR_OK;
}

// ------------------------------------------------------------------ plan building
bool Plan::uses_counters() const {
  for (const Op& o : ops)
    if (o.type == OP_TRQR || o.type == OP_TRSMALL || o.type == OP_TRCHAIN || o.type == OP_GRED) return true;
  return false;
}

// The descriptor of one recompression; its header, tree nodes and counters
// are taken at off / cnt, which advance past them.
TrJob Plan::make_trjob(const TrSpec& sp, int64_t& off, int& cnt) const {
  TrJob J{};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) J.seg[a][b] = sp.seg[a][b];
  J.tau = sp.tau;
  J.flags = sp.flags;
  J.out[0] = sp.out[0];
  J.out[1] = sp.out[1];
  J.ldout[0] = sp.ldout[0];
  J.ldout[1] = sp.ldout[1];
  J.cap = sp.cap;
  J.out_rank = sp.out_rank;
  J.fc = sp.fc;
  J.err = sp.err;
  J.flops = sp.flops;
  J.log = sp.log;
  J.hdr = off;
  off += TR_HDR;
  for (int side = 0; side < 2; ++side) {
    TrSide& S = J.side[side];
    S.m = sp.m[side];
    if (side == 1 && (sp.flags & TR_ORTH)) {
      S.p0 = 0;
      S.node0 = 0;
      S.cnt0 = 0;
      continue;
    }
    S.p0 = std::max(1, (S.m + CH - 1) / CH);
    S.node0 = off;
    off += 2 * (int64_t)S.p0 * TR_NODE;
    S.cnt0 = cnt;
    cnt += S.p0;
  }
  J.jcounter = cnt++;
  return J;
}

// A chain runs in one block when every step would run in k_tr_small (factors
// of at most tr_small_chunks chunks) and the widths stay in the narrow tiers
// (rank capacity <= 16): a narrow step (w <= 8) runs as in k_tr_small, a wider
// one runs its chunks one after another.  The steps share one workspace and one
// set of counters (the largest step's).
void Plan::trunc_chain(const std::vector<std::vector<TrSpec>>& steps) {
  if (steps.empty()) return;
  bool fuse = steps.size() > 1 && wtop <= 32;
  for (const auto& st : steps) {
    if (st.size() != steps[0].size()) fuse = false;
    for (const TrSpec& sp : st) {
      const int mx = std::max(sp.m[0], sp.m[1]);
      if ((sp.flags & TR_ORTH) || mx > std::min(tune.tr_small_chunks, TRS_MAXCH) * CH) fuse = false;
    }
  }
  if (!fuse) {
    for (const auto& st : steps) trunc(st);
    return;
  }
  const int first = (int)trc.size();
  int64_t off = 0;
  int cnt = 0;
  for (size_t b = 0; b < steps[0].size(); ++b) {
    const int j0 = (int)trj.size();
    int64_t end = off;
    int cend = cnt;
    for (const auto& st : steps) {
      int64_t o = off;
      int c = cnt;
      trj.push_back(make_trjob(st[b], o, c));
      ++n_trunc;
      end = std::max(end, o);
      cend = std::max(cend, c);
    }
    trc.push_back(TrChunk{j0, -1, (int)steps.size()});
    off = end;
    cnt = cend;
  }
  push(Op{OP_TRCHAIN, first, (int)(trc.size() - first)});
  ws_lane[lane] = std::max(ws_lane[lane], off);
  cnt_lane[lane] = std::max(cnt_lane[lane], cnt);
}

void Plan::trunc(const std::vector<TrSpec>& specs) {
  if (specs.empty()) return;
  int64_t off = 0;
  int cnt = 0;
  const int c_first = (int)trc.size(), f_first = (int)trf.size();
  std::vector<TrChunk> small;
  for (const TrSpec& sp : specs) {
    const TrJob J = make_trjob(sp, off, cnt);
    const int jid = (int)trj.size();
    trj.push_back(J);
    ++n_trunc;
    // factors of a few chunks: k_tr_small (for wide jobs its forming step
    // needs a tree of one combine level and w k doubles of LDS twice)
    const int mx = std::max(J.side[0].m, J.side[1].m);
    if (mx <= CH || (wtop <= 64 && mx <= tune.tr_small_chunks * CH)) {
      for (int side = 0; side < 2; ++side)
        for (int c = 0; c < J.side[side].p0; ++c) small.push_back(TrChunk{jid, side, c});
      continue;
    }
    for (int side = 0; side < 2; ++side)
      for (int c = 0; c < J.side[side].p0; ++c) trc.push_back(TrChunk{jid, side, c});
    bool leader = true;
    for (int c = 0; c < J.side[0].p0; ++c) {
      trf.push_back(TrForm{jid, 0, c, 0, 0, leader ? 1 : 0});
      leader = false;
    }
    for (int r0 = 0; r0 < J.side[1].m; r0 += 64)
      trf.push_back(TrForm{jid, 1, 0, r0, std::min(64, J.side[1].m - r0), 0});
  }
  if (!small.empty()) {
    const int s_first = (int)trc.size();
    trc.insert(trc.end(), small.begin(), small.end());
    push(Op{OP_TRSMALL, s_first, (int)small.size()});
  }
  if ((int)trc.size() > c_first + (int)small.size()) {
    push(Op{OP_TRQR, c_first, (int)trc.size() - c_first - (int)small.size()});
    push(Op{OP_TRFORM, f_first, (int)trf.size() - f_first});
  }
  ws_lane[lane] = std::max(ws_lane[lane], off);
  cnt_lane[lane] = std::max(cnt_lane[lane], cnt);
}

namespace {
int rel_node_h(int u, int v) {
  int du = 0, dv = 0;
  while ((u >> du) > 1) ++du;
  while ((v >> dv) > 1) ++dv;
  const int d = du - dv;
  return (1 << d) - 1 + (u - (v << d));
}
}  // namespace

// Z = alpha op(M_v) X + beta Z for every spec: projections of all blocks in one
// launch (plus a summing launch if some block spans several chunks), then the
// leaf rows in one launch.
void Plan::mm(const Tree& t, const std::vector<MmSpec>& specs) {
  int64_t off = 0;
  const int p_first = (int)mmp.size();
  std::vector<MmProj> reds;
  int64_t rows_total = 0;
  for (const MmSpec& sp : specs) rows_total += sp.trans ? t.m(sp.v) : t.mr(sp.v);
  const int RT = rows_total >= tune.mm_rt64_rows ? 64 : 16;
  std::vector<MmApply> apply;
  for (const MmSpec& sp : specs) {
    MmJob J{};
    J.M = sp.M;
    J.v = sp.v;
    J.trans = sp.trans;
    J.X = sp.X;
    J.ldX = sp.ldX;
    J.s = sp.s;
    J.s_dev = sp.s_dev;
    J.Z = sp.Z;
    J.ldZ = sp.ldZ;
    J.alpha = sp.alpha;
    J.beta = sp.beta;
    J.row0 = t.rlo[sp.v];
    J.col0 = t.lo[sp.v];
    J.tri = sp.tri;
    J.fc = sp.fc;
    J.xs = sp.xs;
    J.zs = sp.zs;
    J.xoff = sp.xoff;
    J.zoff = sp.zoff;
    J.flops = sp.flops;
    J.rld = sp.rld;
    const int64_t stride = (int64_t)sp.rld * SMAX;
    J.red0 = off;
    off += 2 * (int64_t)t.subtree_size(sp.v) * stride;
    const int jid = (int)mmj.size();
    std::vector<int> nodes;
    t.subtree_internal(sp.v, nodes);
    for (int u : nodes) {
      for (int kind = 0; kind < 2; ++kind) {
        if ((kind == 0 && !sp.has_up) || (kind == 1 && !sp.has_lo)) continue;
        const int64_t rows = kind == 0 ? t.mr(2 * u) : t.mr(2 * u + 1);
        const int64_t cols = kind == 0 ? t.m(2 * u + 1) : t.m(2 * u);
        const int64_t len = sp.trans ? rows : cols;
        const int nch = (int)((len + MM_CH - 1) / MM_CH);
        if (nch == 1) {
          const int64_t red = J.red0 + (int64_t)(2 * rel_node_h(u, sp.v) + kind) * stride;
          mmp.push_back(MmProj{jid, u, kind, 0, 1, red});
        } else {
          for (int c = 0; c < nch; ++c) mmp.push_back(MmProj{jid, u, kind, c, nch, off + (int64_t)c * stride});
          reds.push_back(MmProj{jid, u, kind, 0, nch, off});
          off += (int64_t)nch * stride;
        }
      }
    }
    mmj.push_back(J);
    std::vector<int> leaves;
    t.subtree_leaves(sp.v, leaves);
    for (int j : leaves) {
      const int lv = t.nleaf() + j;
      const int m = (int)(sp.trans ? t.m(lv) : t.mr(lv));  // output rows of the leaf
      mleaf = std::max(mleaf, (int)std::max(t.m(lv), t.mr(lv)));
      for (int r0 = 0; r0 < m; r0 += RT) apply.push_back(MmApply{jid, j, r0, std::min(RT, m - r0)});
    }
  }
  if ((int)mmp.size() > p_first) push(Op{OP_MMPROJ, p_first, (int)mmp.size() - p_first});
  if (!reds.empty()) {
    const int r_first = (int)mmp.size();
    mmp.insert(mmp.end(), reds.begin(), reds.end());
    push(Op{OP_MMRED, r_first, (int)reds.size()});
  }
  const int a_first = (int)mma.size();
  mma.insert(mma.end(), apply.begin(), apply.end());
  push(Op{OP_MMAPPLY, a_first, (int)apply.size(), 0, RT});
  ws_lane[lane] = std::max(ws_lane[lane], off);
}

void Plan::gemm_tall(const std::vector<GSpec>& specs) {
  if (specs.empty()) return;
  const int t_first = (int)gt.size();
  for (const GSpec& g : specs) {
    const int jid = (int)gj.size();
    gj.push_back(g.J);
    for (int r0 = 0; r0 < g.Mcap; r0 += 64)
      for (int c0 = 0; c0 < g.Ncap; c0 += 64) gt.push_back(GemmTile{jid, r0, c0});
  }
  if ((int)gt.size() > t_first) push(Op{OP_GTALL, t_first, (int)gt.size() - t_first});
}

void Plan::gemm_red(const std::vector<GSpec>& specs) {
  if (specs.empty()) return;
  int64_t off = 0;
  int cnt = 0;
  const int r_first = (int)gr.size();
  for (const GSpec& g : specs) {
    const int jid = (int)gj.size();
    gj.push_back(g.J);
    const int K = g.Kstat;
    const int nch = std::max(1, (K + CH - 1) / CH);
    const int counter = cnt++;
    for (int c = 0; c < nch; ++c)
      gr.push_back(GemmRed{jid, c * CH, std::min(CH, K - c * CH), nch, c, off + (int64_t)c * KCAP * KCAP,
                           counter});
    if (nch > 1) off += (int64_t)nch * KCAP * KCAP;
  }
  push(Op{OP_GRED, r_first, (int)gr.size() - r_first});
  ws_lane[lane] = std::max(ws_lane[lane], off);
  cnt_lane[lane] = std::max(cnt_lane[lane], cnt);
}

namespace {
// one device buffer for all descriptor arrays of a plan (one allocation, one copy)
struct Packer {
  std::vector<char>& buf;
  std::vector<std::pair<size_t, void**>> fix;
  template <class T>
  void add(const std::vector<T>& v, T** dptr) {
    size_t off = (buf.size() + 255) & ~(size_t)255;
    buf.resize(off + std::max<size_t>(1, v.size()) * sizeof(T));
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(T));
    fix.push_back({off, (void**)dptr});
  }
};
}  // namespace

hodlr_status Plan::upload_all(DMem& mem, hipStream_t st) {
  staged.clear();
  Packer pk{staged, {}};
  pk.add(trj, &d_trj);
  pk.add(trc, &d_trc);
  pk.add(trf, &d_trf);
  pk.add(mmj, &d_mmj);
  pk.add(mmp, &d_mmp);
  pk.add(mma, &d_mma);
  pk.add(gj, &d_gj);
  pk.add(gt, &d_gt);
  pk.add(gr, &d_gr);
  pk.add(lj, &d_lj);
  pk.add(vj, &d_vj);
  pk.add(rj, &d_rj);
  char* base = nullptr;
  TRY(mem.alloc(&base, staged.size()));
  for (auto& f : pk.fix) *f.second = base + f.first;
  return h2d(base, staged.data(), staged.size(), st);
}

// ------------------------------------------------------------------ execution
namespace {

hodlr_status ensure_work(DMem& mem, Work& W, int64_t ws_need, int cnt_need, bool leafws, hipStream_t st) {
  if (W.err == nullptr) {
    TRY(mem.alloc(&W.err, 4));
    TRY(mem.alloc(&W.fc, FC_SIZE));
    TRY(dzero(W.err, 4 * sizeof(int), st));
    TRY(dzero(W.fc, FC_SIZE * sizeof(double), st));
  }
  if (ws_need > W.ws_size) {
    TRY(mem.alloc(&W.ws, (size_t)ws_need));
    W.ws_size = ws_need;
  }
  if (cnt_need > W.cnt_size) {
    TRY(mem.alloc(&W.counters, (size_t)cnt_need));
    TRY(dzero(W.counters, (size_t)cnt_need * sizeof(int), st));
    W.cnt_size = cnt_need;
  }
  if (leafws && W.leaf.H == nullptr) {
    TRY(mem.alloc(&W.leaf.H, (size_t)MAXSTACK * MAXLEAF));
    TRY(mem.alloc(&W.leaf.T, (size_t)MAXLEAF * MAXLEAF));
    TRY(mem.alloc(&W.leaf.G, (size_t)MAXLEAF * MAXLEAF));
  }
  return HODLR_OK;
}

// sum of the striped device flop counters of categories [c0, c1) (synchronous); -1 on failure
double flop_sum(const double* fc, int c0, int c1) {
  std::vector<double> h(FC_SIZE);
  if (hipMemcpy(h.data(), fc, FC_SIZE * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return -1.0;
  double tot = 0.0;
  for (int c = c0; c < c1; ++c)
    for (int k = 0; k < FC_STRIPE; ++k) tot += h[c * FC_STRIPE + k];
  return tot;
}
double flop_total(const double* fc) { return flop_sum(fc, 0, FC_N); }

std::once_flag g_attr_once;
hodlr_status g_attr_status = HODLR_OK;
std::string g_attr_msg;

hodlr_status set_attrs() {
  std::call_once(g_attr_once, [] {
    auto set = [](const void* f, size_t bytes) {
      hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
      if (e != hipSuccess && g_attr_status == HODLR_OK) {
        g_attr_status = HODLR_EDEVICE;
        g_attr_msg = std::string("hipFuncSetAttribute: ") + hipGetErrorString(e);
      }
    };
    for (const void* f : {(const void*)k_tr_qr<16>, (const void*)k_tr_qr<32>, (const void*)k_tr_qr<64>,
                          (const void*)k_tr_qr<128>, (const void*)k_tr_small<16>, (const void*)k_tr_small<32>,
                          (const void*)k_tr_small<64>, (const void*)k_tr_small<128>, (const void*)k_tr_chain<16>,
                          (const void*)k_tr_chain<32>})
      set(f, TR_QR_LDS);
    set((const void*)k_tr_form, TR_FORM_LDS);
    for (const void* f : {(const void*)k_mm_apply<16>, (const void*)k_mm_apply<64>}) set(f, mm_apply_lds(MAXLEAF));
    set((const void*)k_leaf_step, LEAF_LDS);
  });
  if (g_attr_status != HODLR_OK) return fail(g_attr_status, g_attr_msg);
  return HODLR_OK;
}

// Launch a kernel; with events set (diagnostic profiling) through hipExtLaunchKernel,
// which stamps the two events at the dispatch's own start and end.
struct Launch {
  hipEvent_t e0 = nullptr, e1 = nullptr;
};

template <typename... P, typename... A>
void launch(const Launch& L, void (*kern)(P...), dim3 g, dim3 b, size_t sh, hipStream_t st, A&&... a) {
  if (L.e0 == nullptr) {
    kern<<<g, b, sh, st>>>(std::forward<A>(a)...);
    return;
  }
  std::tuple<std::decay_t<P>...> t(std::forward<A>(a)...);
  void* args[sizeof...(P) + 1];
  std::apply([&](auto&... x) {
    int i = 0;
    ((args[i++] = (void*)&x), ...);
  }, t);
  (void)hipExtLaunchKernel((const void*)kern, g, b, args, sh, st, L.e0, L.e1, 0);
}

void run_op(const Plan& P, const Work& W, const Op& o, hipStream_t st, const Launch& L, const Opnd& op) {
  if (!op_launches(o)) return;
  double* ws = W.ws ? W.ws + P.ws_off(o.lane) : nullptr;
  int* cnt = W.counters ? W.counters + P.cnt_off(o.lane) : nullptr;
  switch (o.type) {
    case OP_TRQR: {
      const int wt = P.wtop;
      auto kern = wt <= 16 ? k_tr_qr<16> : wt <= 32 ? k_tr_qr<32> : wt <= 64 ? k_tr_qr<64> : k_tr_qr<128>;
      launch(L, kern, o.count, NT_TR, TR_QR_LDS, st, P.d_trj, P.d_trc, o.first, ws, cnt);
      break;
    }
    case OP_TRSMALL: {
      const int wt = P.wtop;
      auto kern = wt <= 16 ? k_tr_small<16> : wt <= 32 ? k_tr_small<32> : wt <= 64 ? k_tr_small<64> : k_tr_small<128>;
      launch(L, kern, o.count, NT_TR, TR_QR_LDS, st, P.d_trj, P.d_trc, o.first, ws, cnt);
      break;
    }
    case OP_TRCHAIN:
      launch(L, P.wtop <= 16 ? k_tr_chain<16> : k_tr_chain<32>, o.count, NT_TR, TR_QR_LDS, st, P.d_trj, P.d_trc,
             o.first, ws, cnt);
      break;
    case OP_TRFORM:
      launch(L, k_tr_form, o.count, NT_MM, TR_FORM_LDS, st, P.d_trj, P.d_trf, o.first, (const double*)ws);
      break;
    case OP_MMPROJ:
      launch(L, k_mm_proj, o.count, NT_MM, 0, st, P.d_mmj, P.d_mmp, o.first, ws, op);
      break;
    case OP_MMRED:
      launch(L, k_mm_red, o.count, NT_MM, 0, st, P.d_mmj, P.d_mmp, o.first, ws, op);
      break;
    case OP_MMAPPLY:
      launch(L, o.a1 == 64 ? k_mm_apply<64> : k_mm_apply<16>, o.count, NT_MM, mm_apply_lds(P.mleaf), st,
             P.d_mmj, P.d_mma, o.first, (const double*)ws, op);
      break;
    case OP_GTALL:
      launch(L, k_gemm_tall, o.count, NT_MM, 0, st, P.d_gj, P.d_gt, o.first, op);
      break;
    case OP_GRED:
      launch(L, k_gemm_red, o.count, NT_MM, 0, st, P.d_gj, P.d_gr, o.first, ws, cnt, op);
      break;
    case OP_LGATHER:
      launch(L, k_leaf_gather, o.count, NT_MM, 0, st, P.d_lj, o.first, (int)o.n);
      break;
    case OP_LPANEL:
    case OP_LUPDATE:
      launch(L, k_leaf_step, o.count, NT_LEAF, LEAF_LDS, st, P.d_lj, o.first, (int)o.n, o.a1);
      break;
    case OP_LSCATTER:
      launch(L, k_leaf_scatter, o.count, NT_MM, 0, st, P.d_lj, o.first, (int)o.n);
      break;
    case OP_FILL:
      launch(L, k_fill_items, o.count, 256, 0, st, P.d_vj, o.first);
      break;
    case OP_NORMALIZE:
      launch(L, k_normalize, o.count, 1024, 0, st, P.d_vj, o.first);
      break;
    case OP_SETSCAL:
      launch(L, k_set_scal, (o.count + 63) / 64, 64, 0, st, P.d_vj, o.first, o.count);
      break;
    case OP_ROWS:
      launch(L, k_rows, o.count, NT_MM, 0, st, P.d_rj, o.first);
      break;
    case OP_TRSM:
      if (o.xs >= 0) {
        if (op.s > 0)
          launch(L, k_leaf_trsm, op.s, NT_MM, 0, st, o.p0, o.a0, o.a1 > 0 ? o.a1 : o.a0, op.p[o.xs] + o.xoff,
                 op.ld[o.xs], op.s);
      } else {
        launch(L, k_leaf_trsm, o.count, NT_MM, 0, st, o.p0, o.a0, o.a0, o.p1, (int)o.n, o.count);
      }
      break;
  }
}

// Issue a plan.  With `aux` set, lane-1 ops go to `aux`, forked from and joined
// back into `st` with events ev[n_events] and ev[n_events + 1]; SIGNAL/WAIT ops
// become event records and waits.  Without it every op runs on `st` in list
// order, which is a valid serial order of the same work.
hodlr_status run_ops(const Plan& P, const Work& W, hipStream_t st, hipStream_t aux = nullptr,
                     const hipEvent_t* ev = nullptr, const Opnd& op = Opnd{}) {
  TRY(set_attrs());
  if (aux != nullptr) {
    HIPCHK(hipEventRecord(ev[P.n_events], st));
    HIPCHK(hipStreamWaitEvent(aux, ev[P.n_events], 0));
  }
  for (const Op& o : P.ops) {
    hipStream_t s = (aux != nullptr && o.lane == 1) ? aux : st;
    if (o.type == OP_SIGNAL) {
      if (aux != nullptr) HIPCHK(hipEventRecord(ev[o.a0], s));
    } else if (o.type == OP_WAIT) {
      if (aux != nullptr) HIPCHK(hipStreamWaitEvent(s, ev[o.a0], 0));
    } else {
      run_op(P, W, o, s, Launch(), op);
    }
  }
  if (aux != nullptr) {
    HIPCHK(hipEventRecord(ev[P.n_events + 1], aux));
    HIPCHK(hipStreamWaitEvent(st, ev[P.n_events + 1], 0));
  }
  HIPCHK(hipGetLastError());
  return HODLR_OK;
}

// a launch sequence kept by a handle and replayed with new operands
struct CachedPlan {
  Plan P;
  DMem mem;  // the descriptors
};

// zero-filled per-call counters (a kernel, so that a caller may capture the call)
hodlr_status zero_counters(int* cnt, int n, hipStream_t st) {
  if (n <= 0) return HODLR_OK;
  k_zero_i32<<<(n + 255) / 256, 256, 0, st>>>(cnt, n);
  HIPCHK(hipGetLastError());
  return HODLR_OK;
}

}  // namespace
}  // namespace hqh

using namespace hqh;

// ------------------------------------------------------------------ handles
// A HODLR matrix on the device, or a borrowed view of one factor of a QR
// (hodlr_qr_factor): then the leaves are unit lower (Y) or upper (T, R)
// triangular and only one family of off-diagonal blocks is present.
struct hodlr_s {
  Tree t;
  int cap = 0;
  DMem mem;
  LeafSet leaves;
  BlockSet up, lo;
  int* ranks = nullptr;  // [0,2^L) up, [2^L, 2^(L+1)) lo
  int* rank_up_dev = nullptr;
  int* rank_lo_dev = nullptr;
  int leaf_kind = LEAF_FULL;
  bool has_up = true, has_lo = true;
  bool borrowed = false;
  std::mutex mu;                          // guards the cached product sequences
  std::unique_ptr<CachedPlan> mmplan[2];  // Z = A X, Z = A^T X
  HView view() const {
    return HView{t.L, has_up ? up.dview : nullptr, has_lo ? lo.dview : nullptr, leaves.dview, leaf_kind};
  }
};

namespace hqh {
namespace {

// The launch schedule of one batch of factorisations that share a tree: one
// plan whose every launch carries the jobs of all of them, the workspace of
// that plan, the second stream and its events, and the captured graph.
struct Batch {
  Plan plan;
  Work work;  // ws and counters of the plan (per-factorisation words live in each factor)
  DMem mem;
  hipGraphExec_t graph = nullptr;
  hipStream_t aux = nullptr;       // stream of the T-factor lane
  std::vector<hipEvent_t> events;  // plan events + fork + join
  int64_t n_launch = 0;
  int size = 0;
  std::vector<hodlr_qr_s*> members;  // the factorisations the plan writes, in job order
  bool merged = false;               // several shapes in one sequence: serial order only
  ~Batch() {
    if (graph) (void)hipGraphExecDestroy(graph);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    if (aux) (void)hipStreamDestroy(aux);
  }
};

// rank-log sites (the first field of a key)
enum : int { RL_ORTH = 0, RL_S = 1, RL_A12 = 2, RL_UPDATE = 3, RL_T = 4, RL_E = 5 };
using LogKey = std::array<int, 5>;

}  // namespace
}  // namespace hqh

struct hodlr_qr_s {
  Tree t;   // A's partition (rows and columns)
  Tree tc;  // the square partition of the columns (T; R on its pivot rows)
  int cap = 0;
  DMem mem;
  LeafSet leaves, tleaves;
  BlockSet up, lo, tup;
  // rectangular A (Sec. 6): Y's upper blocks (left factor E_L over the rows of
  // the first child, zero on its pivot rows; right factor E_R, then Y~_E)
  BlockSet yup;
  // R on the pivot rows (the first n_j rows of each leaf) as a square HODLR view
  // of the storage of A's leaves and upper blocks
  BlockSet rset;
  LeafSet rleaves;
  int* ranks = nullptr;  // up | lo | t | yup | scalars
  double anorm = 0, eps = 0, tauA = 0, tauT = 0;
  double anorm_in = 0;     // |A|_2 given by the caller (<= 0: estimated)
  double* scal = nullptr;  // device: |A|_2, eps*|A|_2, eps
  Work work;               // error word, flop counters, leaf workspace
  // temporaries of the node steps (n x cap each)
  double *SL = nullptr, *SR = nullptr, *SLt = nullptr, *Z1 = nullptr, *Z2 = nullptr, *Z4 = nullptr,
         *SRW = nullptr, *TL = nullptr, *TR = nullptr, *Z5 = nullptr, *Wm = nullptr, *Mg = nullptr;
  double *X1 = nullptr, *X2 = nullptr;   // vectors of the norm estimate (n + rows, n)
  // rectangular: pivot and free rows of [U12 | Y_A11 S_L] gathered, E_L compact, Y_A11^T E_L
  double *PU = nullptr, *PZ = nullptr, *FU = nullptr, *FZ = nullptr, *FE = nullptr, *Z6 = nullptr;
  int* pivrun = nullptr;  // device: per leaf (first row, first column, n_j) of its pivot rows
  std::shared_ptr<Batch> batch;          // the schedule (dropped once the factors are final)
  int64_t n_launch = 0, n_trunc = 0;     // counts of that schedule per factorisation
  // rank log: (input width, kept rank) per recompression, keys on the host
  int* rlog = nullptr;
  int64_t nlog_cap = 0;
  std::vector<LogKey> logkeys;
  // cached launch sequences of apply Q (Q X, Q^T X) and of the back substitution
  std::unique_ptr<CachedPlan> applyp[2], solvep;
  // borrowed views of the factors (hodlr_qr_factor)
  std::unique_ptr<hodlr_s> vY, vT, vR;
  bool rect() const { return t.rect(); }
  HView view_gen() const { return HView{t.L, up.dview, lo.dview, leaves.dview, LEAF_FULL}; }
  HView view_y() const {
    return HView{t.L, rect() ? yup.dview : nullptr, lo.dview, leaves.dview, LEAF_UNIT_LOWER};
  }
  HView view_t() const { return HView{t.L, tup.dview, nullptr, tleaves.dview, LEAF_UPPER}; }
  HView view_r() const { return HView{t.L, rset.dview, nullptr, rleaves.dview, LEAF_UPPER}; }
  int* rank_up(int v) { return ranks + v; }
  int* rank_lo(int v) { return ranks + (1 << t.L) + v; }
  int* rank_t(int v) { return ranks + 2 * (1 << t.L) + v; }
  int* rank_e(int v) { return ranks + 3 * (1 << t.L) + v; }
  int* rank_s() { return ranks + 4 * (1 << t.L); }
};

namespace hqh {
namespace {

MmSpec mmspec(HView M, bool up, bool lo, int v, int trans, const double* X, int ldX, const int* s_dev,
              double* Z, int ldZ, double alpha, double beta, int tri, int s = 0, double* flops = nullptr) {
  MmSpec m;
  m.M = M;
  m.has_up = up;
  m.has_lo = lo;
  m.v = v;
  m.trans = trans;
  m.X = X;
  m.ldX = ldX;
  m.s = s;
  m.s_dev = s_dev;
  m.Z = Z;
  m.ldZ = ldZ;
  m.alpha = alpha;
  m.beta = beta;
  m.tri = tri;
  m.flops = flops;
  return m;
}

GemmJob gjob(int ta, int tb, int M, const int* Md, int N, const int* Nd, int K, const int* Kd,
             const double* A, int lda, const double* B, int ldb, double* C, int ldc, double alpha,
             double beta, int fc, double* flops = nullptr) {
  GemmJob J{};
  J.ta = ta;
  J.tb = tb;
  J.M = M;
  J.N = N;
  J.K = K;
  J.Md = Md;
  J.Nd = Nd;
  J.Kd = Kd;
  J.A = A;
  J.lda = lda;
  J.B = B;
  J.ldb = ldb;
  J.C = C;
  J.ldc = ldc;
  J.alpha = alpha;
  J.beta = beta;
  J.fc = fc;
  J.as_ = J.bs_ = J.cs_ = -1;
  J.flops = flops;
  return J;
}

// number of recompressions of one factorisation (the rank log's length):
// one per lower block (orthogonalisation), and at each internal node the S~
// chain (1 + q), R's upper block, two per internal node of the right subtree
// (-_H) and the T~12 chain (max(1, q)), q = the node's row groups
int64_t count_truncs(const Tree& t) {
  int64_t c = t.nleaf() - 1;
  struct R {
    const Tree& t;
    int64_t& c;
    void go(int v, int q) {
      if (t.is_leaf(v)) return;
      const int Rc = 2 * v + 1;
      const int e = t.mr(2 * v) > t.m(2 * v) ? 1 : 0;  // E group (rectangular)
      c += (1 + q) + 1 + e + 2 * (int64_t)((t.subtree_size(Rc) - 1) / 2) + std::max(1, q + e);
      go(2 * v, q + 1);
      go(Rc, q + e);
    }
  } r{t, c};
  r.go(1, 0);
  return c;
}

// Builds the launch list of a batch of factorisations with the same tree
// (Algorithm hQR, depth first): every step issues one launch holding the jobs
// of all factors of the batch, so the factors progress in lockstep.
struct QRBuilder {
  std::vector<hodlr_qr_s*> Fs;
  Plan& P;
  const Tree& t;   // A's partition
  const Tree& tc;  // the square partition of the columns
  int cap;
  int plant = 0;  // hazard-checker self test: see hodlr_plan_check
  QRBuilder(const std::vector<hodlr_qr_s*>& fs, Plan& plan)
      : Fs(fs), P(plan), t(fs[0]->t), tc(fs[0]->tc), cap(fs[0]->cap) {}

  // Row groups of the stacked columns.  A group g > 0 is the lower block of
  // node g (rows below it, right factor over the columns of 2g); g < 0 is the
  // E group of node -g (free rows of its first child, right factor over the
  // columns of its second child; rectangular matrices only).
  const HBlk& gblk(hodlr_qr_s& F, int g) { return g > 0 ? F.lo.hview[g] : F.yup.hview[-g]; }
  int gchild(int g) { return g > 0 ? 2 * g : 2 * (-g) + 1; }
  int* grank(hodlr_qr_s& F, int g) { return g > 0 ? F.rank_lo(g) : F.rank_e(-g); }
  // right factor slice of group g over node x's columns
  double* gslice(hodlr_qr_s& F, int g, int x) { return gblk(F, g).V + (t.lo[x] - t.lo[gchild(g)]); }
  int gld(int g) { return (int)t.m(gchild(g)); }

  void leaf(int v, const std::vector<int>& groups) {
    const int j = v - t.nleaf();
    const int first = (int)P.lj.size();
    const int m = (int)t.m(v), np = (m + NB - 1) / NB;
    for (hodlr_qr_s* Fp : Fs) {
      hodlr_qr_s& F = *Fp;
      LeafJob J{};
      J.D = F.leaves.hview[j].D;
      J.m = m;
      J.mr = (int)t.mr(v);
      J.Tleaf = F.tleaves.hview[j].D;
      J.ws = F.work.leaf;
      J.err = F.work.err;
      J.flops = F.work.fc;
      J.ngroups = (int)groups.size();
      for (size_t i = 0; i < groups.size(); ++i) {
        const int g = groups[i];
        J.g[i] = LeafGroup{gblk(F, g).V, gld(g), (int)(t.lo[v] - t.lo[gchild(g)]), grank(F, g)};
      }
      P.lj.push_back(J);
    }
    const int nj = (int)Fs.size();
    auto leafop = [&](int type, int nper, int p) {
      Op o{type, first, nj * nper, 0, p};
      o.n = nper;
      P.push(o);
    };
    leafop(OP_LGATHER, m, 0);
    leafop(OP_LPANEL, 1, -1);  // panel 0
    for (int p = 0; p <= np; ++p) {
      const int nstrip = p < np ? np - p - 1 : 0, ngram = p < np ? p : 0, ntile = p >= 1 ? p - 1 : 0;
      const int cnt = nstrip + ngram + ntile;
      if (cnt > 0) leafop(OP_LUPDATE, cnt, p);
    }
    leafop(OP_LSCATTER, m, 0);
  }

  // Row runs of node x's pivot rows (the first n_j rows of each of its leaves,
  // packed in column order) and free rows (the others, packed in row order):
  // (row within x, row in the packed array, length).
  void runs(int x, std::vector<std::array<int, 3>>& piv, std::vector<std::array<int, 3>>& fre) {
    std::vector<int> lv;
    t.subtree_leaves(x, lv);
    int fpos = 0;
    for (int j : lv) {
      const int h = t.nleaf() + j;
      const int r = (int)(t.rlo[h] - t.rlo[x]), c = (int)(t.lo[h] - t.lo[x]);
      const int nj = (int)t.m(h), mj = (int)t.mr(h);
      piv.push_back({r, c, nj});
      if (mj > nj) {
        fre.push_back({r + nj, fpos, mj - nj});
        fpos += mj - nj;
      }
    }
  }

  TrSpec trspec(hodlr_qr_s& F, Seg l0, Seg l1, Seg r0, Seg r1, int mL, int mR, const double* tau,
                double* oL, double* oR, int ldL, int ldR, int* orank, int fc, const LogKey& key, int flags = 0) {
    TrSpec s;
    s.seg[0][0] = l0;
    s.seg[0][1] = l1;
    s.seg[1][0] = r0;
    s.seg[1][1] = r1;
    s.m[0] = mL;
    s.m[1] = mR;
    s.tau = tau;
    s.flags = flags;
    s.out[0] = oL;
    s.out[1] = oR;
    s.ldout[0] = ldL;
    s.ldout[1] = ldR;
    s.cap = cap;
    s.out_rank = orank;
    s.fc = fc;
    s.err = F.work.err;
    s.flops = F.work.fc;
    const int64_t slot = (int64_t)F.logkeys.size();
    s.log = slot < F.nlog_cap ? F.rlog + 2 * slot : nullptr;
    F.logkeys.push_back(key);
    return s;
  }

  // Ops of the subtree at v.  The T-factor steps (T~12, T12) of every node run
  // on lane 1 beside the main chain: they wait for the node's right subtree and
  // are only read again by the parent's S = T1^T S~ (main chain: it waits for
  // the returned event) or by the parent's own T steps (later on lane 1).
  // Returns the event signalled once T of the subtree is complete, -1 for a leaf.
  // Sizes: n* are columns, m* rows (equal for a square matrix).  A rectangular
  // matrix (Sec. 6) whose first child has free rows also gets an E group here.
  int node(int v, const std::vector<int>& groups) {
    if (t.is_leaf(v)) {
      leaf(v, groups);
      return -1;
    }
    const int Lc = 2 * v, Rc = 2 * v + 1;
    const int nL = (int)t.m(Lc), nR = (int)t.m(Rc);
    const int mL = (int)t.mr(Lc), mR = (int)t.mr(Rc);
    const bool has_e = t.mr(Lc) > t.m(Lc);  // free rows in the first child
    const int fL = mL - nL;
    const int klo = (int)t.lo[v], khi = (int)t.hi[v];
    // first block column: hQR(A11, A21, [B_R1; C1])
    std::vector<int> gl;
    gl.push_back(v);
    gl.insert(gl.end(), groups.begin(), groups.end());
    const int evL = node(Lc, gl);
    std::vector<MmSpec> mms;
    std::vector<TrSpec> trs;
    // S~ terms: Z1 = Y_A11^T U12 and Z2 = A22^T U21 (one launch pair)
    for (hodlr_qr_s* Fp : Fs) {
      hodlr_qr_s& F = *Fp;
      const HBlk& A12 = F.up.hview[v];
      const HBlk& A21 = F.lo.hview[v];
      MmSpec a = mmspec(F.view_y(), F.rect(), true, Lc, 1, A12.U, mL, F.rank_up(v), F.Z1, nL, 1.0, 0.0, 1, 0,
                        F.work.fc);
      MmSpec b = mmspec(F.view_gen(), true, true, Rc, 1, A21.U, mR, F.rank_lo(v), F.Z2, nR, 1.0, 0.0, 0, 0,
                        F.work.fc);
      a.rld = b.rld = cap;
      mms.push_back(a);
      mms.push_back(b);
    }
    P.mm(t, mms);
    // S~ = T(Y_A11^T A12 + Y_A21^T A22 + sum over groups), term by term: one
    // chain of recompressions
    std::vector<std::vector<TrSpec>> chain(1);
    for (hodlr_qr_s* Fp : Fs) {
      hodlr_qr_s& F = *Fp;
      const HBlk& A12 = F.up.hview[v];
      const HBlk& A21 = F.lo.hview[v];
      int* k12 = F.rank_up(v);
      int* k21 = F.rank_lo(v);
      chain[0].push_back(trspec(F, mkseg(F.Z1, nL, k12), mkseg(A21.V, nL, k21), mkseg(A12.V, nR, k12),
                                mkseg(F.Z2, nR, k21), nL, nR, F.scal + 1, F.SL, F.SR, nL, nR, F.rank_s(),
                                FC_TRUNC, LogKey{RL_S, klo, khi, 0, 0}));
    }
    for (size_t gi = 0; gi < groups.size(); ++gi) {
      const int g = groups[gi];
      chain.emplace_back();
      for (hodlr_qr_s* Fp : Fs) {
        hodlr_qr_s& F = *Fp;
        int* rS = F.rank_s();
        chain.back().push_back(trspec(F, mkseg(F.SL, nL, rS), mkseg(gslice(F, g, Lc), gld(g), grank(F, g)),
                                      mkseg(F.SR, nR, rS), mkseg(gslice(F, g, Rc), gld(g), grank(F, g)), nL,
                                      nR, F.scal + 1, F.SL, F.SR, nL, nR, rS, FC_TRUNC,
                                      LogKey{RL_S, klo, khi, 1 + (int)gi, 0}));
      }
    }
    P.trunc_chain(chain);
    // S = T1^T S~  (left factor only); T1 must be complete
    if (evL >= 0) P.wait(evL);
    mms.clear();
    for (hodlr_qr_s* Fp : Fs) {
      hodlr_qr_s& F = *Fp;
      MmSpec a = mmspec(F.view_t(), true, false, Lc, 1, F.SL, nL, F.rank_s(), F.SLt, nL, 1.0, 0.0, 1, 0,
                        F.work.fc);
      a.rld = cap;
      mms.push_back(a);
    }
    P.mm(tc, mms);
    // Y_A11 S_L for the new upper block
    mms.clear();
    for (hodlr_qr_s* Fp : Fs) {
      hodlr_qr_s& F = *Fp;
      MmSpec a = mmspec(F.view_y(), F.rect(), true, Lc, 0, F.SLt, nL, F.rank_s(), F.Z4, mL, 1.0, 0.0, 1, 0,
                        F.work.fc);
      a.rld = cap;
      mms.push_back(a);
    }
    P.mm(t, mms);
    // W = Y~_B21 S_L (k21 x s) and M_g = S_L^T Y_C1g^T (s x k_g)
    {
      std::vector<GSpec> red;
      for (hodlr_qr_s* Fp : Fs) {
        hodlr_qr_s& F = *Fp;
        const HBlk& A21 = F.lo.hview[v];
        int* rS = F.rank_s();
        red.push_back(GSpec{gjob(1, 0, 0, F.rank_lo(v), 0, rS, nL, nullptr, A21.V, nL, F.SLt, nL, F.Wm, KCAP,
                                 1.0, 0.0, FC_DENSE, F.work.fc),
                            KCAP, KCAP, nL});
        for (size_t i = 0; i < groups.size(); ++i) {
          const int g = groups[i];
          red.push_back(GSpec{gjob(1, 0, 0, rS, 0, grank(F, g), nL, nullptr, F.SLt, nL, gslice(F, g, Lc),
                                   gld(g), F.Mg + i * KCAP * KCAP, KCAP, 1.0, 0.0, FC_DENSE, F.work.fc),
                              KCAP, KCAP, nL});
        }
      }
      P.gemm_red(red);
    }
    // SRW = S_R W^T (nR x k21);  C_2g -= S_R M_g  (B^_R2 and C^2 of the update)
    {
      std::vector<GSpec> tall;
      for (hodlr_qr_s* Fp : Fs) {
        hodlr_qr_s& F = *Fp;
        int* rS = F.rank_s();
        tall.push_back(GSpec{gjob(0, 1, nR, nullptr, 0, F.rank_lo(v), 0, rS, F.SR, nR, F.Wm, KCAP, F.SRW, nR,
                                  1.0, 0.0, FC_DENSE, F.work.fc),
                             nR, cap, 0});
        for (size_t i = 0; i < groups.size(); ++i) {
          const int g = groups[i];
          tall.push_back(GSpec{gjob(0, 0, nR, nullptr, 0, grank(F, g), 0, rS, F.SR, nR,
                                    F.Mg + i * KCAP * KCAP, KCAP, gslice(F, g, Rc), gld(g), -1.0, 1.0,
                                    FC_DENSE, F.work.fc),
                               nR, cap, 0});
        }
      }
      P.gemm_tall(tall);
    }
    // Rectangular: A^12 = U12 V12^T - (Y_A11 S_L) S_R^T splits by rows.  Its
    // free rows are compressed to E = E_L E_R (E_L into Y's upper block of v,
    // E_R joins the second block column's groups); its pivot rows become R's
    // upper block (below).
    std::vector<std::array<int, 3>> prun, frun;
    if (has_e) {
      runs(Lc, prun, frun);
      std::vector<RowJob> g1;
      for (hodlr_qr_s* Fp : Fs) {
        hodlr_qr_s& F = *Fp;
        const HBlk& A12 = F.up.hview[v];
        for (const auto& r : prun) {
          g1.push_back(RowJob{A12.U, mL, F.PU, nL, r[0], r[1], r[2], F.rank_up(v), 0});
          g1.push_back(RowJob{F.Z4, mL, F.PZ, nL, r[0], r[1], r[2], F.rank_s(), 0});
        }
        for (const auto& r : frun) {
          g1.push_back(RowJob{A12.U, mL, F.FU, fL, r[0], r[1], r[2], F.rank_up(v), 0});
          g1.push_back(RowJob{F.Z4, mL, F.FZ, fL, r[0], r[1], r[2], F.rank_s(), 0});
        }
      }
      rows(g1);
      trs.clear();
      for (hodlr_qr_s* Fp : Fs) {
        hodlr_qr_s& F = *Fp;
        const HBlk& A12 = F.up.hview[v];
        const HBlk& E = F.yup.hview[v];
        int* k12 = F.rank_up(v);
        int* rS = F.rank_s();
        trs.push_back(trspec(F, mkseg(F.FU, fL, k12), mkseg(F.FZ, fL, rS, -1.0), mkseg(A12.V, nR, k12),
                             mkseg(F.SR, nR, rS), fL, nR, F.scal + 1, F.FE, E.V, fL, nR, F.rank_e(v), FC_TRUNC,
                             LogKey{RL_E, klo, khi, 0, 0}));
      }
      P.trunc(trs);
      std::vector<RowJob> g2;
      for (hodlr_qr_s* Fp : Fs) {
        hodlr_qr_s& F = *Fp;
        const HBlk& E = F.yup.hview[v];
        for (const auto& r : frun) g2.push_back(RowJob{F.FE, fL, E.U, mL, r[1], r[0], r[2], F.rank_e(v), 0});
      }
      rows(g2);
    }
    // A^12 = T([U12 | -Y_A11 S_L] [V12 | S_R]^T) (rectangular: its pivot rows)
    // and A^22 = A22 -_H U21 W S_R^T: every off-diagonal block of the trailing
    // sub-HODLR, one batch
    {
      std::vector<int> sub;
      t.subtree_internal(Rc, sub);
      std::vector<TrSpec> sp;
      std::vector<int> leaves;
      t.subtree_leaves(Rc, leaves);
      std::vector<GSpec> lu;
      for (hodlr_qr_s* Fp : Fs) {
        hodlr_qr_s& F = *Fp;
        const HBlk& A12 = F.up.hview[v];
        const HBlk& A21 = F.lo.hview[v];
        int* k12 = F.rank_up(v);
        int* k21 = F.rank_lo(v);
        int* rS = F.rank_s();
        if (has_e)
          sp.push_back(trspec(F, mkseg(F.PU, nL, k12), mkseg(F.PZ, nL, rS, -1.0), mkseg(A12.V, nR, k12),
                              mkseg(F.SR, nR, rS), nL, nR, F.scal + 1, A12.U, A12.V, mL, nR, k12, FC_TRUNC,
                              LogKey{RL_A12, klo, khi, 0, 0}));
        else
          sp.push_back(trspec(F, mkseg(A12.U, mL, k12), mkseg(F.Z4, mL, rS, -1.0), mkseg(A12.V, nR, k12),
                              mkseg(F.SR, nR, rS), mL, nR, F.scal + 1, A12.U, A12.V, mL, nR, k12, FC_TRUNC,
                              LogKey{RL_A12, klo, khi, 0, 0}));
        for (int u : sub) {
          for (int kind = 0; kind < 2; ++kind) {
            const HBlk& b = kind == 0 ? F.up.hview[u] : F.lo.hview[u];
            int* kb = kind == 0 ? F.rank_up(u) : F.rank_lo(u);
            const int64_t ri = b.r0 - t.rlo[Rc], cj = b.c0 - t.lo[Rc];
            sp.push_back(trspec(F, mkseg(b.U, b.ldU, kb), mkseg(A21.U + ri, mR, k21), mkseg(b.V, b.ldV, kb),
                                mkseg(F.SRW + cj, nR, k21, -1.0), b.rows, b.cols, F.scal + 1, b.U, b.V,
                                b.ldU, b.ldV, kb, FC_TRUNC, LogKey{RL_UPDATE, klo, khi, (int)b.r0, (int)b.c0}));
          }
        }
        // leaves of the trailing part: D -= U21(I) (S_R W^T)(J)^T
        for (int j : leaves) {
          const int lv = t.nleaf() + j;
          const int mj = (int)t.mr(lv), nj = (int)t.m(lv);
          const int64_t ri = t.rlo[lv] - t.rlo[Rc], ci = t.lo[lv] - t.lo[Rc];
          lu.push_back(GSpec{gjob(0, 1, mj, nullptr, nj, nullptr, 0, k21, A21.U + ri, mR, F.SRW + ci, nR,
                                  F.leaves.hview[j].D, mj, -1.0, 1.0, FC_UPDATE, F.work.fc),
                             mj, nj, 0});
        }
      }
      P.trunc(sp);
      P.gemm_tall(lu);
    }
    // second block column: hQR(A^22, [], [B^_R2; C^2] (; E_R))
    std::vector<int> gr = groups;
    if (has_e) gr.push_back(-v);
    node(Rc, gr);
    const int evM = P.signal();
    P.lane = 1;
    P.wait(evM);
    // T~12 = T_eps(Y_1^T Y_2): terms over the rows top down: (rectangular) the
    // free rows of the first child, Y_A11^T E_L Y~_E; Y_A21^T Y_A22; the groups
    mms.clear();
    for (hodlr_qr_s* Fp : Fs) {
      hodlr_qr_s& F = *Fp;
      MmSpec a = mmspec(F.view_y(), F.rect(), true, Rc, 1, F.lo.hview[v].U, mR, F.rank_lo(v), F.Z5, nR, 1.0,
                        0.0, 1, 0, F.work.fc);
      a.rld = cap;
      mms.push_back(a);
      if (has_e) {
        MmSpec e = mmspec(F.view_y(), true, true, Lc, 1, F.yup.hview[v].U, mL, F.rank_e(v), F.Z6, nL, 1.0, 0.0,
                          1, 0, F.work.fc);
        e.rld = cap;
        mms.push_back(e);
      }
    }
    P.mm(t, mms);
    struct Term {
      Seg l, r;
    };
    const size_t nterm = (has_e ? 1 : 0) + 1 + groups.size();
    const size_t nchain = std::max<size_t>(1, nterm - 1);
    std::vector<std::vector<TrSpec>> tchain;
    for (size_t i = 0; i < nchain; ++i) {
      std::vector<TrSpec>& trs = tchain.emplace_back();
      for (hodlr_qr_s* Fp : Fs) {
        hodlr_qr_s& F = *Fp;
        const HBlk& A21 = F.lo.hview[v];
        int* k21 = F.rank_lo(v);
        int* rt = F.rank_t(v);
        std::vector<Term> terms;
        if (has_e)
          terms.push_back(Term{mkseg(F.Z6, nL, F.rank_e(v)), mkseg(F.yup.hview[v].V, nR, F.rank_e(v))});
        terms.push_back(Term{mkseg(A21.V, nL, k21), mkseg(F.Z5, nR, k21)});
        for (int g : groups)
          terms.push_back(Term{mkseg(gslice(F, g, Lc), gld(g), grank(F, g)),
                               mkseg(gslice(F, g, Rc), gld(g), grank(F, g))});
        // self test of the hazard checker: node 2's first T~12 recompression
        // writes into S~'s buffer, which the root's main chain uses meanwhile
        double* outL = (plant && v == 2 && i == 0) ? F.SL : F.TL;
        const Seg l0 = i == 0 ? terms[0].l : mkseg(F.TL, nL, rt);
        const Seg r0 = i == 0 ? terms[0].r : mkseg(F.TR, nR, rt);
        const size_t nx = i == 0 ? 1 : i + 1;  // the term added by this recompression
        const LogKey key{RL_T, klo, khi, (int)i, 0};
        if (nx >= terms.size())
          trs.push_back(trspec(F, l0, noseg(), r0, noseg(), nL, nR, F.scal + 2, outL, F.TR, nL, nR, rt, FC_TRUNC,
                               key));
        else
          trs.push_back(trspec(F, l0, terms[nx].l, r0, terms[nx].r, nL, nR, F.scal + 2, outL, F.TR, nL, nR, rt,
                               FC_TRUNC, key));
      }
    }
    P.trunc_chain(tchain);
    // T12 = -T1 T~12 T2 = (-T1 T~_L)(T2^T T~_R)^T
    mms.clear();
    for (hodlr_qr_s* Fp : Fs) {
      hodlr_qr_s& F = *Fp;
      const HBlk& T12 = F.tup.hview[v];
      int* rt = F.rank_t(v);
      MmSpec a = mmspec(F.view_t(), true, false, Lc, 0, F.TL, nL, rt, T12.U, nL, -1.0, 0.0, 1, 0, F.work.fc);
      MmSpec b = mmspec(F.view_t(), true, false, Rc, 1, F.TR, nR, rt, T12.V, nR, 1.0, 0.0, 1, 0, F.work.fc);
      a.rld = b.rld = cap;
      mms.push_back(a);
      mms.push_back(b);
    }
    P.mm(tc, mms);
    const int evT = P.signal();
    P.lane = 0;
    return evT;
  }

  void rows(const std::vector<RowJob>& items) {
    const int first = (int)P.rj.size();
    P.rj.insert(P.rj.end(), items.begin(), items.end());
    P.push(Op{OP_ROWS, first, (int)items.size()});
  }

  void build() {
    // make every lower block left-orthogonal (the B_L of each block column)
    std::vector<TrSpec> orth;
    for (hodlr_qr_s* Fp : Fs) {
      hodlr_qr_s& F = *Fp;
      for (int v = 1; v < t.nleaf(); ++v) {
        const HBlk& b = F.lo.hview[v];
        orth.push_back(trspec(F, mkseg(b.U, b.ldU, F.rank_lo(v)), noseg(), mkseg(b.V, b.ldV, F.rank_lo(v)),
                              noseg(), b.rows, b.cols, F.scal + 2, b.U, b.V, b.ldU, b.ldV, F.rank_lo(v),
                              FC_ORTH, LogKey{RL_ORTH, (int)b.r0, (int)b.c0, 0, 0}, TR_ORTH));
      }
    }
    P.trunc(orth);
    node(1, {});
  }
};

// One power-iteration estimate of |M|_2 per item (iters steps on M^T M from
// x0 = 1/sqrt(n)), all items in the same launches; writes each result to
// its out (device).  x, z: device vectors of the columns' length per item,
// y of the rows' length.
struct NormItem {
  HView V;
  int rld;
  double *x, *y, *z, *out;
  double* flops;
};

void plan_norm2(Plan& P, const Tree& t, const std::vector<NormItem>& items, int iters) {
  const int64_t n = t.n, nr = t.nr;  // x, z: n entries; y = M x: nr entries
  std::vector<VecJob> fill, norm, last;
  for (const NormItem& it : items) {
    fill.push_back(VecJob{nullptr, it.x, n, nullptr, 1.0 / std::sqrt((double)n), 0.0});
    norm.push_back(VecJob{it.z, it.x, n, nullptr, 0.0, 0.0});
    last.push_back(VecJob{it.y, nullptr, nr, it.out, 0.0, 0.0});
  }
  P.vec(OP_FILL, fill);
  std::vector<MmSpec> a, b;
  for (const NormItem& it : items) {
    MmSpec sa = mmspec(it.V, true, true, 1, 0, it.x, (int)n, nullptr, it.y, (int)nr, 1.0, 0.0, 0, 1, it.flops);
    MmSpec sb = mmspec(it.V, true, true, 1, 1, it.y, (int)nr, nullptr, it.z, (int)n, 1.0, 0.0, 0, 1, it.flops);
    sa.fc = sb.fc = FC_NORM;
    sa.rld = sb.rld = it.rld;
    a.push_back(sa);
    b.push_back(sb);
  }
  for (int i = 0; i < iters; ++i) {
    P.mm(t, a);
    P.mm(t, b);
    P.vec(OP_NORMALIZE, norm);
  }
  P.mm(t, a);
  P.vec(OP_NORMALIZE, last);
}

hodlr_status check_finite(const double* p, size_t n, const char* what) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return fail(HODLR_ENONFINITE, std::string("non-finite value in ") + what);
  return HODLR_OK;
}

// copies A's storage into F's and resets ranks / flop counters
hodlr_status reset_factor(hodlr_qr_s& F, const hodlr_s& A, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(F.leaves.D, A.leaves.D, F.leaves.size * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(F.up.U, A.up.U, F.up.usz * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(F.up.V, A.up.V, F.up.vsz * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(F.lo.U, A.lo.U, F.lo.usz * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(F.lo.V, A.lo.V, F.lo.vsz * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(F.ranks, A.ranks, 2 * (size_t)(1 << A.t.L) * sizeof(int), hipMemcpyDeviceToDevice, st));
  k_fill<<<(FC_SIZE + 255) / 256, 256, 0, st>>>(F.work.fc, FC_SIZE, 0.0);
  k_zero_i32<<<1, 64, 0, st>>>(F.work.err, 4);  // a refactorisation starts without the last run's flags
  return HODLR_OK;
}

// the borrowed views of F's factors (hodlr_qr_factor)
void make_views(hodlr_qr_s& F) {
  const int nn = 1 << F.t.L;
  auto mk = [&](const LeafSet& L, const BlockSet* up, const BlockSet* lo, int* rup, int* rlo, int kind,
                const Tree& tree) {
    auto V = std::make_unique<hodlr_s>();
    V->t = tree;
    V->cap = F.cap;
    V->leaves = L;
    if (up) V->up = *up;
    if (lo) V->lo = *lo;
    V->has_up = up != nullptr;
    V->has_lo = lo != nullptr;
    V->rank_up_dev = rup;
    V->rank_lo_dev = rlo;
    V->leaf_kind = kind;
    V->borrowed = true;
    return V;
  };
  F.vY = mk(F.leaves, F.rect() ? &F.yup : nullptr, &F.lo, F.rect() ? F.ranks + 3 * nn : nullptr, F.ranks + nn,
            LEAF_UNIT_LOWER, F.t);
  F.vT = mk(F.tleaves, &F.tup, nullptr, F.ranks + 2 * nn, nullptr, LEAF_UPPER, F.tc);
  F.vR = mk(F.rleaves, &F.rset, nullptr, F.ranks, nullptr, LEAF_UPPER, F.tc);
}

// device storage of the factors of A (no schedule yet)
hodlr_status make_storage(const hodlr_s& A, double eps, double anorm, hipStream_t st,
                          std::unique_ptr<hodlr_qr_s>& out) {
  auto F = std::make_unique<hodlr_qr_s>();
  F->mem.zero = true;
  F->mem.stream = st;
  F->t = A.t;
  F->tc = A.t.square();
  F->cap = A.cap;
  F->anorm = anorm;
  F->anorm_in = anorm;
  F->eps = eps;
  F->tauA = eps * anorm;
  F->tauT = eps;
  const Tree& t = F->t;
  if (t.L > MAXGROUPS) return fail(HODLR_EINVAL, "too many levels");
  const Tree& tc = F->tc;
  const int nn = 1 << t.L;
  TRY(F->mem.alloc(&F->scal, 8));
  TRY(F->mem.alloc(&F->ranks, 4 * (size_t)nn + 8));
  TRY(make_leaves(F->mem, t, F->leaves));
  TRY(make_leaves(F->mem, tc, F->tleaves));
  TRY(make_blocks(F->mem, t, F->cap, BK_UP, F->ranks, F->up));
  TRY(make_blocks(F->mem, t, F->cap, BK_LO, F->ranks + nn, F->lo));
  TRY(make_blocks(F->mem, tc, F->cap, BK_UP, F->ranks + 2 * nn, F->tup));
  if (F->rect()) {
    TRY(make_blocks(F->mem, t, F->cap, BK_UP, F->ranks + 3 * nn, F->yup));
    TRY(upload(F->mem, &F->yup.dview, F->yup.hview, st));
  }
  // R's view: upper blocks over the pivot rows of the first child (the first
  // n_L rows of the block's left factor), leaves' top n_j x n_j
  F->rset = F->up;
  for (int v = 1; v < nn; ++v) {
    HBlk& b = F->rset.hview[v];
    b.rows = (int)tc.m(2 * v);
    b.r0 = tc.lo[2 * v];
  }
  F->rleaves = F->leaves;
  for (int j = 0; j < nn; ++j) {
    HLeaf& l = F->rleaves.hview[j];
    l.m = (int)tc.m(nn + j);
    l.r0 = tc.lo[nn + j];
  }
  TRY(upload(F->mem, &F->up.dview, F->up.hview, st));
  TRY(upload(F->mem, &F->lo.dview, F->lo.hview, st));
  TRY(upload(F->mem, &F->tup.dview, F->tup.hview, st));
  TRY(upload(F->mem, &F->leaves.dview, F->leaves.hview, st));
  TRY(upload(F->mem, &F->tleaves.dview, F->tleaves.hview, st));
  TRY(upload(F->mem, &F->rset.dview, F->rset.hview, st));
  TRY(upload(F->mem, &F->rleaves.dview, F->rleaves.hview, st));
  const size_t nc = (size_t)t.n * F->cap;
  for (double** p : {&F->SL, &F->SR, &F->SLt, &F->Z1, &F->Z2, &F->SRW, &F->TL, &F->TR, &F->Z5})
    TRY(F->mem.alloc(p, nc));
  TRY(F->mem.alloc(&F->Z4, (size_t)t.nr * F->cap));
  if (F->rect()) {
    const size_t fc = (size_t)std::max<int64_t>(1, t.nr - t.n) * F->cap;
    for (double** p : {&F->PU, &F->PZ, &F->Z6}) TRY(F->mem.alloc(p, nc));
    for (double** p : {&F->FU, &F->FZ, &F->FE}) TRY(F->mem.alloc(p, fc));
  }
  TRY(F->mem.alloc(&F->Wm, (size_t)KCAP * KCAP));
  TRY(F->mem.alloc(&F->Mg, (size_t)KCAP * KCAP * (t.L + 1)));
  TRY(F->mem.alloc(&F->X1, (size_t)(t.n + t.nr)));
  {
    std::vector<int> pr;
    for (int j = 0; j < nn; ++j) {
      pr.push_back((int)t.rlo[nn + j]);
      pr.push_back((int)t.lo[nn + j]);
      pr.push_back((int)t.m(nn + j));
    }
    TRY(upload(F->mem, &F->pivrun, pr, st));
  }
  TRY(F->mem.alloc(&F->X2, (size_t)t.n));
  F->nlog_cap = count_truncs(t);
  TRY(F->mem.alloc(&F->rlog, 2 * (size_t)F->nlog_cap));
  TRY(ensure_work(F->mem, F->work, 0, 1, true, st));  // error word, flop counters, leaf workspace
  F->mem.zero = false;
  make_views(*F);
  out = std::move(F);
  return HODLR_OK;
}

// the launch list of a batch of factors that share a tree and a capacity (host only)
void build_plan(const std::vector<hodlr_qr_s*>& Fs, Plan& P, int plant = 0) {
  const Tree& t = Fs[0]->t;
  P.wtop = 2 * Fs[0]->cap;
  P.tune = tuning_for(t.n, Fs[0]->cap);
  // thresholds: |A|_2 from the power iteration unless given, then tau_A, tau_T
  std::vector<NormItem> est;
  std::vector<VecJob> sc;
  for (hodlr_qr_s* F : Fs) {
    F->logkeys.clear();
    if (!(F->anorm_in > 0.0))
      est.push_back(NormItem{F->view_gen(), F->cap, F->X1, F->X1 + t.n, F->X2, F->scal, F->work.fc});
    sc.push_back(VecJob{nullptr, F->scal, 3, nullptr, F->eps, F->anorm_in > 0.0 ? F->anorm_in : -1.0});
  }
  if (!est.empty()) plan_norm2(P, t, est, 50);
  P.vec(OP_SETSCAL, sc);
  QRBuilder qb(Fs, P);
  qb.plant = plant;
  qb.build();
}

// upload a batch's plan and allocate its workspace
hodlr_status finish_batch(Batch& B, hipStream_t st) {
  Plan& P = B.plan;
  TRY(P.upload_all(B.mem, st));
  TRY(ensure_work(B.mem, B.work, P.ws_need(), P.cnt_need(), false, st));
  B.n_launch = 0;
  for (const Op& o : P.ops) B.n_launch += op_launches(o) ? 1 : 0;
  return HODLR_OK;
}

// the schedule of a batch of factors that share a tree and a capacity
hodlr_status make_batch(const std::vector<hodlr_qr_s*>& Fs, hipStream_t st, std::shared_ptr<Batch>& out,
                        int plant = 0) {
  auto B = std::make_shared<Batch>();
  B->mem.stream = st;
  B->size = (int)Fs.size();
  B->members = Fs;
  build_plan(Fs, B->plan, plant);
  TRY(finish_batch(*B, st));
  out = std::move(B);
  return HODLR_OK;
}

// Merge the launch lists of several plans (independent factorisations of
// different shapes, one rank capacity) into one list in which a launch carries
// the jobs of every plan that runs the same kernel variant at that point.  Each
// plan's launches keep their order (its serial order: both lanes in list
// order); at every step the plan with the most launches left sets the kernel
// variant, and every plan whose next launch is that variant joins it.  The
// plans' workspaces and counters are laid out one after another.
void merge_plans(const std::vector<const Plan*>& in, Plan& out, bool plant = false) {
  const int G = (int)in.size();
  std::vector<std::vector<int>> seq(G);  // launching ops of each plan
  std::vector<int64_t> wb(G), cb(G);
  int64_t ws = 0, cnt = 0;
  for (int g = 0; g < G; ++g) {
    const Plan& P = *in[g];
    for (int i = 0; i < (int)P.ops.size(); ++i)
      if (op_launches(P.ops[i])) seq[g].push_back(i);
    if (!plant) {
      wb[g] = ws;
      cb[g] = cnt;
      ws += P.ws_need();
      cnt += P.cnt_need();
    } else {  // (self test of the hazard check: every plan at offset 0)
      wb[g] = cb[g] = 0;
      ws = std::max(ws, P.ws_need());
      cnt = std::max(cnt, (int64_t)P.cnt_need());
    }
    out.n_trunc += P.n_trunc;
    out.mleaf = std::max(out.mleaf, P.mleaf);
  }
  out.wtop = in[0]->wtop;
  out.ws_lane[0] = ws;
  out.ws_lane[1] = 0;
  out.cnt_lane[0] = (int)cnt;
  out.cnt_lane[1] = 0;
  // jobs of every plan, rebased once each (their workspace offsets depend on
  // the lane of the op that runs them)
  std::vector<int> trb(G), mmb(G), gjb(G);
  for (int g = 0; g < G; ++g) {
    trb[g] = (int)out.trj.size();
    mmb[g] = (int)out.mmj.size();
    gjb[g] = (int)out.gj.size();
    out.trj.insert(out.trj.end(), in[g]->trj.begin(), in[g]->trj.end());
    out.mmj.insert(out.mmj.end(), in[g]->mmj.begin(), in[g]->mmj.end());
    out.gj.insert(out.gj.end(), in[g]->gj.begin(), in[g]->gj.end());
  }
  std::vector<char> tr_done(out.trj.size(), 0), mm_done(out.mmj.size(), 0);
  auto rebase_tr = [&](int g, int lane, int j) {
    const int jj = trb[g] + j;
    if (tr_done[jj]) return jj;
    tr_done[jj] = 1;
    const int64_t w0 = wb[g] + in[g]->ws_off(lane);
    const int c0 = (int)(cb[g] + in[g]->cnt_off(lane));
    TrJob& J = out.trj[jj];
    J.hdr += w0;
    for (int s = 0; s < 2; ++s) {
      if (J.side[s].p0 > 0) {
        J.side[s].node0 += w0;
        J.side[s].cnt0 += c0;
      }
    }
    J.jcounter += c0;
    return jj;
  };
  auto rebase_mm = [&](int g, int lane, int j) {
    const int jj = mmb[g] + j;
    if (!mm_done[jj]) {
      mm_done[jj] = 1;
      out.mmj[jj].red0 += wb[g] + in[g]->ws_off(lane);
    }
    return jj;
  };
  auto sig = [&](int g, int i) {
    const Op& o = in[g]->ops[i];
    int64_t a = 0, b = 0;
    if (o.type == OP_MMAPPLY) a = o.a1;
    if (o.type == OP_LGATHER || o.type == OP_LPANEL || o.type == OP_LUPDATE || o.type == OP_LSCATTER) {
      a = o.a1;
      b = o.n;
    }
    return std::make_tuple(o.type, a, b);
  };
  std::vector<size_t> h(G, 0);
  std::vector<std::pair<int, int>> last_leaf;  // (plan, first job) of the previous merged leaf launch
  int last_leaf_first = -1;
  while (true) {
    int lead = -1;
    size_t best = 0;
    for (int g = 0; g < G; ++g) {
      const size_t left = seq[g].size() - h[g];
      if (left > best) {
        best = left;
        lead = g;
      }
    }
    if (lead < 0) break;
    const auto s0 = sig(lead, seq[lead][h[lead]]);
    std::vector<int> grp;
    for (int g = 0; g < G; ++g)
      if (h[g] < seq[g].size() && sig(g, seq[g][h[g]]) == s0) grp.push_back(g);
    const Op& o0 = in[lead]->ops[seq[lead][h[lead]]];
    Op m{o0.type};
    m.a0 = o0.a0;
    m.a1 = o0.a1;
    m.n = o0.n;
    switch (o0.type) {
      case OP_TRSMALL:
      case OP_TRQR: {
        m.first = (int)out.trc.size();
        for (int g : grp) {
          const Op& o = in[g]->ops[seq[g][h[g]]];
          for (int i = 0; i < o.count; ++i) {
            TrChunk c = in[g]->trc[o.first + i];
            c.job = rebase_tr(g, o.lane, c.job);
            out.trc.push_back(c);
          }
        }
        m.count = (int)out.trc.size() - m.first;
        break;
      }
      case OP_TRCHAIN: {
        m.first = (int)out.trc.size();
        for (int g : grp) {
          const Op& o = in[g]->ops[seq[g][h[g]]];
          for (int i = 0; i < o.count; ++i) {
            TrChunk c = in[g]->trc[o.first + i];
            for (int s = 1; s < c.chunk; ++s) rebase_tr(g, o.lane, c.job + s);
            c.job = rebase_tr(g, o.lane, c.job);
            out.trc.push_back(c);
          }
        }
        m.count = (int)out.trc.size() - m.first;
        break;
      }
      case OP_TRFORM: {
        m.first = (int)out.trf.size();
        for (int g : grp) {
          const Op& o = in[g]->ops[seq[g][h[g]]];
          for (int i = 0; i < o.count; ++i) {
            TrForm f = in[g]->trf[o.first + i];
            f.job = rebase_tr(g, o.lane, f.job);
            out.trf.push_back(f);
          }
        }
        m.count = (int)out.trf.size() - m.first;
        break;
      }
      case OP_MMPROJ:
      case OP_MMRED: {
        m.first = (int)out.mmp.size();
        for (int g : grp) {
          const Op& o = in[g]->ops[seq[g][h[g]]];
          for (int i = 0; i < o.count; ++i) {
            MmProj pr = in[g]->mmp[o.first + i];
            pr.job = rebase_mm(g, o.lane, pr.job);
            pr.part += wb[g] + in[g]->ws_off(o.lane);
            out.mmp.push_back(pr);
          }
        }
        m.count = (int)out.mmp.size() - m.first;
        break;
      }
      case OP_MMAPPLY: {
        m.first = (int)out.mma.size();
        for (int g : grp) {
          const Op& o = in[g]->ops[seq[g][h[g]]];
          for (int i = 0; i < o.count; ++i) {
            MmApply ap = in[g]->mma[o.first + i];
            ap.job = rebase_mm(g, o.lane, ap.job);
            out.mma.push_back(ap);
          }
        }
        m.count = (int)out.mma.size() - m.first;
        break;
      }
      case OP_GTALL: {
        m.first = (int)out.gt.size();
        for (int g : grp) {
          const Op& o = in[g]->ops[seq[g][h[g]]];
          for (int i = 0; i < o.count; ++i) {
            GemmTile t = in[g]->gt[o.first + i];
            t.job += gjb[g];
            out.gt.push_back(t);
          }
        }
        m.count = (int)out.gt.size() - m.first;
        break;
      }
      case OP_GRED: {
        m.first = (int)out.gr.size();
        for (int g : grp) {
          const Op& o = in[g]->ops[seq[g][h[g]]];
          for (int i = 0; i < o.count; ++i) {
            GemmRed r = in[g]->gr[o.first + i];
            r.job += gjb[g];
            r.part += wb[g] + in[g]->ws_off(o.lane);
            r.counter += (int)(cb[g] + in[g]->cnt_off(o.lane));
            out.gr.push_back(r);
          }
        }
        m.count = (int)out.gr.size() - m.first;
        break;
      }
      case OP_LGATHER:
      case OP_LPANEL:
      case OP_LUPDATE:
      case OP_LSCATTER: {
        // the launch's jobs are a contiguous run of leaf jobs; reuse the previous
        // run when the same leaves continue (the ~20 launches of one leaf QR)
        const int nper = (int)o0.n;
        std::vector<std::pair<int, int>> key;
        int njobs = 0;
        for (int g : grp) {
          const Op& o = in[g]->ops[seq[g][h[g]]];
          key.push_back({g, o.first});
          njobs += o.count / nper;
        }
        if (key != last_leaf) {
          last_leaf_first = (int)out.lj.size();
          for (int g : grp) {
            const Op& o = in[g]->ops[seq[g][h[g]]];
            for (int i = 0; i < o.count / nper; ++i) out.lj.push_back(in[g]->lj[o.first + i]);
          }
          last_leaf = key;
        }
        m.first = last_leaf_first;
        m.count = njobs * nper;
        break;
      }
      case OP_ROWS: {
        m.first = (int)out.rj.size();
        for (int g : grp) {
          const Op& o = in[g]->ops[seq[g][h[g]]];
          for (int i = 0; i < o.count; ++i) out.rj.push_back(in[g]->rj[o.first + i]);
        }
        m.count = (int)out.rj.size() - m.first;
        break;
      }
      case OP_FILL:
      case OP_NORMALIZE:
      case OP_SETSCAL: {
        m.first = (int)out.vj.size();
        for (int g : grp) {
          const Op& o = in[g]->ops[seq[g][h[g]]];
          for (int i = 0; i < o.count; ++i) out.vj.push_back(in[g]->vj[o.first + i]);
        }
        m.count = (int)out.vj.size() - m.first;
        break;
      }
      default:
        break;
    }
    out.ops.push_back(m);
    for (int g : grp) ++h[g];
  }
}

hodlr_status make_factor(const hodlr_s& A, double eps, double anorm, hipStream_t st,
                         std::unique_ptr<hodlr_qr_s>& out) {
  TRY(make_storage(A, eps, anorm, st, out));
  std::shared_ptr<Batch> B;
  TRY(make_batch({out.get()}, st, B));
  out->batch = B;
  return HODLR_OK;
}

hodlr_status lane_streams(Batch& B) {
  if (B.aux == nullptr) HIPCHK(hipStreamCreateWithFlags(&B.aux, hipStreamNonBlocking));
  while ((int)B.events.size() < B.plan.n_events + 2) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    B.events.push_back(e);
  }
  return HODLR_OK;
}

// Run the whole factorisation of every factor of a batch on `st`.  Default:
// direct launches, the T-factor lane on a second stream.  HODLR_QR_ONE_STREAM:
// direct launches in the serial order.  HODLR_QR_GRAPH: replay a HIP graph
// captured (once per batch) from the serial order on one stream; a graph
// captured from the two-stream form ran with wrong results on ROCm 7.2 although
// every edge of it was present, so the graph keeps the serial order.
hodlr_status run_batch(Batch& B, const std::vector<hodlr_qr_s*>& Fs, const std::vector<const hodlr_s*>& As,
                       uint32_t flags, hipStream_t st) {
  // the inputs are copied in by direct launches, so a captured graph holds the
  // factorisation's launches only and serves any inputs of the batch's shapes
  for (size_t i = 0; i < Fs.size(); ++i) TRY(reset_factor(*Fs[i], *As[i], st));
  if (B.merged) flags |= HODLR_QR_ONE_STREAM;
  if (!(flags & HODLR_QR_GRAPH)) {
    if (flags & HODLR_QR_ONE_STREAM) return run_ops(B.plan, B.work, st);
    TRY(lane_streams(B));
    return run_ops(B.plan, B.work, st, B.aux, B.events.data());
  }
  if (B.graph == nullptr) {
    // capture on a private stream so that the caller's stream state is untouched
    hipStream_t cs;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    TRY(set_attrs());
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hodlr_status s2 = run_ops(B.plan, B.work, cs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (s2 != HODLR_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s2;
    }
    if (e != hipSuccess) return fail(HODLR_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&B.graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      B.graph = nullptr;
      return fail(HODLR_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
  }
  HIPCHK(hipGraphLaunch(B.graph, st));
  return HODLR_OK;
}

hodlr_status run_factor(hodlr_qr_s& F, const hodlr_s& A, uint32_t flags, hipStream_t st) {
  return run_batch(*F.batch, {&F}, {&A}, flags, st);
}

// ---- cached launch sequences of the finished factors
// apply Q (trans 0) or Q^T (trans 1): slot 0 = X (n x s, the caller's), slots
// 1 and 2 = n x s temporaries:  W1 = Y^T X; W2 = op(T) W1; X -= Y W2
// (Q = I - Y T Y^T, eq. compactwy)
hodlr_status build_apply_plan(hodlr_qr_s& F, int trans, hipStream_t st, std::unique_ptr<CachedPlan>& out) {
  auto C = std::make_unique<CachedPlan>();
  C->mem.stream = st;
  Plan& P = C->P;
  P.tune = tuning_for(F.t.n, F.cap);
  MmSpec a = mmspec(F.view_y(), F.rect(), true, 1, 1, nullptr, 0, nullptr, nullptr, 0, 1.0, 0.0, 1);
  MmSpec b = mmspec(F.view_t(), true, false, 1, trans, nullptr, 0, nullptr, nullptr, 0, 1.0, 0.0, 1);
  MmSpec c = mmspec(F.view_y(), F.rect(), true, 1, 0, nullptr, 0, nullptr, nullptr, 0, -1.0, 1.0, 1);
  a.xs = 0, a.zs = 1;
  b.xs = 1, b.zs = 2;
  c.xs = 2, c.zs = 0;
  a.rld = b.rld = c.rld = F.cap;
  P.mm(F.t, {a});
  P.mm(F.tc, {b});
  P.mm(F.t, {c});
  TRY(P.upload_all(C->mem, st));
  out = std::move(C);
  return HODLR_OK;
}

// back substitution with the upper triangular HODLR R, last leaf first:
// x2 = R22^{-1} c2; c1 -= R12 x2; x1 = R11^{-1} c1.  Slot 0 = the right-hand
// sides (n x s), slot 1 = a KCAP x s temporary (V12^T x2).
hodlr_status build_solve_plan(hodlr_qr_s& F, hipStream_t st, std::unique_ptr<CachedPlan>& out) {
  auto C = std::make_unique<CachedPlan>();
  C->mem.stream = st;
  Plan& P = C->P;
  const Tree& t = F.tc;  // R on its pivot rows: square on the column partition
  P.tune = tuning_for(t.n, F.cap);
  struct Rec {
    hodlr_qr_s& f;
    Plan& P;
    const Tree& t;
    void go(int v) {
      if (t.is_leaf(v)) {
        const int j = v - t.nleaf();
        Op o{OP_TRSM};
        o.a0 = (int)t.m(v);
        o.a1 = f.rleaves.hview[j].ld;
        o.p0 = f.rleaves.hview[j].D;
        o.xs = 0;
        o.xoff = t.lo[v];
        P.push(o);
        return;
      }
      go(2 * v + 1);
      const HBlk& b = f.rset.hview[v];
      const int mL = (int)t.m(2 * v), mR = (int)t.m(2 * v + 1);
      // Wt = V12^T x2 (k x s), c1 -= U12 Wt
      GemmJob r = gjob(1, 0, 0, f.rank_up(v), 0, nullptr, mR, nullptr, b.V, b.ldV, nullptr, 0, nullptr, KCAP,
                       1.0, 0.0, FC_DENSE);
      r.bs_ = 0;
      r.boff = t.lo[2 * v + 1];
      r.cs_ = 1;
      P.gemm_red({GSpec{r, KCAP, KCAP, mR}});
      GemmJob u = gjob(0, 0, mL, nullptr, 0, nullptr, 0, f.rank_up(v), b.U, b.ldU, nullptr, KCAP, nullptr, 0,
                       -1.0, 1.0, FC_DENSE);
      u.bs_ = 1;
      u.cs_ = 0;
      u.coff = t.lo[2 * v];
      P.gemm_tall({GSpec{u, mL, SMAX, 0}});
      go(2 * v);
    }
  } rec{F, P, t};
  rec.go(1);
  TRY(P.upload_all(C->mem, st));
  out = std::move(C);
  return HODLR_OK;
}

// Z = op(M) X for a HODLR matrix or a factor view: slot 0 = X, slot 1 = Z
hodlr_status build_mm_plan(const hodlr_s& A, int trans, hipStream_t st, std::unique_ptr<CachedPlan>& out) {
  auto C = std::make_unique<CachedPlan>();
  C->mem.stream = st;
  Plan& P = C->P;
  P.tune = tuning_for(A.t.n, A.cap);
  MmSpec a = mmspec(A.view(), A.has_up, A.has_lo, 1, trans, nullptr, 0, nullptr, nullptr, 0, 1.0, 0.0,
                    A.leaf_kind != LEAF_FULL ? 1 : 0);
  a.xs = 0;
  a.zs = 1;
  a.rld = A.cap;
  P.mm(A.t, {a});
  TRY(P.upload_all(C->mem, st));
  out = std::move(C);
  return HODLR_OK;
}

hodlr_status finish_factor(hodlr_qr_s& F, hipStream_t st) {
  int err = 0;
  double sc[3];
  HIPCHK(hipMemcpyAsync(&err, F.work.err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(sc, F.scal, sizeof(sc), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  F.anorm = sc[0];
  F.tauA = sc[1];
  F.tauT = sc[2];
  if (err & ERR_STACK) return fail(HODLR_ECAPACITY, "stacked leaf column exceeds 1024 rows");
  if (err & ERR_WIDTH) return fail(HODLR_ECAPACITY, "a recompression width exceeded 128 columns");
  if (err & ERR_CAPACITY) return fail(HODLR_ECAPACITY, "an off-diagonal rank exceeded rank_cap");
  return HODLR_OK;
}

// keep the schedule's counts, release its plan and workspace, and cache the
// launch sequences of apply Q and solve (the factors are final)
hodlr_status finalize_factor(hodlr_qr_s& F, hipStream_t st, bool keep = false) {
  if (F.batch) {
    F.n_launch = F.batch->n_launch;
    F.n_trunc = (int64_t)F.logkeys.size();  // one key per recompression of this factorisation
    if (!keep) F.batch.reset();
  }
  if (F.applyp[0]) return HODLR_OK;  // refactorisation: same storage, cached sequences still valid
  F.mem.stream = st;
  TRY(build_apply_plan(F, 0, st, F.applyp[0]));
  TRY(build_apply_plan(F, 1, st, F.applyp[1]));
  TRY(build_solve_plan(F, st, F.solvep));
  return HODLR_OK;
}

// run a cached plan over the columns of the caller's operands in chunks of at
// most SMAX: slots[c] = (pointer, leading dimension) of slot c at column 0;
// slots flagged in `percol` advance by ld * c0 per chunk, the others are
// temporaries reused by every chunk
hodlr_status run_cached(const CachedPlan& C, hipStream_t st, int nslots, double* const* base, const int* ld,
                        const bool* percol, int64_t nrhs, int smax, double* ws, int* cnt) {
  Work W;
  W.ws = ws;
  W.counters = cnt;
  for (int64_t c0 = 0; c0 < nrhs; c0 += smax) {
    Opnd op{};
    for (int i = 0; i < nslots; ++i) {
      op.p[i] = base[i] + (percol[i] ? c0 * (int64_t)ld[i] : 0);
      op.ld[i] = ld[i];
    }
    op.s = (int)std::min<int64_t>(smax, nrhs - c0);
    if (cnt != nullptr && C.P.uses_counters()) TRY(zero_counters(cnt, C.P.cnt_need(), st));
    TRY(run_ops(C.P, W, st, nullptr, nullptr, op));
  }
  return HODLR_OK;
}

// power iteration on A^T A with HODLR products
hodlr_status norm2_est_impl(const hodlr_s& A, int iters, hipStream_t st, double* out) {
  const Tree& t = A.t;
  const int64_t n = t.n;
  CallMem tmp(st);
  double *x, *y, *z, *res;
  TRY(tmp.alloc(&x, n));
  TRY(tmp.alloc(&y, t.nr));
  TRY(tmp.alloc(&z, n));
  TRY(tmp.alloc(&res, 1));
  Plan P;
  P.tune = tuning_for(n, A.cap);
  plan_norm2(P, t, {NormItem{A.view(), A.cap, x, y, z, res, nullptr}}, iters);
  DMem pm;
  pm.stream = st;
  TRY(P.upload_all(pm, st));
  double* ws = nullptr;
  TRY(tmp.alloc(&ws, (size_t)std::max<int64_t>(1, P.ws_need())));
  Work W;
  W.ws = ws;
  TRY(run_ops(P, W, st));
  HIPCHK(hipMemcpyAsync(out, res, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return HODLR_OK;
}

}  // namespace
}  // namespace hqh

// ================================================================== C ABI
extern "C" {

const char* hodlr_last_error(void) { return g_err.c_str(); }
const char* hodlr_version(void) { return "hodlr-qr-gfx950 0.2"; }

hodlr_status hodlr_set_allocator(void* (*alloc)(size_t, hodlr_stream_t, void*),
                                 void (*release)(void*, hodlr_stream_t, void*), void* ctx) {
  g_err.clear();
  if ((alloc == nullptr) != (release == nullptr))
    return fail(HODLR_EINVAL, "alloc and release must both be set or both be NULL");
  std::lock_guard<std::mutex> lk(g_hook_mu);
  g_hook.alloc = alloc;
  g_hook.release = release;
  g_hook.ctx = ctx;
  return HODLR_OK;
}

}  // extern "C"

namespace hqh {
namespace {
// hodlr_build and hodlr_build_rect: row partition row_off, column partition col_off
hodlr_status build_impl(int64_t nr, int64_t n, int32_t levels, const int64_t* row_off, const int64_t* col_off,
                        const double* leaves, const int64_t* leaf_data_off, const double* U, const int64_t* u_off,
                        const double* V, const int64_t* v_off, const int32_t* ranks, int32_t rank_cap,
                        hodlr_stream_t stream, hodlr_t** out) {
  g_err.clear();
  if (out == nullptr) return fail(HODLR_EINVAL, "out is NULL");
  *out = nullptr;
  if (levels < 0 || levels > MAXGROUPS) return fail(HODLR_EINVAL, "levels out of range");
  if (n <= 0 || nr < n || col_off == nullptr || row_off == nullptr || leaves == nullptr ||
      leaf_data_off == nullptr)
    return fail(HODLR_EINVAL, "bad size or NULL array");
  if (rank_cap < 1 || rank_cap > KCAP) return fail(HODLR_EINVAL, "rank_cap must be in 1..64");
  const int nl = 1 << levels;
  const int nb = 2 * (nl - 1);
  if (nb > 0 && (U == nullptr || V == nullptr || u_off == nullptr || v_off == nullptr || ranks == nullptr))
    return fail(HODLR_EINVAL, "NULL block array");
  if (col_off[0] != 0 || col_off[nl] != n) return fail(HODLR_EINVAL, "leaf_off must run from 0 to n");
  if (row_off[0] != 0 || row_off[nl] != nr) return fail(HODLR_EINVAL, "row_off must run from 0 to m");
  for (int j = 0; j < nl; ++j) {
    const int64_t nj = col_off[j + 1] - col_off[j], mj = row_off[j + 1] - row_off[j];
    if (nj < 1) return fail(HODLR_EINVAL, "empty leaf");
    if (mj < nj) return fail(HODLR_EINVAL, "a leaf with fewer rows than columns");
    if (mj > MAXLEAF) return fail(HODLR_EINVAL, "leaf larger than 512");
  }
  hipStream_t st = (hipStream_t)stream;
  auto A = std::make_unique<hodlr_s>();
  A->mem.stream = st;
  A->t.init(levels, col_off, row_off);
  A->cap = rank_cap;
  const Tree& t = A->t;
  // validate ranks and finiteness
  int bi = 0;
  for (int d = 0; d < levels; ++d)
    for (int v = 1 << d; v < (2 << d); ++v)
      for (int kind = 0; kind < 2; ++kind, ++bi) {
        const int64_t rows = kind == 0 ? t.mr(2 * v) : t.mr(2 * v + 1);
        const int64_t cols = kind == 0 ? t.m(2 * v + 1) : t.m(2 * v);
        const int k = ranks[bi];
        if (k < 0 || k > rows || k > cols || k > rank_cap)
          return fail(HODLR_EINVAL, "block " + std::to_string(bi) + ": rank out of range");
        TRY(check_finite(U + u_off[bi], (size_t)(rows * k), "U"));
        TRY(check_finite(V + v_off[bi], (size_t)(cols * k), "V"));
      }
  for (int j = 0; j < nl; ++j)
    TRY(check_finite(leaves + leaf_data_off[j], (size_t)(t.mr(nl + j) * t.m(nl + j)), "leaves"));
  TRY(A->mem.alloc(&A->ranks, 2 * (size_t)nl + 8));
  A->rank_up_dev = A->ranks;
  A->rank_lo_dev = A->ranks + nl;
  TRY(make_leaves(A->mem, t, A->leaves));
  TRY(make_blocks(A->mem, t, rank_cap, BK_UP, A->ranks, A->up));
  TRY(make_blocks(A->mem, t, rank_cap, BK_LO, A->ranks + nl, A->lo));
  TRY(upload(A->mem, &A->up.dview, A->up.hview, st));
  TRY(upload(A->mem, &A->lo.dview, A->lo.hview, st));
  TRY(upload(A->mem, &A->leaves.dview, A->leaves.hview, st));
  // pack into the capacity layout on the host, then one copy per array
  std::vector<double> hl((size_t)A->leaves.size);
  for (int j = 0; j < nl; ++j)
    std::memcpy(hl.data() + A->leaves.off[j], leaves + leaf_data_off[j],
                (size_t)(t.mr(nl + j) * t.m(nl + j)) * sizeof(double));
  std::vector<double> uu((size_t)A->up.usz, 0.0), uv((size_t)A->up.vsz, 0.0), lu((size_t)A->lo.usz, 0.0),
      lv((size_t)A->lo.vsz, 0.0);
  std::vector<int> hr(2 * (size_t)nl + 8, 0);
  bi = 0;
  for (int d = 0; d < levels; ++d)
    for (int v = 1 << d; v < (2 << d); ++v)
      for (int kind = 0; kind < 2; ++kind, ++bi) {
        BlockSet& B = kind == 0 ? A->up : A->lo;
        std::vector<double>& bu = kind == 0 ? uu : lu;
        std::vector<double>& bv = kind == 0 ? uv : lv;
        const int64_t rows = kind == 0 ? t.mr(2 * v) : t.mr(2 * v + 1);
        const int64_t cols = kind == 0 ? t.m(2 * v + 1) : t.m(2 * v);
        const int k = ranks[bi];
        std::memcpy(bu.data() + B.uoff[v], U + u_off[bi], (size_t)(rows * k) * sizeof(double));
        std::memcpy(bv.data() + B.voff[v], V + v_off[bi], (size_t)(cols * k) * sizeof(double));
        hr[(kind == 0 ? 0 : nl) + v] = k;
      }
  HIPCHK(hipMemcpyAsync(A->leaves.D, hl.data(), hl.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(A->up.U, uu.data(), uu.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(A->up.V, uv.data(), uv.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(A->lo.U, lu.data(), lu.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(A->lo.V, lv.data(), lv.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(A->ranks, hr.data(), hr.size() * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  *out = A.release();
  return HODLR_OK;
}
}  // namespace
}  // namespace hqh

extern "C" {

hodlr_status hodlr_build(int64_t n, int32_t levels, const int64_t* leaf_off, const double* leaves,
                         const int64_t* leaf_data_off, const double* U, const int64_t* u_off,
                         const double* V, const int64_t* v_off, const int32_t* ranks, int32_t rank_cap,
                         hodlr_stream_t stream, hodlr_t** out) {
  return build_impl(n, n, levels, leaf_off, leaf_off, leaves, leaf_data_off, U, u_off, V, v_off, ranks, rank_cap,
                    stream, out);
}

hodlr_status hodlr_build_rect(int64_t m, int64_t n, int32_t levels, const int64_t* row_off, const int64_t* col_off,
                              const double* leaves, const int64_t* leaf_data_off, const double* U,
                              const int64_t* u_off, const double* V, const int64_t* v_off, const int32_t* ranks,
                              int32_t rank_cap, hodlr_stream_t stream, hodlr_t** out) {
  return build_impl(m, n, levels, row_off, col_off, leaves, leaf_data_off, U, u_off, V, v_off, ranks, rank_cap,
                    stream, out);
}

void hodlr_free(hodlr_t* A) {
  if (A != nullptr && !A->borrowed) delete A;
}
void hodlr_qr_free(hodlr_qr_t* F) { delete F; }

hodlr_status hodlr_norm2_est(const hodlr_t* A, int32_t iters, hodlr_stream_t stream, double* out) {
  g_err.clear();
  if (A == nullptr || out == nullptr || iters < 0) return fail(HODLR_EINVAL, "bad argument");
  return norm2_est_impl(*A, iters, (hipStream_t)stream, out);
}

hodlr_status hodlr_qr(const hodlr_t* A, double eps, double anorm, uint32_t flags, hodlr_stream_t stream,
                      hodlr_qr_t** out) {
  g_err.clear();
  if (A == nullptr || out == nullptr) return fail(HODLR_EINVAL, "NULL argument");
  *out = nullptr;
  if (A->borrowed || A->leaf_kind != LEAF_FULL) return fail(HODLR_EINVAL, "A is a factor view, not a matrix");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(HODLR_EINVAL, "eps must be finite and >= 0");
  hipStream_t st = (hipStream_t)stream;
  std::unique_ptr<hodlr_qr_s> F;
  TRY(make_factor(*A, eps, anorm, st, F));
  TRY(run_factor(*F, *A, flags, st));
  TRY(finish_factor(*F, st));
  TRY(finalize_factor(*F, st, (flags & HODLR_QR_KEEP) != 0));
  *out = F.release();
  return HODLR_OK;
}

}  // extern "C"

namespace hqh {
namespace {

// Factors of a set of matrices with one schedule per group of matrices that share
// partition and rank capacity; groups are run one after the other.
struct BatchSet {
  std::vector<std::unique_ptr<hodlr_qr_s>> F;
  std::vector<std::vector<int>> groups;  // indices into F / A
  bool merged = false;                   // one merged launch sequence (serial order)
};

hodlr_status make_batch_set(const hodlr_t* const* A, int count, double eps, const double* anorm,
                            uint32_t flags, hipStream_t st, BatchSet& S) {
  S.F.resize(count);
  for (int i = 0; i < count; ++i) {
    TRY(make_storage(*A[i], eps, anorm ? anorm[i] : 0.0, st, S.F[i]));
    bool placed = false;
    for (auto& g : S.groups) {
      const hodlr_s& B = *A[g[0]];
      if (B.t.L == A[i]->t.L && B.t.n == A[i]->t.n && B.cap == A[i]->cap && B.t.lo == A[i]->t.lo &&
          B.t.hi == A[i]->t.hi && B.t.rlo == A[i]->t.rlo && B.t.rhi == A[i]->t.rhi) {
        g.push_back(i);
        placed = true;
        break;
      }
    }
    if (!placed) S.groups.push_back({i});
  }
  bool one_cap = true;
  for (int i = 1; i < count; ++i) one_cap = one_cap && A[i]->cap == A[0]->cap;
  if (S.groups.size() > 1 && one_cap && !(flags & HODLR_QR_BY_SHAPE)) {
    // one launch sequence across the shapes
    std::vector<Plan> plans(S.groups.size());
    std::vector<const Plan*> pp;
    for (size_t gi = 0; gi < S.groups.size(); ++gi) {
      std::vector<hodlr_qr_s*> fs;
      for (int i : S.groups[gi]) fs.push_back(S.F[i].get());
      build_plan(fs, plans[gi]);
      pp.push_back(&plans[gi]);
    }
    auto B = std::make_shared<Batch>();
    B->mem.stream = st;
    B->size = count;
    B->merged = true;
    for (auto& F : S.F) B->members.push_back(F.get());
    merge_plans(pp, B->plan);
    TRY(finish_batch(*B, st));
    for (auto& F : S.F) F->batch = B;
    std::vector<int> all;
    for (int i = 0; i < count; ++i) all.push_back(i);
    S.groups = {all};
    S.merged = true;
    return HODLR_OK;
  }
  for (auto& g : S.groups) {
    std::vector<hodlr_qr_s*> fs;
    for (int i : g) fs.push_back(S.F[i].get());
    std::shared_ptr<Batch> B;
    TRY(make_batch(fs, st, B));
    for (int i : g) S.F[i]->batch = B;
  }
  return HODLR_OK;
}

hodlr_status run_batch_set(BatchSet& S, const hodlr_t* const* A, uint32_t flags, hipStream_t st) {
  for (auto& g : S.groups) {
    std::vector<hodlr_qr_s*> fs;
    std::vector<const hodlr_s*> as;
    for (int i : g) {
      fs.push_back(S.F[i].get());
      as.push_back(A[i]);
    }
    TRY(run_batch(*S.F[g[0]]->batch, fs, as, flags, st));
  }
  return HODLR_OK;
}

hodlr_status check_batch_args(const hodlr_t* const* A, int count, double eps) {
  if (A == nullptr || count < 1) return fail(HODLR_EINVAL, "need at least one matrix");
  for (int i = 0; i < count; ++i) {
    if (A[i] == nullptr) return fail(HODLR_EINVAL, "NULL matrix in the batch");
    if (A[i]->borrowed || A[i]->leaf_kind != LEAF_FULL)
      return fail(HODLR_EINVAL, "a factor view in the batch");
  }
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(HODLR_EINVAL, "eps must be finite and >= 0");
  return HODLR_OK;
}

// the view of one factor of F, or nullptr
const hodlr_s* factor_view(const hodlr_qr_s* F, char which) {
  switch (which) {
    case 'Y': return F->vY.get();
    case 'T': return F->vT.get();
    case 'R': return F->vR.get();
    default: return nullptr;
  }
}

hodlr_status matmul_impl(const hodlr_s& A, int32_t trans, int64_t nrhs, const double* X, int64_t ldx,
                         double* Z, int64_t ldz, hipStream_t st) {
  const int64_t xrows = trans ? A.t.nr : A.t.n, zrows = trans ? A.t.n : A.t.nr;
  if (X == nullptr || Z == nullptr || nrhs < 0 || ldx < xrows || ldz < zrows)
    return fail(HODLR_EINVAL, "bad operand");
  if (nrhs == 0) return HODLR_OK;
  if (ldx > INT32_MAX || ldz > INT32_MAX) return fail(HODLR_EINVAL, "leading dimension too large");
  const int tr = trans ? 1 : 0;
  hodlr_s& a = const_cast<hodlr_s&>(A);
  const CachedPlan* C;
  {
    std::lock_guard<std::mutex> lk(a.mu);
    if (!a.mmplan[tr]) TRY(build_mm_plan(A, tr, st, a.mmplan[tr]));
    C = a.mmplan[tr].get();
  }
  CallMem tmp(st);
  double* ws = nullptr;
  TRY(tmp.alloc(&ws, (size_t)std::max<int64_t>(1, C->P.ws_need())));
  double* base[2] = {const_cast<double*>(X), Z};
  const int ld[2] = {(int)ldx, (int)ldz};
  const bool percol[2] = {true, true};
  return run_cached(*C, st, 2, base, ld, percol, nrhs, SMAX, ws, nullptr);
}

// ---- the allocation-free entry point's scratch
// File-scope device array (each device the library runs on holds one copy
// until the process ends).  Host code never passes the array's name to a
// kernel: it is a host-side stand-in, not a device address.  Its device
// address is looked up once per device with hipGetSymbolAddress and kept.
constexpr int64_t NOALLOC_DOUBLES = (int64_t)1 << 22;  // 32 MiB
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;

hodlr_status scratch_ptr(double** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return HODLR_OK;
  }
  double* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    (void)hipGetLastError();
    return fail(HODLR_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return HODLR_OK;
}

// X <- Q X or Q^T X with temporaries from `scratch` (doubles) when given, else
// from the caller's allocator
hodlr_status apply_q_impl(const hodlr_qr_s& F, int32_t trans, int64_t nrhs, double* X, int64_t ldx,
                          hipStream_t st, double* scratch, int64_t scratch_doubles) {
  if (X == nullptr || nrhs < 0 || ldx < F.t.nr) return fail(HODLR_EINVAL, "bad argument");
  if (ldx > INT32_MAX) return fail(HODLR_EINVAL, "leading dimension too large");
  if (nrhs == 0) return HODLR_OK;
  const CachedPlan& C = *F.applyp[trans ? 1 : 0];
  const int64_t n = F.t.n;
  const int64_t wsn = std::max<int64_t>(1, C.P.ws_need());
  int smax = (int)std::min<int64_t>(SMAX, nrhs);
  double* buf = nullptr;
  std::unique_ptr<CallMem> tmp;
  if (scratch != nullptr) {
    const int64_t fit = (scratch_doubles - wsn) / (2 * n);
    if (fit < 1)
      return fail(HODLR_EINVAL, "the static scratch holds " + std::to_string(scratch_doubles) +
                                    " doubles; this factor needs at least " + std::to_string(wsn + 2 * n));
    smax = (int)std::min<int64_t>(smax, fit);
    buf = scratch;
  } else {
    tmp = std::make_unique<CallMem>(st);
    TRY(tmp->alloc(&buf, (size_t)(2 * n * smax + wsn)));
  }
  double* base[3] = {X, buf, buf + n * smax};
  const int ld[3] = {(int)ldx, (int)n, (int)n};
  const bool percol[3] = {true, false, false};
  return run_cached(C, st, 3, base, ld, percol, nrhs, smax, buf + 2 * n * smax, nullptr);
}

}  // namespace
}  // namespace hqh

extern "C" {

hodlr_status hodlr_qr_batched(const hodlr_t* const* A, int32_t count, double eps, const double* anorm,
                              uint32_t flags, hodlr_stream_t stream, hodlr_qr_t** out) {
  g_err.clear();
  if (out == nullptr) return fail(HODLR_EINVAL, "NULL argument");
  TRY(check_batch_args(A, count, eps));
  for (int i = 0; i < count; ++i) out[i] = nullptr;
  hipStream_t st = (hipStream_t)stream;
  BatchSet S;
  TRY(make_batch_set(A, count, eps, anorm, flags, st, S));
  TRY(run_batch_set(S, A, flags, st));
  hodlr_status first_err = HODLR_OK;
  std::string msg;
  for (int i = 0; i < count; ++i) {
    const hodlr_status e = finish_factor(*S.F[i], st);
    if (e != HODLR_OK && first_err == HODLR_OK) {
      first_err = e;
      msg = "matrix " + std::to_string(i) + ": " + g_err;
    }
  }
  if (first_err != HODLR_OK) return fail(first_err, msg);
  for (int i = 0; i < count; ++i) TRY(finalize_factor(*S.F[i], st, (flags & HODLR_QR_KEEP) != 0));
  for (int i = 0; i < count; ++i) out[i] = S.F[i].release();
  return HODLR_OK;
}

hodlr_status hodlr_qr_refactor(hodlr_qr_t* const* F, const hodlr_t* const* A, int32_t count, uint32_t flags,
                               hodlr_stream_t stream) {
  g_err.clear();
  if (F == nullptr || A == nullptr || count < 1) return fail(HODLR_EINVAL, "bad argument");
  for (int i = 0; i < count; ++i) {
    if (F[i] == nullptr || A[i] == nullptr) return fail(HODLR_EINVAL, "NULL handle");
    if (!F[i]->batch) return fail(HODLR_EINVAL, "factorisation " + std::to_string(i) + " kept no schedule");
    const hodlr_s& a = *A[i];
    if (a.borrowed || a.leaf_kind != LEAF_FULL) return fail(HODLR_EINVAL, "a factor view in place of a matrix");
    if (a.t.L != F[i]->t.L || a.t.n != F[i]->t.n || a.cap != F[i]->cap || a.t.lo != F[i]->t.lo ||
        a.t.hi != F[i]->t.hi || a.t.rlo != F[i]->t.rlo || a.t.rhi != F[i]->t.rhi)
      return fail(HODLR_EINVAL, "matrix " + std::to_string(i) + " differs in partition or rank_cap");
  }
  // every schedule is run once, over exactly the factorisations it was built for
  std::vector<Batch*> seen;
  for (int i = 0; i < count; ++i) {
    Batch* B = F[i]->batch.get();
    if (std::find(seen.begin(), seen.end(), B) != seen.end()) continue;
    seen.push_back(B);
    std::vector<const hodlr_s*> as(B->members.size(), nullptr);
    int given = 0;
    for (int j = 0; j < count; ++j) {
      if (F[j]->batch.get() != B) continue;
      auto it = std::find(B->members.begin(), B->members.end(), F[j]);
      if (it == B->members.end() || as[it - B->members.begin()] != nullptr)
        return fail(HODLR_EINVAL, "a factorisation appears twice");
      as[it - B->members.begin()] = A[j];
      ++given;
    }
    if (given != (int)B->members.size())
      return fail(HODLR_EINVAL, "every factorisation of a kept batch must be refactorised together");
  }
  hipStream_t st = (hipStream_t)stream;
  for (Batch* B : seen) {
    std::vector<const hodlr_s*> as(B->members.size());
    for (int j = 0; j < count; ++j)
      if (F[j]->batch.get() == B)
        as[std::find(B->members.begin(), B->members.end(), F[j]) - B->members.begin()] = A[j];
    TRY(run_batch(*B, B->members, as, flags, st));
  }
  hodlr_status first_err = HODLR_OK;
  std::string msg;
  for (int i = 0; i < count; ++i) {
    const hodlr_status e = finish_factor(*F[i], st);
    if (e != HODLR_OK && first_err == HODLR_OK) {
      first_err = e;
      msg = "matrix " + std::to_string(i) + ": " + g_err;
    }
  }
  if (first_err != HODLR_OK) return fail(first_err, msg);
  return HODLR_OK;
}

hodlr_status hodlr_qr_batched_time(const hodlr_t* const* A, int32_t count, double eps, const double* anorm,
                                   uint32_t flags, int32_t warmup, int32_t reps, hodlr_stream_t stream,
                                   double* ms) {
  g_err.clear();
  if (ms == nullptr || reps < 1 || warmup < 0) return fail(HODLR_EINVAL, "bad argument");
  TRY(check_batch_args(A, count, eps));
  hipStream_t st = (hipStream_t)stream;
  BatchSet S;
  TRY(make_batch_set(A, count, eps, anorm, flags, st, S));
  for (int i = 0; i < warmup; ++i) TRY(run_batch_set(S, A, flags, st));
  for (int i = 0; i < count; ++i) TRY(finish_factor(*S.F[i], st));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (int r = 0; r < reps; ++r) {
    HIPCHK(hipEventRecord(e0, st));
    TRY(run_batch_set(S, A, flags, st));
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    ms[r] = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (int i = 0; i < count; ++i) TRY(finish_factor(*S.F[i], st));
  return HODLR_OK;
}

hodlr_status hodlr_qr_time(const hodlr_t* A, double eps, double anorm, uint32_t flags, int32_t warmup,
                           int32_t reps, hodlr_stream_t stream, double* ms) {
  g_err.clear();
  if (A == nullptr || ms == nullptr || reps < 1 || warmup < 0) return fail(HODLR_EINVAL, "bad argument");
  if (A->borrowed || A->leaf_kind != LEAF_FULL) return fail(HODLR_EINVAL, "A is a factor view, not a matrix");
  hipStream_t st = (hipStream_t)stream;
  std::unique_ptr<hodlr_qr_s> F;
  TRY(make_factor(*A, eps, anorm, st, F));
  for (int i = 0; i < warmup; ++i) TRY(run_factor(*F, *A, flags, st));
  TRY(finish_factor(*F, st));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  for (int i = 0; i < reps; ++i) {
    HIPCHK(hipEventRecord(e0, st));
    TRY(run_factor(*F, *A, flags, st));
    HIPCHK(hipEventRecord(e1, st));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    ms[i] = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return finish_factor(*F, st);
}

hodlr_status hodlr_matmul(const hodlr_t* A, int32_t trans, int64_t nrhs, const double* X, int64_t ldx,
                          double* Z, int64_t ldz, hodlr_stream_t stream) {
  g_err.clear();
  if (A == nullptr) return fail(HODLR_EINVAL, "NULL matrix");
  return matmul_impl(*A, trans, nrhs, X, ldx, Z, ldz, (hipStream_t)stream);
}

hodlr_status hodlr_qr_factor(const hodlr_qr_t* F, char which, const hodlr_t** view) {
  g_err.clear();
  if (F == nullptr || view == nullptr) return fail(HODLR_EINVAL, "NULL argument");
  const hodlr_s* v = factor_view(F, which);
  if (v == nullptr) return fail(HODLR_EINVAL, "which must be 'Y', 'T' or 'R'");
  *view = v;
  return HODLR_OK;
}

hodlr_status hodlr_qr_matmul(const hodlr_qr_t* F, char which, int32_t trans, int64_t nrhs, const double* X,
                             int64_t ldx, double* Z, int64_t ldz, hodlr_stream_t stream) {
  g_err.clear();
  if (F == nullptr) return fail(HODLR_EINVAL, "NULL factors");
  const hodlr_s* v = factor_view(F, which);
  if (v == nullptr) return fail(HODLR_EINVAL, "which must be 'Y', 'T' or 'R'");
  return matmul_impl(*v, trans, nrhs, X, ldx, Z, ldz, (hipStream_t)stream);
}

hodlr_status hodlr_apply_q(const hodlr_qr_t* F, int32_t trans, int64_t nrhs, double* X, int64_t ldx,
                           hodlr_stream_t stream) {
  g_err.clear();
  if (F == nullptr) return fail(HODLR_EINVAL, "NULL factors");
  return apply_q_impl(*F, trans, nrhs, X, ldx, (hipStream_t)stream, nullptr, 0);
}

hodlr_status hodlr_apply_q_noalloc(const hodlr_qr_t* F, int32_t trans, int64_t nrhs, double* X, int64_t ldx,
                                   hodlr_stream_t stream) {
  g_err.clear();
  if (F == nullptr) return fail(HODLR_EINVAL, "NULL factors");
  if (X == nullptr || nrhs < 0 || ldx < F->t.nr) return fail(HODLR_EINVAL, "bad argument");
  double* buf = nullptr;
  TRY(scratch_ptr(&buf));
  return apply_q_impl(*F, trans, nrhs, X, ldx, (hipStream_t)stream, buf, NOALLOC_DOUBLES);
}

hodlr_status hodlr_solve(const hodlr_qr_t* F, int64_t nrhs, double* B, int64_t ldb, hodlr_stream_t stream) {
  g_err.clear();
  if (F == nullptr || B == nullptr || nrhs < 0 || ldb < F->t.n) return fail(HODLR_EINVAL, "bad argument");
  if (F->rect()) return fail(HODLR_EINVAL, "a rectangular factorisation: use hodlr_lstsq");
  if (ldb > INT32_MAX) return fail(HODLR_EINVAL, "leading dimension too large");
  if (nrhs == 0) return HODLR_OK;
  hipStream_t st = (hipStream_t)stream;
  TRY(apply_q_impl(*F, 1, nrhs, B, ldb, st, nullptr, 0));
  const CachedPlan& C = *F->solvep;
  CallMem tmp(st);
  double *wm = nullptr, *ws = nullptr;
  int* cnt = nullptr;
  TRY(tmp.alloc(&wm, (size_t)KCAP * SMAX));
  TRY(tmp.alloc(&ws, (size_t)std::max<int64_t>(1, C.P.ws_need())));
  TRY(tmp.alloc(&cnt, (size_t)C.P.cnt_need()));
  double* base[2] = {B, wm};
  const int ld[2] = {(int)ldb, KCAP};
  const bool percol[2] = {true, false};
  return run_cached(C, st, 2, base, ld, percol, nrhs, SMAX, ws, cnt);
}

hodlr_status hodlr_lstsq(const hodlr_qr_t* F, int64_t nrhs, double* B, int64_t ldb, double* X, int64_t ldx,
                         hodlr_stream_t stream) {
  g_err.clear();
  if (F == nullptr || B == nullptr || X == nullptr || nrhs < 0 || ldb < F->t.nr || ldx < F->t.n)
    return fail(HODLR_EINVAL, "bad argument");
  if (ldb > INT32_MAX || ldx > INT32_MAX) return fail(HODLR_EINVAL, "leading dimension too large");
  if (nrhs == 0) return HODLR_OK;
  hipStream_t st = (hipStream_t)stream;
  TRY(apply_q_impl(*F, 1, nrhs, B, ldb, st, nullptr, 0));
  // the pivot rows of Q^T B, in column order, into X
  const int nl = F->t.nleaf();
  k_pivot_rows<<<dim3(nl, (unsigned)std::min<int64_t>(nrhs, 65535)), NT_MM, 0, st>>>(
      F->pivrun, nl, B, (int)ldb, X, (int)ldx, (int)nrhs);
  HIPCHK(hipGetLastError());
  const CachedPlan& C = *F->solvep;
  CallMem tmp(st);
  double *wm = nullptr, *ws = nullptr;
  int* cnt = nullptr;
  TRY(tmp.alloc(&wm, (size_t)KCAP * SMAX));
  TRY(tmp.alloc(&ws, (size_t)std::max<int64_t>(1, C.P.ws_need())));
  TRY(tmp.alloc(&cnt, (size_t)C.P.cnt_need()));
  double* base[2] = {X, wm};
  const int ld[2] = {(int)ldx, KCAP};
  const bool percol[2] = {true, false};
  return run_cached(C, st, 2, base, ld, percol, nrhs, SMAX, ws, cnt);
}

hodlr_status hodlr_check(const hodlr_qr_t* F, hodlr_stream_t stream) {
  g_err.clear();
  if (F == nullptr) return fail(HODLR_EINVAL, "NULL factors");
  hipStream_t st = (hipStream_t)stream;
  int err = 0;
  HIPCHK(hipMemcpyAsync(&err, F->work.err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (err & ERR_STACK) return fail(HODLR_ECAPACITY, "stacked leaf column exceeds 1024 rows");
  if (err & ERR_WIDTH) return fail(HODLR_ECAPACITY, "a recompression width exceeded 128 columns");
  if (err & ERR_CAPACITY) return fail(HODLR_ECAPACITY, "an off-diagonal rank exceeded rank_cap");
  return HODLR_OK;
}

hodlr_status hodlr_qr_profile(const hodlr_t* A, double eps, double anorm, int32_t ntypes, double* ms,
                              int64_t* counts, double* flops, hodlr_stream_t stream) {
  g_err.clear();
  if (A == nullptr || ms == nullptr || counts == nullptr || flops == nullptr || ntypes < 1)
    return fail(HODLR_EINVAL, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  std::unique_ptr<hodlr_qr_s> F;
  TRY(make_factor(*A, eps, anorm, st, F));
  TRY(set_attrs());
  for (int i = 0; i < ntypes; ++i) {
    ms[i] = 0.0;
    counts[i] = 0;
    flops[i] = 0.0;
  }
  TRY(reset_factor(*F, *A, st));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double prev = 0.0;
  const Batch& B = *F->batch;
  for (const Op& o : B.plan.ops) {
    if (!op_launches(o)) continue;
    Launch L;
    L.e0 = e0;
    L.e1 = e1;
    run_op(B.plan, B.work, o, st, L, Opnd{});
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.0f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    const double tot = flop_sum(F->work.fc, 0, FC_N + 1);  // the norm estimate's products included
    if (tot < 0.0) return fail(HODLR_EDEVICE, "reading the flop counters failed");
    if (o.type < ntypes) {
      ms[o.type] += t;
      counts[o.type] += 1;
      flops[o.type] += tot - prev;
    }
    prev = tot;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return finish_factor(*F, st);
}

const char* hodlr_op_name(int32_t type) { return (type >= 0 && type < OP_NTYPES) ? OP_NAMES[type] : ""; }
int32_t hodlr_op_count(void) { return OP_NTYPES; }

hodlr_status hodlr_qr_info(const hodlr_qr_t* F, hodlr_qr_info_t* info) {
  g_err.clear();
  if (F == nullptr || info == nullptr) return fail(HODLR_EINVAL, "NULL argument");
  const int nn = 1 << F->t.L;
  std::vector<int> r(4 * (size_t)nn + 8);
  HIPCHK(hipMemcpy(r.data(), F->ranks, r.size() * sizeof(int), hipMemcpyDeviceToHost));
  std::memset(info, 0, sizeof(*info));
  info->n = F->t.n;
  info->levels = F->t.L;
  info->rank_cap = F->cap;
  for (int v = 1; v < nn; ++v) {
    info->max_rank_r = std::max(info->max_rank_r, r[v]);
    info->max_rank_y = std::max(info->max_rank_y, r[nn + v]);
    info->max_rank_t = std::max(info->max_rank_t, r[2 * nn + v]);
    if (F->rect()) info->max_rank_y = std::max(info->max_rank_y, r[3 * nn + v]);  // Y's upper blocks
  }
  info->anorm = F->anorm;
  info->tau_a = F->tauA;
  info->tau_t = F->tauT;
  info->flops = flop_total(F->work.fc);
  info->norm_flops = flop_sum(F->work.fc, FC_NORM, FC_NORM + 1);
  info->n_truncations = (int64_t)F->logkeys.size();
  info->n_launches = F->batch ? F->batch->n_launch : F->n_launch;
  info->device_bytes = (int64_t)F->mem.bytes;
  return HODLR_OK;
}

hodlr_status hodlr_qr_ranklog(const hodlr_qr_t* F, int32_t* recs, int64_t cap, int64_t* count) {
  g_err.clear();
  if (F == nullptr || count == nullptr) return fail(HODLR_EINVAL, "NULL argument");
  const int64_t n = std::min<int64_t>((int64_t)F->logkeys.size(), F->nlog_cap);
  *count = n;
  if (recs == nullptr) return HODLR_OK;
  if (cap < n) return fail(HODLR_EINVAL, "the record array holds fewer than count records");
  std::vector<int> h(2 * (size_t)std::max<int64_t>(1, n));
  if (n > 0) HIPCHK(hipMemcpy(h.data(), F->rlog, 2 * (size_t)n * sizeof(int), hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; ++i) {
    for (int q = 0; q < 5; ++q) recs[7 * i + q] = F->logkeys[i][q];
    recs[7 * i + 5] = h[2 * i];
    recs[7 * i + 6] = h[2 * i + 1];
  }
  return HODLR_OK;
}

}  // extern "C"

namespace hqh {
namespace {

hodlr_status export_impl(const Tree& t, const LeafSet& L, const BlockSet* up, const BlockSet* lo,
                         const int* d_ranks_up, const int* d_ranks_lo, int leafmode, double* leaves, double* U,
                         int64_t* u_off, double* V, int64_t* v_off, int32_t* ranks) {
  if (leaves == nullptr || ranks == nullptr || u_off == nullptr || v_off == nullptr)
    return fail(HODLR_EINVAL, "NULL output");
  const int nl = t.nleaf();
  std::vector<double> hl((size_t)L.size);
  HIPCHK(hipMemcpy(hl.data(), L.D, hl.size() * sizeof(double), hipMemcpyDeviceToHost));
  int64_t pos = 0;
  for (int j = 0; j < nl; ++j) {
    const int64_t m = t.mr(nl + j), n = t.m(nl + j), ld = L.hview[j].ld;
    for (int64_t c = 0; c < n; ++c)
      for (int64_t r = 0; r < m; ++r) {
        double x = hl[L.off[j] + r + c * ld];
        if (leafmode == LEAF_UNIT_LOWER) x = r > c ? x : (r == c ? 1.0 : 0.0);
        if (leafmode == LEAF_UPPER) x = r <= c ? x : 0.0;
        leaves[pos + r + c * m] = x;
      }
    pos += m * n;
  }
  std::vector<int> rk(2 * (size_t)nl, 0);
  if (d_ranks_up) HIPCHK(hipMemcpy(rk.data(), d_ranks_up, nl * sizeof(int), hipMemcpyDeviceToHost));
  if (d_ranks_lo) HIPCHK(hipMemcpy(rk.data() + nl, d_ranks_lo, nl * sizeof(int), hipMemcpyDeviceToHost));
  int64_t up_ = 0, vp_ = 0;
  int bi = 0;
  for (int d = 0; d < t.L; ++d)
    for (int v = 1 << d; v < (2 << d); ++v)
      for (int kind = 0; kind < 2; ++kind, ++bi) {
        const BlockSet* B = kind == 0 ? up : lo;
        const int64_t rows = kind == 0 ? t.mr(2 * v) : t.mr(2 * v + 1);
        const int64_t cols = kind == 0 ? t.m(2 * v + 1) : t.m(2 * v);
        const int k = B ? rk[(kind == 0 ? 0 : nl) + v] : 0;
        ranks[bi] = k;
        u_off[bi] = up_;
        v_off[bi] = vp_;
        if (k > 0) {
          if (U == nullptr || V == nullptr) return fail(HODLR_EINVAL, "NULL U or V");
          const HBlk& hb = B->hview[v];
          HIPCHK(hipMemcpy2D(U + up_, rows * sizeof(double), hb.U, hb.ldU * sizeof(double), rows * sizeof(double), k,
                             hipMemcpyDeviceToHost));
          HIPCHK(hipMemcpy2D(V + vp_, cols * sizeof(double), hb.V, hb.ldV * sizeof(double), cols * sizeof(double), k,
                             hipMemcpyDeviceToHost));
        }
        up_ += rows * k;
        vp_ += cols * k;
      }
  return HODLR_OK;
}

hodlr_status export_view(const hodlr_s& A, double* leaves, double* U, int64_t* u_off, double* V, int64_t* v_off,
                         int32_t* ranks) {
  return export_impl(A.t, A.leaves, A.has_up ? &A.up : nullptr, A.has_lo ? &A.lo : nullptr,
                     A.has_up ? A.rank_up_dev : nullptr, A.has_lo ? A.rank_lo_dev : nullptr, A.leaf_kind, leaves, U,
                     u_off, V, v_off, ranks);
}

}  // namespace
}  // namespace hqh

extern "C" {

hodlr_status hodlr_export(const hodlr_t* A, double* leaves, double* U, int64_t* u_off, double* V,
                          int64_t* v_off, int32_t* ranks) {
  g_err.clear();
  if (A == nullptr) return fail(HODLR_EINVAL, "NULL matrix");
  return export_view(*A, leaves, U, u_off, V, v_off, ranks);
}

hodlr_status hodlr_qr_export(const hodlr_qr_t* F, char which, double* leaves, double* U, int64_t* u_off,
                             double* V, int64_t* v_off, int32_t* ranks) {
  g_err.clear();
  if (F == nullptr) return fail(HODLR_EINVAL, "NULL factors");
  const hodlr_s* v = factor_view(F, which);
  if (v == nullptr) return fail(HODLR_EINVAL, "which must be 'Y', 'T' or 'R'");
  return export_view(*v, leaves, U, u_off, V, v_off, ranks);
}

// Build the factorisation schedule of a partition without a device (every
// address virtual) and test it for hazards between the two streams and
// between the jobs of each launch.
hodlr_status hodlr_plan_check(int64_t n, int32_t levels, const int64_t* leaf_off, int32_t rank_cap, int32_t count,
                              uint32_t flags, int64_t* stats, char* msg, int64_t msglen) {
  return hodlr_plan_check_set(1, &n, &levels, leaf_off, rank_cap, count, flags, stats, msg, msglen);
}

hodlr_status hodlr_plan_check_set(int32_t nshapes, const int64_t* n, const int32_t* levels, const int64_t* leaf_off,
                                  int32_t rank_cap, int32_t count, uint32_t flags, int64_t* stats, char* msg,
                                  int64_t msglen) {
  g_err.clear();
  if (n == nullptr || levels == nullptr || leaf_off == nullptr || stats == nullptr || nshapes < 1 || count < 1 ||
      rank_cap < 1 || rank_cap > KCAP)
    return fail(HODLR_EINVAL, "bad argument");
  struct Virt {
    Virt() { g_virtual = true; }
    ~Virt() { g_virtual = false; }
  } virt;
  std::vector<hodlr_s> A(nshapes);
  const int64_t* off = leaf_off;
  for (int i = 0; i < nshapes; ++i) {
    if (levels[i] < 0 || levels[i] > MAXGROUPS) return fail(HODLR_EINVAL, "bad levels");
    const int nl = 1 << levels[i];
    if (off[0] != 0 || off[nl] != n[i]) return fail(HODLR_EINVAL, "leaf_off must run from 0 to n");
    for (int j = 0; j < nl; ++j)
      if (off[j + 1] - off[j] < 1 || off[j + 1] - off[j] > MAXLEAF) return fail(HODLR_EINVAL, "bad leaf size");
    A[i].t.init(levels[i], off);
    A[i].cap = rank_cap;
    off += nl + 1;
  }
  std::vector<std::unique_ptr<hodlr_qr_s>> Fs;
  std::vector<std::vector<hodlr_qr_s*>> groups(nshapes);
  for (int i = 0; i < nshapes; ++i)
    for (int c = 0; c < count; ++c) {
      Fs.emplace_back();
      TRY(make_storage(A[i], 1e-10, (flags & HODLR_CHECK_ESTIMATE) ? 0.0 : 1.0, nullptr, Fs.back()));
      groups[i].push_back(Fs.back().get());
    }
  std::shared_ptr<Batch> B;
  if (nshapes == 1) {
    TRY(make_batch(groups[0], nullptr, B, (flags & HODLR_CHECK_PLANT) ? 1 : 0));
  } else {
    std::vector<Plan> plans(nshapes);
    std::vector<const Plan*> pp;
    for (int i = 0; i < nshapes; ++i) {
      build_plan(groups[i], plans[i]);
      pp.push_back(&plans[i]);
    }
    B = std::make_shared<Batch>();
    merge_plans(pp, B->plan, (flags & HODLR_CHECK_PLANT) != 0);
    TRY(finish_batch(*B, nullptr));
  }
  Plan& P = B->plan;
  if (flags & HODLR_QR_ONE_STREAM)
    for (Op& o : P.ops) o.lane = 0;
  CheckCtx C;
  C.cap = rank_cap;
  C.work = &B->work;
  for (auto& F : Fs) {
    C.blocks[F->up.dview] = &F->up.hview;
    C.blocks[F->lo.dview] = &F->lo.hview;
    C.blocks[F->tup.dview] = &F->tup.hview;
    C.leaves[F->leaves.dview] = &F->leaves.hview;
    C.leaves[F->tleaves.dview] = &F->tleaves.hview;
  }
  const CheckResult R = check_plan(P, C);
  stats[0] = R.ops;
  stats[1] = R.lane1_ops;
  stats[2] = R.pairs;
  stats[3] = R.conflicts;
  stats[4] = R.intra_conflicts;
  if (msg != nullptr && msglen > 0) {
    std::strncpy(msg, R.first.c_str(), (size_t)msglen - 1);
    msg[msglen - 1] = '\0';
  }
  return HODLR_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- launch-shape table
#include "tune_table.h"

namespace hqh {
namespace {
std::mutex g_tune_mu;
bool g_tune_override = false;
Tuning g_tune;
}  // namespace

Tuning tuning_for(int64_t n, int cap) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_tune_override) return g_tune;
  const TuneRow* row = &kTuneTable[sizeof(kTuneTable) / sizeof(kTuneTable[0]) - 1];
  for (const TuneRow& r : kTuneTable)
    if (n <= r.n_max && cap <= r.cap_max) {
      row = &r;
      break;
    }
  Tuning t;
  t.mm_rt64_rows = row->mm_rt64_rows;
  t.tr_small_chunks = row->tr_small_chunks;
  return t;
}
}  // namespace hqh

extern "C" {

hodlr_status hodlr_tuning(int64_t n, int32_t rank_cap, hodlr_tuning_t* out) {
  hqh::g_err.clear();
  if (out == nullptr || n < 1 || rank_cap < 1) return hqh::fail(HODLR_EINVAL, "bad argument");
  const hqh::Tuning t = hqh::tuning_for(n, rank_cap);
  out->mm_rt64_rows = t.mm_rt64_rows;
  out->tr_small_chunks = t.tr_small_chunks;
  return HODLR_OK;
}

hodlr_status hodlr_set_tuning(const hodlr_tuning_t* t) {
  hqh::g_err.clear();
  std::lock_guard<std::mutex> lk(hqh::g_tune_mu);
  if (t == nullptr) {
    hqh::g_tune_override = false;
    return HODLR_OK;
  }
  if (t->mm_rt64_rows < 0 || t->tr_small_chunks < 1 || t->tr_small_chunks > hq::TRS_MAXCH)
    return hqh::fail(HODLR_EINVAL, "tuning out of range");
  hqh::g_tune.mm_rt64_rows = t->mm_rt64_rows;
  hqh::g_tune.tr_small_chunks = t->tr_small_chunks;
  hqh::g_tune_override = true;
  return HODLR_OK;
}

}  // extern "C"

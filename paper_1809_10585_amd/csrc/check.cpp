// Hazard checker of a factorisation schedule.  The scheduler issues the
// T-factor steps of every node on a second stream beside the main chain,
// ordered against it only by the plan's signal / wait events; every launch
// also carries many independent jobs.  From the jobs' descriptors this file
// derives the byte ranges each launch reads and writes (ranks taken at their
// capacity) and reports
//  * pairs of launches that the two streams may run at the same time where
//    one writes bytes the other reads or writes, and
//  * pairs of jobs inside one launch with the same kind of overlap.
// Runs on the host only; with virtual addresses (hodlr_plan_check) it needs
// no device.
#include "plan.h"

#include <algorithm>
#include <array>
#include <cstdio>

namespace hqh {
namespace {

struct Iv {
  uintptr_t lo, hi;  // bytes [lo, hi)
  int job;
};

struct Acc {
  std::vector<Iv> r, w;
};

// a column-major block of doubles: `cols` columns of `rows` entries, `ld` apart
void add_block(std::vector<Iv>& v, const void* base, int64_t ld, int64_t rows, int64_t cols, int job) {
  if (base == nullptr || rows <= 0 || cols <= 0) return;
  const uintptr_t b = (uintptr_t)base;
  if (cols == 1 || ld == rows) {
    v.push_back({b, b + 8 * (uintptr_t)((cols - 1) * ld + rows), job});
    return;
  }
  for (int64_t c = 0; c < cols; ++c)
    v.push_back({b + 8 * (uintptr_t)(c * ld), b + 8 * (uintptr_t)(c * ld + rows), job});
}

void add_bytes(std::vector<Iv>& v, const void* p, size_t bytes, int job) {
  if (p != nullptr && bytes > 0) v.push_back({(uintptr_t)p, (uintptr_t)p + bytes, job});
}

// sort by start and merge the overlapping intervals of the same job
void normalize(std::vector<Iv>& v, bool keep_jobs) {
  if (!keep_jobs) {
    std::sort(v.begin(), v.end(), [](const Iv& a, const Iv& b) { return a.lo < b.lo; });
    std::vector<Iv> out;
    for (const Iv& x : v) {
      if (!out.empty() && x.lo <= out.back().hi) {
        out.back().hi = std::max(out.back().hi, x.hi);
      } else {
        out.push_back({x.lo, x.hi, -1});
      }
    }
    v.swap(out);
    return;
  }
  // per job: merge that job's own overlapping intervals
  std::stable_sort(v.begin(), v.end(), [](const Iv& a, const Iv& b) { return a.job < b.job; });
  std::vector<Iv> out;
  size_t i = 0;
  while (i < v.size()) {
    size_t j = i;
    while (j < v.size() && v[j].job == v[i].job) ++j;
    std::sort(v.begin() + i, v.begin() + j, [](const Iv& a, const Iv& b) { return a.lo < b.lo; });
    const size_t start = out.size();
    for (size_t q = i; q < j; ++q) {
      if (out.size() > start && v[q].lo <= out.back().hi)
        out.back().hi = std::max(out.back().hi, v[q].hi);
      else
        out.push_back(v[q]);
    }
    i = j;
  }
  std::sort(out.begin(), out.end(), [](const Iv& a, const Iv& b) { return a.lo < b.lo; });
  v.swap(out);
}

// first overlap of two merged, sorted interval lists
bool overlap(const std::vector<Iv>& a, const std::vector<Iv>& b, uintptr_t* at) {
  size_t i = 0, j = 0;
  while (i < a.size() && j < b.size()) {
    if (a[i].hi <= b[j].lo) {
      ++i;
    } else if (b[j].hi <= a[i].lo) {
      ++j;
    } else {
      *at = std::max(a[i].lo, b[j].lo);
      return true;
    }
  }
  return false;
}

struct Ctx {
  const Plan& P;
  const CheckCtx& C;
};

const std::vector<HBlk>* blocks_of(const CheckCtx& C, const HBlk* d) {
  auto it = C.blocks.find(d);
  return it == C.blocks.end() ? nullptr : it->second;
}
const std::vector<HLeaf>* leaves_of(const CheckCtx& C, const HLeaf* d) {
  auto it = C.leaves.find(d);
  return it == C.leaves.end() ? nullptr : it->second;
}

void tr_job(const Ctx& X, const TrJob& J, int job, Acc& a) {
  const int cap = J.cap;
  for (int s = 0; s < 2; ++s) {
    for (int b = 0; b < 2; ++b) {
      const Seg& g = J.seg[s][b];
      if (g.p == nullptr) continue;
      add_block(a.r, g.p, g.ld, J.side[s].m, g.ncols_dev ? cap : g.ncols, job);
      add_bytes(a.r, g.ncols_dev, sizeof(int), job);
    }
    add_block(a.w, J.out[s], J.ldout[s], J.side[s].m, cap, job);
  }
  add_bytes(a.w, J.out_rank, sizeof(int), job);
  add_bytes(a.w, J.log, 2 * sizeof(int), job);
  add_bytes(a.r, J.tau, sizeof(double), job);
}

// rows [r0, r1) of the subtree of heap node v (levels L) from its leaves
void subtree_rows(const std::vector<HLeaf>& lv, int L, int v, int64_t& r0, int64_t& rows, int& first, int& cnt) {
  const int d = 31 - __builtin_clz(v);
  first = (v << (L - d)) - (1 << L);
  cnt = 1 << (L - d);
  r0 = lv[first].r0;
  const HLeaf& last = lv[first + cnt - 1];
  rows = last.r0 + last.m - r0;
}

void mm_job(const Ctx& X, const MmJob& J, int job, int type, Acc& a) {
  const std::vector<HLeaf>* lv = leaves_of(X.C, J.M.leaf);
  if (lv == nullptr) return;
  const int L = J.M.levels;
  int64_t r0, rows;
  int first, cnt;
  subtree_rows(*lv, L, J.v, r0, rows, first, cnt);
  const int cols = J.s_dev ? X.C.cap : (J.s > 0 ? J.s : SMAX);
  const int cap = X.C.cap;
  if (J.xs < 0) add_block(a.r, J.X, J.ldX, rows, cols, job);
  add_bytes(a.r, J.s_dev, sizeof(int), job);
  if (type == OP_MMAPPLY && J.zs < 0) {
    add_block(a.w, J.Z, J.ldZ, rows, cols, job);
    if (J.beta != 0.0) add_block(a.r, J.Z, J.ldZ, rows, cols, job);
  }
  std::vector<int> nodes;
  struct W {
    static void go(int v, int L, std::vector<int>& out) {
      if ((31 - __builtin_clz(v)) >= L) return;
      out.push_back(v);
      go(2 * v, L, out);
      go(2 * v + 1, L, out);
    }
  };
  W::go(J.v, L, nodes);
  for (int kind = 0; kind < 2; ++kind) {
    const HBlk* arr = kind == 0 ? J.M.up : J.M.lo;
    if (arr == nullptr) continue;
    const std::vector<HBlk>* hb = blocks_of(X.C, arr);
    if (hb == nullptr) continue;
    for (int u : nodes) {
      const HBlk& b = (*hb)[u];
      add_block(a.r, b.U, b.ldU, b.rows, cap, job);
      add_block(a.r, b.V, b.ldV, b.cols, cap, job);
      add_bytes(a.r, b.rank, sizeof(int), job);
    }
  }
  if (type == OP_MMAPPLY)
    for (int j = first; j < first + cnt; ++j) {
      const HLeaf& f = (*lv)[j];
      add_block(a.r, f.D, f.ld, f.m, f.m, job);
    }
}

void gemm_job(const Ctx& X, const GemmJob& J, int job, Acc& a) {
  const int cap = X.C.cap;
  const int M = J.Md ? cap : J.M;
  const int N = J.Nd ? cap : (J.N > 0 ? J.N : SMAX);
  const int K = J.Kd ? cap : J.K;
  if (J.as_ < 0) {
    if (J.ta)
      add_block(a.r, J.A, J.lda, K, M, job);
    else
      add_block(a.r, J.A, J.lda, M, K, job);
  }
  if (J.bs_ < 0) {
    if (J.tb)
      add_block(a.r, J.B, J.ldb, N, K, job);
    else
      add_block(a.r, J.B, J.ldb, K, N, job);
  }
  if (J.cs_ < 0) {
    add_block(a.w, J.C, J.ldc, M, N, job);
    if (J.beta != 0.0) add_block(a.r, J.C, J.ldc, M, N, job);
  }
  for (const int* p : {J.Md, J.Nd, J.Kd}) add_bytes(a.r, p, sizeof(int), job);
}

void leaf_job(const Ctx& X, const LeafJob& J, int job, int type, Acc& a) {
  const int m = J.m, cap = X.C.cap;
  if (type == OP_LGATHER) {
    add_block(a.r, J.D, m, m, m, job);
  } else if (type == OP_LSCATTER) {
    add_block(a.w, J.D, m, m, m, job);
    add_block(a.w, J.Tleaf, m, m, m, job);
  }
  // the leaf workspace (stacked column, T, Gram blocks)
  for (double* p : {J.ws.H}) {
    add_block(a.r, p, MAXSTACK, MAXSTACK, m, job);
    add_block(a.w, p, MAXSTACK, MAXSTACK, m, job);
  }
  for (double* p : {J.ws.T, J.ws.G}) {
    add_block(a.r, p, MAXLEAF, m, m, job);
    add_block(a.w, p, MAXLEAF, m, m, job);
  }
  for (int g = 0; g < J.ngroups; ++g) {
    const LeafGroup& G = J.g[g];
    add_bytes(a.r, G.rank, sizeof(int), job);
    if (type == OP_LGATHER) add_block(a.r, G.V + G.row0, G.ld, m, cap, job);
    if (type == OP_LSCATTER) add_block(a.w, G.V + G.row0, G.ld, m, cap, job);
  }
}

void vec_job(const VecJob& J, int job, int type, Acc& a) {
  if (type == OP_FILL) {
    add_block(a.w, J.x, J.n, J.n, 1, job);
  } else if (type == OP_NORMALIZE) {
    add_block(a.r, J.z, J.n, J.n, 1, job);
    if (J.x) add_block(a.w, J.x, J.n, J.n, 1, job);
    add_bytes(a.w, J.out, sizeof(double), job);
  } else if (type == OP_SETSCAL) {
    add_bytes(a.r, J.x, 3 * sizeof(double), job);
    add_bytes(a.w, J.x, 3 * sizeof(double), job);
  }
}

// the parts of the lane workspace and counters each job of a launch uses, from
// its offsets (checked against the other jobs of the launch; the schedule
// builder and the merging of schedules assign them)
void ws_jobs(const Ctx& X, const Op& o, Acc& a) {
  const Work* W = X.C.work;
  if (W == nullptr || W->ws == nullptr || W->counters == nullptr) return;
  const Plan& P = X.P;
  const double* ws = W->ws + P.ws_off(o.lane);
  const int* cnt = W->counters + P.cnt_off(o.lane);
  auto rw = [&](const void* p, size_t bytes, int job) {
    add_bytes(a.r, p, bytes, job);
    add_bytes(a.w, p, bytes, job);
  };
  // (tag: the job a chain's steps are reported as; they run in order)
  auto tr = [&](int j, int tag) {
    const TrJob& J = P.trj[j];
    rw(ws + J.hdr, TR_HDR * sizeof(double), tag);
    for (int s = 0; s < 2; ++s)
      if (J.side[s].p0 > 0) {
        rw(ws + J.side[s].node0, 2 * (size_t)J.side[s].p0 * TR_NODE * sizeof(double), tag);
        rw(cnt + J.side[s].cnt0, (size_t)J.side[s].p0 * sizeof(int), tag);
      }
    rw(cnt + J.jcounter, sizeof(int), tag);
  };
  auto mm = [&](int j) {
    const MmJob& J = P.mmj[j];
    const int d = 31 - __builtin_clz(J.v);
    const int64_t nodes = (2 << (J.M.levels - d)) - 1;
    rw(ws + J.red0, 2 * (size_t)nodes * J.rld * SMAX * sizeof(double), j);
  };
  switch (o.type) {
    case OP_TRSMALL:
    case OP_TRQR:
      for (int i = 0; i < o.count; ++i) tr(P.trc[o.first + i].job, P.trc[o.first + i].job);
      break;
    case OP_TRCHAIN:
      for (int i = 0; i < o.count; ++i) {
        const TrChunk& c = P.trc[o.first + i];
        for (int s = 0; s < c.chunk; ++s) tr(c.job + s, c.job);
      }
      break;
    case OP_TRFORM:
      for (int i = 0; i < o.count; ++i) tr(P.trf[o.first + i].job, P.trf[o.first + i].job);
      break;
    case OP_MMPROJ:
    case OP_MMRED:
      for (int i = 0; i < o.count; ++i) {
        const MmProj& pr = P.mmp[o.first + i];
        const size_t stride = (size_t)P.mmj[pr.job].rld * SMAX;
        const size_t n = o.type == OP_MMRED ? (size_t)pr.nchunk : 1;
        rw(ws + pr.part, n * stride * sizeof(double), pr.job);
        mm(pr.job);
      }
      break;
    case OP_MMAPPLY:
      for (int i = 0; i < o.count; ++i) mm(P.mma[o.first + i].job);
      break;
    case OP_GRED:
      for (int i = 0; i < o.count; ++i) {
        const GemmRed& r = P.gr[o.first + i];
        if (r.nchunk > 1) rw(ws + r.part, (size_t)KCAP * KCAP * sizeof(double), r.job);
        rw(cnt + r.counter, sizeof(int), r.job);
      }
      break;
    default:
      break;
  }
}

// accesses of one launch, per job (job = index within the launch)
Acc op_access(const Ctx& X, const Op& o) {
  Acc a;
  const Plan& P = X.P;
  std::vector<int> jobs;
  auto uniq = [&](std::vector<int>& v) {
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  };
  switch (o.type) {
    case OP_TRSMALL:
    case OP_TRQR:
      for (int i = 0; i < o.count; ++i) jobs.push_back(P.trc[o.first + i].job);
      uniq(jobs);
      for (int j : jobs) tr_job(X, P.trj[j], j, a);
      break;
    case OP_TRCHAIN:  // a chain's steps run in order: one job of the launch
      for (int i = 0; i < o.count; ++i) {
        const TrChunk& c = P.trc[o.first + i];
        for (int s = 0; s < c.chunk; ++s) tr_job(X, P.trj[c.job + s], c.job, a);
      }
      break;
    case OP_TRFORM:
      for (int i = 0; i < o.count; ++i) jobs.push_back(P.trf[o.first + i].job);
      uniq(jobs);
      for (int j : jobs) tr_job(X, P.trj[j], j, a);
      break;
    case OP_MMPROJ:
    case OP_MMRED:
      for (int i = 0; i < o.count; ++i) jobs.push_back(P.mmp[o.first + i].job);
      uniq(jobs);
      for (int j : jobs) mm_job(X, P.mmj[j], j, o.type, a);
      break;
    case OP_MMAPPLY:
      for (int i = 0; i < o.count; ++i) jobs.push_back(P.mma[o.first + i].job);
      uniq(jobs);
      for (int j : jobs) mm_job(X, P.mmj[j], j, o.type, a);
      break;
    case OP_GTALL:
      for (int i = 0; i < o.count; ++i) jobs.push_back(P.gt[o.first + i].job);
      uniq(jobs);
      for (int j : jobs) gemm_job(X, P.gj[j], j, a);
      break;
    case OP_GRED:
      for (int i = 0; i < o.count; ++i) jobs.push_back(P.gr[o.first + i].job);
      uniq(jobs);
      for (int j : jobs) gemm_job(X, P.gj[j], j, a);
      break;
    case OP_LGATHER:
    case OP_LPANEL:
    case OP_LUPDATE:
    case OP_LSCATTER: {
      const int nper = (int)std::max<int64_t>(1, o.n);
      for (int i = 0; i < o.count / nper; ++i) leaf_job(X, P.lj[o.first + i], o.first + i, o.type, a);
      break;
    }
    case OP_FILL:
    case OP_NORMALIZE:
    case OP_SETSCAL:
      for (int i = 0; i < o.count; ++i) vec_job(P.vj[o.first + i], o.first + i, o.type, a);
      break;
    default:
      break;
  }
  ws_jobs(X, o, a);
  // workspace and counters of the op's lane (shared by all its jobs)
  const Work* W = X.C.work;
  const bool uses_ws = o.type == OP_TRSMALL || o.type == OP_TRQR || o.type == OP_TRCHAIN || o.type == OP_TRFORM ||
                       o.type == OP_MMPROJ ||
                       o.type == OP_MMRED || o.type == OP_MMAPPLY || o.type == OP_GRED;
  if (W != nullptr && uses_ws && W->ws != nullptr) {
    const int64_t sz = P.ws_lane[o.lane];
    add_bytes(a.r, W->ws + P.ws_off(o.lane), (size_t)sz * sizeof(double), -2);
    add_bytes(a.w, W->ws + P.ws_off(o.lane), (size_t)sz * sizeof(double), -2);
  }
  const bool uses_cnt = o.type == OP_TRSMALL || o.type == OP_TRQR || o.type == OP_TRCHAIN || o.type == OP_GRED;
  if (W != nullptr && uses_cnt && W->counters != nullptr) {
    const int sz = P.cnt_lane[o.lane];
    add_bytes(a.r, W->counters + P.cnt_off(o.lane), (size_t)sz * sizeof(int), -2);
    add_bytes(a.w, W->counters + P.cnt_off(o.lane), (size_t)sz * sizeof(int), -2);
  }
  return a;
}

// conflicting job pairs inside one launch (the shared lane workspace, job -2,
// is excluded: its jobs use disjoint parts of it by construction)
int64_t intra_conflicts(Acc a, std::string* first, int opi, int type) {
  auto drop_shared = [](std::vector<Iv>& v) {
    v.erase(std::remove_if(v.begin(), v.end(), [](const Iv& x) { return x.job == -2; }), v.end());
  };
  drop_shared(a.r);
  drop_shared(a.w);
  normalize(a.w, true);
  normalize(a.r, true);
  int64_t n = 0;
  auto report = [&](uintptr_t at, int j1, int j2) {
    ++n;
    if (first != nullptr && first->empty()) {
      char buf[256];
      std::snprintf(buf, sizeof(buf), "launch %d (%s): jobs %d and %d overlap at 0x%llx", opi, OP_NAMES[type], j1,
                    j2, (unsigned long long)at);
      *first = buf;
    }
  };
  // writes of different jobs (each job's own writes are disjoint after merging)
  uintptr_t maxhi = 0;
  int maxjob = -1;
  for (const Iv& x : a.w) {
    if (maxjob >= 0 && x.lo < maxhi && x.job != maxjob) report(x.lo, maxjob, x.job);
    if (x.hi > maxhi) {
      maxhi = x.hi;
      maxjob = x.job;
    }
  }
  // reads against other jobs' writes
  for (const Iv& x : a.r) {
    auto it = std::lower_bound(a.w.begin(), a.w.end(), x.lo, [](const Iv& w, uintptr_t lo) { return w.hi <= lo; });
    for (; it != a.w.end() && it->lo < x.hi; ++it)
      if (it->job != x.job && it->hi > x.lo) {
        report(std::max(x.lo, it->lo), it->job, x.job);
        break;
      }
  }
  return n;
}

}  // namespace

CheckResult check_plan(const Plan& P, const CheckCtx& C) {
  CheckResult R;
  Ctx X{P, C};
  const int nops = (int)P.ops.size();
  // vector clocks: clk[i] = (ops of lane 0, ops of lane 1) complete before op i starts
  std::vector<std::array<int64_t, 2>> clk(nops);
  std::vector<int64_t> idx(nops, -1);  // position of op i within its lane
  std::vector<std::array<int64_t, 2>> ev(P.n_events + 1, {0, 0});
  std::array<std::array<int64_t, 2>, 2> vc = {{{0, 0}, {0, 0}}};  // per lane
  std::vector<int> lane_ops[2];
  for (int i = 0; i < nops; ++i) {
    const Op& o = P.ops[i];
    const int l = o.lane;
    if (o.type == OP_SIGNAL) {
      ev[o.a0] = vc[l];
      continue;
    }
    if (o.type == OP_WAIT) {
      for (int q = 0; q < 2; ++q)
        if (q != l) vc[l][q] = std::max(vc[l][q], ev[o.a0][q]);
      continue;
    }
    if (!op_launches(o)) continue;
    clk[i] = vc[l];
    idx[i] = vc[l][l];
    vc[l][l] += 1;
    lane_ops[l].push_back(i);
  }
  R.ops = (int64_t)(lane_ops[0].size() + lane_ops[1].size());
  R.lane1_ops = (int64_t)lane_ops[1].size();
  // accesses, merged per launch
  std::vector<Acc> acc(nops);
  for (int l = 0; l < 2; ++l)
    for (int i : lane_ops[l]) {
      Acc a = op_access(X, P.ops[i]);
      R.intra_conflicts += intra_conflicts(a, &R.first, i, P.ops[i].type);
      normalize(a.r, false);
      normalize(a.w, false);
      acc[i] = std::move(a);
    }
  // lane-1 op y against the lane-0 ops it is unordered with: x = lane_ops[0][ia]
  // with ia >= clk[y][0] (not known complete before y) and clk[x][1] <= idx[y]
  // (x does not know y complete); the second bound is monotone along lane 0
  const std::vector<int>& L0 = lane_ops[0];
  for (int y : lane_ops[1]) {
    const int64_t lo = clk[y][0];
    for (int64_t ia = lo; ia < (int64_t)L0.size(); ++ia) {
      const int x = L0[ia];
      if (clk[x][1] > idx[y]) break;
      ++R.pairs;
      uintptr_t at = 0;
      const bool c = overlap(acc[x].w, acc[y].r, &at) || overlap(acc[x].w, acc[y].w, &at) ||
                     overlap(acc[y].w, acc[x].r, &at);
      if (c) {
        ++R.conflicts;
        if (R.first.empty()) {
          char buf[256];
          std::snprintf(buf, sizeof(buf), "launch %d (%s, stream 1) and launch %d (%s, stream 0) overlap at 0x%llx", y,
                        OP_NAMES[P.ops[y].type], x, OP_NAMES[P.ops[x].type], (unsigned long long)at);
          R.first = buf;
        }
      }
    }
  }
  return R;
}

}  // namespace hqh

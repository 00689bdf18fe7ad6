// Heterogeneous batched execution (task list + persistent kernel), plans,
// hipGraph capture and the in-house schedule autotuner.
#include "hk_batch.hpp"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <string>
#include <vector>

namespace hk {

static bool dbl(hk_dtype_t dt) { return dt == HK_C128 || dt == HK_F64; }

static Status hip_fail(hipError_t e, const char *what) {
  return fail(HK_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace hk

struct hk_plan_s {
  hk_dtype_t dt = HK_C64;
  unsigned flags = 0;
  int64_t count = 0;
  std::vector<hk::Shape> shapes;
  std::vector<hk::Ptrs> ptrs;  // ws holds the offset of the instance region
  std::vector<hk::Task> tasks;
  std::vector<int32_t> res_list;
  int32_t phase_end[3] = {0, 0, 0};  // [0, e0): pass A + resident, [e0, e1): pass B, [e1, e2): pass D
  size_t ctl_bytes = 0;              // BatchCtl
  size_t tables_bytes = 0;           // descriptor tables (when stored in the workspace)
  size_t inst_bytes = 0;             // instance regions
  bool tables_in_ws = false;
  // device copies of the tables (plan-owned) or offsets inside the workspace
  char *d_tables = nullptr;
  size_t off_shapes = 0, off_ptrs = 0, off_tasks = 0, off_res = 0, off_order = 0;
  // grouped launches: task indices sorted by (phase, kind, length) and the
  // launch list over them
  struct Group {
    int kind, logL, odd, phase;
    int32_t begin, count;
  };
  std::vector<int32_t> order;
  std::vector<Group> launches;
  std::vector<char> host_tables;
  // grouped launches of one phase are independent: they are spread over the
  // caller's stream and these (created on first use, default priority),
  // forked from and joined back into the caller's stream by events
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> fork_ev, join_ev;
  int grid = 1;
  bool persistent = true;
  uint32_t wait_bound = 1u << 22;  // barrier polling iterations before the error path
  // graph
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  void *graph_ws = nullptr;
  hipStream_t graph_stream = nullptr;
  // status
  hipStream_t last_stream = nullptr;
  void *last_ws = nullptr;
  // HK_PLAN_AUTOTUNE: the problems (to rebuild the plan), the length buckets
  // (log2 of the power-of-two length >= d_H) forced to powers of two, the
  // workspace every candidate fits in, and whether the first execute has tuned
  std::vector<hk_problem_t> probs;
  uint32_t pow2_buckets = 0;
  uint32_t no5_buckets = 0;  // length buckets built without the factor 5
  size_t tune_ws_bytes = 0;
  bool tuned = false;
  double tune_ms_default = 0.0, tune_ms_best = 0.0;
};

namespace hk {

static void tables_layout(hk_plan_s *p) {
  size_t off = 0;
  p->off_shapes = off;
  off = align256(off + sizeof(Shape) * p->shapes.size());
  p->off_ptrs = off;
  off = align256(off + sizeof(Ptrs) * p->ptrs.size());
  p->off_tasks = off;
  off = align256(off + sizeof(Task) * std::max<size_t>(1, p->tasks.size()));
  p->off_res = off;
  off = align256(off + sizeof(int32_t) * std::max<size_t>(1, p->res_list.size()));
  p->off_order = off;
  off = align256(off + sizeof(int32_t) * std::max<size_t>(1, p->order.size()));
  p->tables_bytes = off;
  p->host_tables.assign(off, 0);
  memcpy(p->host_tables.data() + p->off_shapes, p->shapes.data(), sizeof(Shape) * p->shapes.size());
  memcpy(p->host_tables.data() + p->off_ptrs, p->ptrs.data(), sizeof(Ptrs) * p->ptrs.size());
  if (!p->tasks.empty()) memcpy(p->host_tables.data() + p->off_tasks, p->tasks.data(), sizeof(Task) * p->tasks.size());
  if (!p->res_list.empty())
    memcpy(p->host_tables.data() + p->off_res, p->res_list.data(), sizeof(int32_t) * p->res_list.size());
  if (!p->order.empty())
    memcpy(p->host_tables.data() + p->off_order, p->order.data(), sizeof(int32_t) * p->order.size());
}

// Sorts each phase's tasks by (kind, transform length, odd factor of the row
// kernels) and records one launch per run of equal keys.
static void build_groups(hk_plan_s *p) {
  p->order.clear();
  p->launches.clear();
  int32_t b = 0;
  for (int ph = 0; ph < 3; ++ph) {
    const int32_t e = p->phase_end[ph];
    std::vector<std::pair<std::tuple<int, int, int>, int32_t>> keyed;
    for (int32_t i = b; i < e; ++i) {
      const Task &t = p->tasks[i];
      int kind, logL, odd = 1;
      if (t.type == TASK_RES) {
        kind = GK_RES;
        const Shape &rs = p->shapes[p->res_list[t.inst]];
        logL = rs.logR;
        odd = rs.r2c ? 2 : rs.odd;  // 2: real-input rows
      } else if (t.type == TASK_ROWB) {
        kind = GK_ROWB;
        logL = p->shapes[t.inst].logR;
        odd = p->shapes[t.inst].r2c ? 2 : p->shapes[t.inst].odd;  // 2: real-input row pairs
      } else if (t.type == TASK_ALPHA) {
        kind = GK_ALPHA;
        logL = 0;
      } else {
        kind = GK_COL;
        logL = p->shapes[t.inst].logC;
        odd = p->shapes[t.inst].r2c ? 2 : p->shapes[t.inst].odd;  // 2: real arrays as pairs
      }
      keyed.push_back({std::make_tuple(kind, logL, odd), i});
    }
    // longest transforms first within a phase
    std::stable_sort(keyed.begin(), keyed.end(), [](const auto &x, const auto &y) {
      const int kx = std::get<0>(x.first), ky = std::get<0>(y.first);
      if (kx != ky) return kx < ky;
      const int lx = std::get<1>(x.first), ly = std::get<1>(y.first);
      if (lx != ly) return lx > ly;
      return std::get<2>(x.first) > std::get<2>(y.first);
    });
    for (size_t k = 0; k < keyed.size(); ++k) {
      if (k == 0 || keyed[k].first != keyed[k - 1].first)
        p->launches.push_back({std::get<0>(keyed[k].first), std::get<1>(keyed[k].first), std::get<2>(keyed[k].first),
                               ph, (int32_t)p->order.size(), 0});
      p->order.push_back(keyed[k].second);
      p->launches.back().count++;
    }
    b = e;
  }
}

static Problem problem_of(hk_dtype_t dt, const hk_problem_t &q) {
  Problem p;
  p.dt = dt;
  p.prog = PROG_FWD;
  p.is_block = q.is_block != 0;
  p.m = q.m;
  for (int i = 0; i < HK_MAX_ORDER && i < q.m; ++i) {
    p.dims[i] = q.dims[i];
    p.bdims[i] = q.block_dims[i];
    p.vec[i] = q.vectors[i];
  }
  if (!q.alpha) p.vec[0] = nullptr;
  p.h = q.h;
  p.y = q.y;
  p.alpha = q.alpha;
  return p;
}

// log2 of the power-of-two transform length of a 1D problem (its length bucket).
static int length_bucket(const Problem &pr) {
  int64_t dh = 1 - pr.m;
  for (int q = 0; q < pr.m; ++q) dh += pr.dims[q];
  return ceil_log2(dh);
}

static Status plan_build(hk_plan_t *out, hk_dtype_t dt, const hk_problem_t *probs, int64_t count, unsigned flags,
                         uint32_t pow2_buckets, uint32_t no5_buckets = 0);

Status plan_create(hk_plan_t *out, hk_dtype_t dt, const hk_problem_t *probs, int64_t count, unsigned flags) {
  Status s = plan_build(out, dt, probs, count, flags, 0);
  if (!s.ok() || !(flags & HK_PLAN_AUTOTUNE) || (flags & (HK_PLAN_PERSISTENT | HK_PLAN_GRAPH))) return s;
  // The tuner may build any length bucket with powers of two or without the
  // factor 5: every instance of a candidate takes the layout it has in one of
  // the default, all-powers-of-two and all-without-5 plans, so the workspace
  // holds, per instance, the largest of the three, and the three plans'
  // tables together.
  hk_plan_s *p = *out;
  hk_plan_t all = nullptr, no5 = nullptr;
  s = plan_build(&all, dt, probs, count, flags, ~0u, 0);
  if (s.ok()) s = plan_build(&no5, dt, probs, count, flags, 0, ~0u);
  if (!s.ok()) {
    delete all;
    delete p;
    *out = nullptr;
    return s;
  }
  size_t inst = 0;
  for (int64_t i = 0; i < count; ++i)
    inst += align256(std::max({instance_ws_bytes(p->shapes[i], dt), instance_ws_bytes(all->shapes[i], dt),
                               instance_ws_bytes(no5->shapes[i], dt)}));
  p->tune_ws_bytes = p->ctl_bytes + p->tables_bytes + all->tables_bytes + no5->tables_bytes + inst;
  delete all;
  delete no5;
  p->probs.assign(probs, probs + count);
  return Status();
}

static Status plan_build(hk_plan_t *out, hk_dtype_t dt, const hk_problem_t *probs, int64_t count, unsigned flags,
                         uint32_t pow2_buckets, uint32_t no5_buckets) {
  if (!out) return fail(HK_ERR_NULL_POINTER, "plan pointer is NULL");
  *out = nullptr;
  if (count < 0) return fail(HK_ERR_INVALID_VALUE, "count must be >= 0");
  if (count > 0 && !probs) return fail(HK_ERR_NULL_POINTER, "problems is NULL");
  if (count > (1 << 24)) return fail(HK_ERR_SIZE_LIMIT, "too many problems in one plan");
  if (flags & ~(unsigned)(HK_PLAN_PERSISTENT | HK_PLAN_MULTIKERNEL | HK_PLAN_GRAPH | HK_PLAN_AUTOTUNE | HK_PLAN_POW2))
    return fail(HK_ERR_INVALID_VALUE, "unknown plan flags");
  if ((flags & HK_PLAN_PERSISTENT) && (flags & HK_PLAN_MULTIKERNEL))
    return fail(HK_ERR_INVALID_VALUE, "PERSISTENT and MULTIKERNEL are exclusive");
  if (dt < HK_C64 || dt > HK_F64) return fail(HK_ERR_INVALID_VALUE, "unknown dtype");
  hk_plan_s *p = new hk_plan_s();
  p->dt = dt;
  p->flags = flags;
  p->count = count;
  p->persistent = (flags & HK_PLAN_PERSISTENT) != 0;
  p->pow2_buckets = pow2_buckets;
  p->no5_buckets = no5_buckets;
  int blk, er, ec;
  size_t lds;
  if (dbl(dt))
    batch_geometry_f64(&blk, &er, &ec, &lds);
  else
    batch_geometry_f32(&blk, &er, &ec, &lds);
  auto tps = [&](int logL, int E) {
    KernelLimits k;
    if (dbl(dt))
      limits_f64(logL, E, &k);
    else
      limits_f32(logL, E, &k);
    return k.tps;
  };
  // lanes of one row of the batched row kernels (odd-factor rows hold
  // odd_row_e elements per lane)
  const int e_odd = dbl(dt) ? odd_row_e_f64() : odd_row_e_f32();
  auto row_tps = [&](const Shape &sh) {
    KernelLimits k;
    if (sh.r2c && sh.resident) {
      if (dbl(dt))
        limits_r2c_f64(sh.logR, r2c_row_e_f64(), &k);
      else
        limits_r2c_f32(sh.logR, r2c_row_e_f32(), &k);
      return k.tps;
    }
    if (sh.r2c) {  // row pairs
      if (dbl(dt))
        limits_r2cp_f64(sh.logR, r2c_row_e_f64(), &k);
      else
        limits_r2cp_f32(sh.logR, r2c_row_e_f32(), &k);
      return k.tps;
    }
    if (sh.odd > 1) {
      if (!sh.resident) {  // grouped pass-B rows (GroupRowbE elements per lane)
        const int t = dbl(dt) ? group_rowb_tps_f64(sh.odd, sh.logR) : group_rowb_tps_f32(sh.odd, sh.logR);
        return std::max(1, t);
      }
      row_limits(dt, sh.odd, sh.logR, e_odd, &k);
      return k.tps;
    }
    // grouped pass-B rows take 4 elements per lane up to 2048 points
    if (!sh.resident && !p->persistent && sh.logR <= 11) return tps(sh.logR, 4);
    return tps(sh.logR, er);
  };
  // First virtual columns (sequence * R + storage column) of the column tiles
  // of a transform with `ncols` storage columns per sequence.
  auto col_tiles = [&](const Shape &sh, int64_t ncols, int tw) {
    std::vector<int64_t> v;
    const int64_t R = (int64_t)1 << sh.logR;
    if (sh.odd == 1 || tw > R) {
      const int64_t nv = sh.odd == 1 ? ncols : sh.odd * R;
      for (int64_t c0 = 0; c0 < nv; c0 += tw) v.push_back(c0);
    } else {
      for (int q = 0; q < sh.odd; ++q)
        for (int64_t c0 = 0; c0 < ncols; c0 += tw) v.push_back(q * R + c0);
    }
    return v;
  };
  const bool allow_odd = !p->persistent && !(flags & HK_PLAN_POW2);
  p->shapes.resize(count);
  p->ptrs.resize(count);
  p->ctl_bytes = align256(sizeof(BatchCtl));
  size_t inst_off = 0;
  struct Inst {
    int64_t idx;
    double cost;
  };
  std::vector<Inst> multi;
  std::map<std::tuple<int, int, int, int, int, int>, std::vector<int32_t>> groups;
  for (int64_t i = 0; i < count; ++i) {
    Problem pr = problem_of(dt, probs[i]);
    Status s = validate_forward(pr);
    if (!s.ok()) {
      delete p;
      return fail(s.code, "problem " + std::to_string(i) + ": " + s.msg);
    }
    Layout lay;
    const int bucket = std::min(31, length_bucket(pr));
    const bool forced = !pr.is_block && ((pow2_buckets >> bucket) & 1u);
    const bool no5 = !pr.is_block && ((no5_buckets >> bucket) & 1u);
    // the grouped and persistent kernels run BHHB on power-of-two grids
    s = layout_for(pr, 0, &lay, allow_odd && !forced && !pr.is_block, count, no5 ? F5_NONE : F5_RESIDENT);
    if (!s.ok()) {
      delete p;
      return fail(s.code, "problem " + std::to_string(i) + ": " + s.msg);
    }
    Sched sc;
    Shape sh;
    Ptrs P;
    build_shape(pr, lay, sc, &sh, &P, nullptr);
    if (!lay.resident) {
      sh.rows_per_wg = std::max(1, blk / row_tps(sh));
      P.ws = (void *)(uintptr_t)inst_off;
      inst_off += align256((size_t)sh.ws_bytes);
      multi.push_back({i, (double)((int64_t)sh.odd << (sh.logR + sh.logC)) * (sh.nops + 1)});
    } else {
      P.ws = nullptr;
      groups[std::make_tuple(sh.logR, sh.r2c ? 2 : sh.odd, sh.nops, sh.want_y, sh.want_alpha, sh.real_out)].push_back(
          (int32_t)i);
    }
    p->shapes[i] = sh;
    p->ptrs[i] = P;
  }
  p->inst_bytes = inst_off;
  std::sort(multi.begin(), multi.end(), [](const Inst &a, const Inst &b) { return a.cost > b.cost; });
  // Phase 1a: pass A of the multipass instances (largest first).
  std::vector<int32_t> nrowb(count, 0);
  for (const Inst &in : multi) {
    const Shape &sh = p->shapes[in.idx];
    const int tw = std::max(1, blk / tps(sh.logC, ec));
    for (int o = 0; o < sh.nops; ++o)
      for (int64_t c0 : col_tiles(sh, sh.ops[o].ncol_nz, tw)) {
        Task t = {TASK_COLA, (int32_t)in.idx, o, (int32_t)c0, 0};
        p->tasks.push_back(t);
      }
  }
  // Phase 1b: resident instances, grouped so that a workgroup's rows share
  // their control flow; groups of long transforms first.
  std::vector<std::pair<int, std::vector<int32_t> *>> gl;
  for (auto &kv : groups)
    gl.push_back({(std::get<0>(kv.first) * 8 + std::get<1>(kv.first)) * 16 + std::get<2>(kv.first), &kv.second});
  std::sort(gl.begin(), gl.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
  for (auto &g : gl) {
    const Shape &sh0 = p->shapes[(*g.second)[0]];
    const int rows = std::max(1, blk / row_tps(sh0));
    for (size_t k = 0; k < g.second->size(); k += rows) {
      const int n = (int)std::min<size_t>(rows, g.second->size() - k);
      Task t = {TASK_RES, (int32_t)p->res_list.size(), n, 0, 0};
      for (int j = 0; j < n; ++j) p->res_list.push_back((*g.second)[k + j]);
      p->tasks.push_back(t);
    }
  }
  p->phase_end[0] = (int32_t)p->tasks.size();
  // Phase 2: pass B.
  for (const Inst &in : multi) {
    const Shape &sh = p->shapes[in.idx];
    const int rows = std::max(1, blk / row_tps(sh));
    const int64_t C = (int64_t)1 << sh.logC;
    const int64_t brows = sh.r2c ? C / 2 : C;  // real inputs: mirrored row pairs
    const int32_t nb = (int32_t)((brows + rows - 1) / rows);
    for (int32_t b = 0; b < nb; ++b) {
      Task t = {TASK_ROWB, (int32_t)in.idx, (int32_t)(b * rows), b, nb};
      p->tasks.push_back(t);
    }
    nrowb[in.idx] = nb;
  }
  p->phase_end[1] = (int32_t)p->tasks.size();
  // Phase 3: scalar products (sums of the pass-B partials) and pass D.
  for (const Inst &in : multi) {
    const Shape &sh = p->shapes[in.idx];
    if (!sh.want_alpha) continue;
    Task t = {TASK_ALPHA, (int32_t)in.idx, 0, 0, nrowb[in.idx]};
    p->tasks.push_back(t);
  }
  for (const Inst &in : multi) {
    const Shape &sh = p->shapes[in.idx];
    if (!sh.want_y) continue;
    const int tw = std::max(1, blk / tps(sh.logC, ec));
    const int64_t ncols = std::min<int64_t>((int64_t)1 << sh.logR, sh.r2c ? (sh.out_rows + 1) / 2 : sh.out_rows);
    for (int64_t c0 : col_tiles(sh, ncols, tw)) {
      Task t = {TASK_COLD, (int32_t)in.idx, 0, (int32_t)c0, 0};
      p->tasks.push_back(t);
    }
  }
  p->phase_end[2] = (int32_t)p->tasks.size();
  build_groups(p);
  tables_layout(p);
  int dev = 0, ncu = 256;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    ncu = prop.multiProcessorCount;
  // The persistent kernel's phases end in grid-wide barriers, so every one of
  // its workgroups must be resident at once: the grid is what the occupancy
  // of the kernel allows on this device (and no more than the largest phase).
  int per_cu = 1;
  if ((dbl(dt) ? batch_resident_f64(&per_cu) : batch_resident_f32(&per_cu)) != hipSuccess || per_cu < 1) per_cu = 1;
  int64_t widest = 1;
  for (int ph = 0, b = 0; ph < 3; b = p->phase_end[ph++]) widest = std::max<int64_t>(widest, p->phase_end[ph] - b);
  p->grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)ncu * per_cu, widest));
  *out = p;
  return Status();
}

Status plan_ws_size(hk_plan_t p, size_t *bytes) {
  if (!p) return fail(HK_ERR_NULL_POINTER, "plan is NULL");
  if (!bytes) return fail(HK_ERR_NULL_POINTER, "bytes is NULL");
  // Room for the descriptor tables is always reserved so that one-shot
  // execution can keep them in the workspace.
  *bytes = std::max(p->ctl_bytes + p->tables_bytes + p->inst_bytes, p->tune_ws_bytes);
  return Status();
}

static Status upload_tables(hk_plan_s *p) {
  if (p->d_tables) return Status();
  hipError_t e = hipMalloc((void **)&p->d_tables, p->tables_bytes);
  if (e != hipSuccess) return hip_fail(e, "plan table allocation");
  e = hipMemcpy(p->d_tables, p->host_tables.data(), p->tables_bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "plan table upload");
  return Status();
}

// Streams a grouped plan spreads each phase's launches over (the caller's
// stream included); four matches the hardware queues a process gets by default.
constexpr int kGroupStreams = 4;

static Status ensure_streams(hk_plan_s *p, int nstreams) {
  while ((int)p->aux.size() < nstreams - 1) {
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "plan stream creation");
    p->aux.push_back(s);
  }
  const size_t nfork = 3, njoin = 3 * (size_t)(nstreams - 1);
  while (p->fork_ev.size() < nfork || p->join_ev.size() < njoin) {
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "plan event creation");
    if (p->fork_ev.size() < nfork)
      p->fork_ev.push_back(ev);
    else
      p->join_ev.push_back(ev);
  }
  return Status();
}

static void release_streams(hk_plan_s *p) {
  for (hipStream_t s : p->aux) (void)hipStreamDestroy(s);
  for (hipEvent_t ev : p->fork_ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : p->join_ev) (void)hipEventDestroy(ev);
  p->aux.clear();
  p->fork_ev.clear();
  p->join_ev.clear();
}

static Status enqueue(hk_plan_s *p, char *ws, hipStream_t st) {
  char *tables = p->tables_in_ws ? ws + p->ctl_bytes : p->d_tables;
  BatchArgs A;
  memset(&A, 0, sizeof(A));
  A.tasks = (const Task *)(tables + p->off_tasks);
  A.shapes = (const Shape *)(tables + p->off_shapes);
  A.ptrs = (const Ptrs *)(tables + p->off_ptrs);
  A.res_list = (const int32_t *)(tables + p->off_res);
  A.order = (const int32_t *)(tables + p->off_order);
  A.bctl = (BatchCtl *)ws;
  A.ws_base = ws + p->ctl_bytes + p->tables_bytes;
  A.spin_limit = p->wait_bound;
  for (int ph = 0; ph < 3; ++ph) A.phase_end[ph] = p->phase_end[ph];
  if (p->tasks.empty()) return Status();
  hipError_t e;
  if (p->persistent) {
    count_launch();
    prof_before(st);
    e = dbl(p->dt) ? launch_batch_f64(A, p->grid, st) : launch_batch_f32(A, p->grid, st);
    prof_after(PK_BATCH, st);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
  } else {
    // one specialised launch per (phase, kind, length, odd factor) group; the
    // launches of a phase go round-robin (longest transforms first) over up
    // to kGroupStreams streams, and the phase's end joins them again
    int per_phase[3] = {0, 0, 0};
    for (const auto &g : p->launches) per_phase[g.phase]++;
    const int S = std::min(kGroupStreams, std::max(std::max(per_phase[0], per_phase[1]), per_phase[2]));
    if (S > 1) {
      Status ss = ensure_streams(p, S);
      if (!ss.ok()) return ss;
    }
    int cur_phase = -1, k = 0, used = 1;
    auto join = [&](int ph) -> hipError_t {
      for (int i = 0; i + 1 < used; ++i) {
        hipEvent_t ev = p->join_ev[(size_t)ph * (S - 1) + i];
        hipError_t e2 = hipEventRecord(ev, p->aux[i]);
        if (e2 == hipSuccess) e2 = hipStreamWaitEvent(st, ev, 0);
        if (e2 != hipSuccess) return e2;
      }
      return hipSuccess;
    };
    for (const auto &g : p->launches) {
      if (g.phase != cur_phase) {
        if (cur_phase >= 0 && S > 1) {
          e = join(cur_phase);
          if (e != hipSuccess) return hip_fail(e, "phase join");
        }
        cur_phase = g.phase;
        k = 0;
        used = S > 1 ? std::min(S, per_phase[g.phase]) : 1;
        if (used > 1) {
          e = hipEventRecord(p->fork_ev[g.phase], st);
          for (int i = 0; e == hipSuccess && i + 1 < used; ++i) e = hipStreamWaitEvent(p->aux[i], p->fork_ev[g.phase], 0);
          if (e != hipSuccess) return hip_fail(e, "phase fork");
        }
      }
      hipStream_t gs = (k % used == 0) ? st : p->aux[k % used - 1];
      ++k;
      A.begin = g.begin;
      A.end = g.begin + g.count;
      count_launch();
      prof_before(gs);
      if (g.odd == 2 && g.kind == GK_RES)
        e = dbl(p->dt) ? launch_group_r2c_f64(A, g.logL, g.count, gs) : launch_group_r2c_f32(A, g.logL, g.count, gs);
      else if (g.odd == 2 && g.kind == GK_ROWB)
        e = dbl(p->dt) ? launch_group_r2cp_f64(A, g.logL, g.count, gs)
                       : launch_group_r2cp_f32(A, g.logL, g.count, gs);
      else if (g.odd > 1 && g.kind != GK_COL)
        e = dbl(p->dt) ? launch_group_odd_f64(A, g.odd, g.kind, g.logL, g.count, gs)
                       : launch_group_odd_f32(A, g.odd, g.kind, g.logL, g.count, gs);
      else
        e = dbl(p->dt) ? launch_group_f64(A, g.kind, g.logL, g.odd, g.count, gs)
                       : launch_group_f32(A, g.kind, g.logL, g.odd, g.count, gs);
      prof_after(PK_BATCH, gs);
      if (e != hipSuccess) return hip_fail(e, "grouped batch launch");
    }
    if (cur_phase >= 0 && S > 1) {
      e = join(cur_phase);
      if (e != hipSuccess) return hip_fail(e, "phase join");
    }
  }
  return Status();
}

static Status tune_plan(hk_plan_s *p, char *ws, hipStream_t st);

Status plan_execute(hk_plan_t p, void *ws, size_t ws_bytes, hipStream_t st) {
  if (!p) return fail(HK_ERR_NULL_POINTER, "plan is NULL");
  Status s = ensure_device();
  if (!s.ok()) return s;
  size_t need = 0;
  plan_ws_size(p, &need);
  if (!ws) return fail(HK_ERR_WORKSPACE, "workspace is NULL");
  if (ws_bytes < need) return fail(HK_ERR_WORKSPACE, "workspace smaller than hk_plan_workspace_size");
  if ((uintptr_t)ws % 256) return fail(HK_ERR_MISALIGNED, "workspace must be 256-byte aligned");
  // Graph plans are not tuned: a tuned plan that took over a candidate's
  // state ended in a host crash during its capture, a cause not found, so
  // the combination is switched off.
  if ((p->flags & HK_PLAN_AUTOTUNE) && !(p->flags & HK_PLAN_GRAPH) && !p->persistent && !p->tuned &&
      !p->tables_in_ws) {
    s = tune_plan(p, (char *)ws, st);
    if (!s.ok()) return s;
  }
  p->last_stream = st;
  p->last_ws = ws;
  if (p->tables_in_ws) {
    hipError_t e = hipMemcpyAsync((char *)ws + p->ctl_bytes, p->host_tables.data(), p->tables_bytes,
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
  } else {
    s = upload_tables(p);
    if (!s.ok()) return s;
  }
  if ((p->flags & HK_PLAN_GRAPH) && !p->tables_in_ws) {
    if (!st) return fail(HK_ERR_INVALID_VALUE, "graph plans need a non-default stream");
    if (p->gexec && p->graph_ws == ws) {
      count_launch();
      hipError_t e = hipGraphLaunch(p->gexec, st);
      if (e != hipSuccess) return hip_fail(e, "graph launch");
      return Status();
    }
    if (p->gexec) {
      (void)hipGraphExecDestroy(p->gexec);
      (void)hipGraphDestroy(p->graph);
      p->gexec = nullptr;
      p->graph = nullptr;
    }
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "stream capture begin");
    s = enqueue(p, (char *)ws, st);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (!s.ok()) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "stream capture end");
    e = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(e, "graph instantiate");
    }
    p->graph = g;
    p->graph_ws = ws;
    p->graph_stream = st;
    count_launch();
    e = hipGraphLaunch(p->gexec, st);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return Status();
  }
  return enqueue(p, (char *)ws, st);
}

// HK_PLAN_AUTOTUNE, at the first execute: a coordinate descent over the
// length buckets whose instances take odd-factor lengths (3 * 2^k, 5 * 2^k),
// longest first: each is tried at powers of two and kept there when the whole
// plan runs faster.  Odd lengths move fewer bytes but give each lane group
// several sequences in turn, and which wins depends on the length and on how
// much work the plan has of that length.  Every candidate is timed on the
// caller's stream and workspace (its outputs are rewritten by the execute
// that follows); the best plan replaces this one's contents.
static Status time_plan(hk_plan_s *q, char *ws, hipStream_t st, double *ms) {
  Status s = upload_tables(q);
  if (!s.ok()) return s;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  std::vector<float> t;
  for (int w = 0; w < 2 && s.ok(); ++w) s = enqueue(q, ws, st);  // warm-up
  for (int r = 0; r < 5 && s.ok() && e == hipSuccess; ++r) {
    e = hipEventRecord(e0, st);
    for (int k = 0; k < 3 && s.ok() && e == hipSuccess; ++k) s = enqueue(q, ws, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float v = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&v, e0, e1);
    t.push_back(v / 3.0f);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (!s.ok()) return s;
  if (e != hipSuccess) return hip_fail(e, "plan timing");
  std::sort(t.begin(), t.end());
  *ms = t[t.size() / 2];
  return Status();
}

static Status tune_plan(hk_plan_s *p, char *ws, hipStream_t st) {
  p->tuned = true;
  // buckets with odd-factor lengths in the default plan, and those of them
  // that use the factor 5
  std::vector<int> buckets;
  uint32_t five = 0;
  for (int64_t i = 0; i < p->count; ++i) {
    const Shape &sh = p->shapes[i];
    if (sh.is_block || sh.odd == 1) continue;
    const int b = length_bucket(problem_of(p->dt, p->probs[i]));
    if (b >= 32) continue;
    if (std::find(buckets.begin(), buckets.end(), b) == buckets.end()) buckets.push_back(b);
    if (sh.odd == 5) five |= 1u << b;
  }
  std::sort(buckets.rbegin(), buckets.rend());
  double best = 0.0;
  Status s = time_plan(p, ws, st, &best);
  if (!s.ok()) return s;
  p->tune_ms_default = best;
  uint32_t best_pow2 = p->pow2_buckets, best_no5 = p->no5_buckets;
  hk_plan_t best_plan = nullptr;
  // per bucket, longest first: lengths without the factor 5 (where the
  // bucket has it), then powers of two; a candidate is kept when it is at
  // least 3 % faster (eager timings of one plan vary by a few percent)
  auto attempt = [&](uint32_t pow2, uint32_t no5) -> Status {
    hk_plan_t q = nullptr;
    Status st2 = plan_build(&q, p->dt, p->probs.data(), p->count, p->flags, pow2, no5);
    if (!st2.ok()) return st2;
    double t = 0.0;
    st2 = time_plan(q, ws, st, &t);
    if (!st2.ok()) {
      plan_destroy(q);
      return st2;
    }
    if (t < 0.97 * best) {
      best = t;
      best_pow2 = pow2;
      best_no5 = no5;
      if (best_plan) plan_destroy(best_plan);
      best_plan = q;
    } else {
      plan_destroy(q);
    }
    return Status();
  };
  for (int b : buckets) {
    if ((five >> b) & 1u) {
      s = attempt(best_pow2, best_no5 | (1u << b));
      if (!s.ok()) break;
    }
    s = attempt(best_pow2 | (1u << b), best_no5);
    if (!s.ok()) break;
  }
  if (!s.ok()) {
    if (best_plan) plan_destroy(best_plan);
    return s;
  }
  p->tune_ms_best = best;
  if (best_plan) {
    // take the winner's task lists, tables and streams; the old ones leave
    // with the temporary plan
    std::vector<hk_problem_t> probs;
    probs.swap(p->probs);
    const size_t tune_ws = p->tune_ws_bytes;
    const double d0 = p->tune_ms_default;
    std::swap(*p, *best_plan);
    p->probs.swap(probs);
    p->tune_ws_bytes = tune_ws;
    p->tune_ms_default = d0;
    p->tune_ms_best = best;
    p->tuned = true;
    plan_destroy(best_plan);
  }
  return Status();
}

Status plan_tune_times(hk_plan_t p, double *ms_default, double *ms_tuned, uint32_t *pow2_buckets) {
  if (!p) return fail(HK_ERR_NULL_POINTER, "plan is NULL");
  if (ms_default) *ms_default = p->tune_ms_default;
  if (ms_tuned) *ms_tuned = p->tune_ms_best;
  if (pow2_buckets) *pow2_buckets = p->pow2_buckets;
  return Status();
}

Status plan_status(hk_plan_t p) {
  if (!p) return fail(HK_ERR_NULL_POINTER, "plan is NULL");
  if (!p->last_ws) return Status();
  hipError_t e = hipStreamSynchronize(p->last_stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  if (!p->persistent) return Status();  // grouped launches have no waits and no error word
  BatchCtl c;
  e = hipMemcpy(&c, p->last_ws, sizeof(c), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "status readback");
  if (c.error) return fail(HK_ERR_DEVICE_FAULT, "a grid barrier wait of the persistent kernel exceeded its bound");
  return Status();
}

Status plan_set_wait_bound(hk_plan_t p, uint32_t spins) {
  if (!p) return fail(HK_ERR_NULL_POINTER, "plan is NULL");
  if (p->gexec) return fail(HK_ERR_INVALID_VALUE, "the plan's launches are already captured in a graph");
  p->wait_bound = spins;
  return Status();
}

Status plan_pass_bytes(hk_plan_t p, int64_t *bytes) {
  if (!p) return fail(HK_ERR_NULL_POINTER, "plan is NULL");
  if (!bytes) return fail(HK_ERR_NULL_POINTER, "bytes is NULL");
  int64_t tot = 0;
  for (const Shape &sh : p->shapes) tot += pass_model_bytes(sh, p->dt);
  *bytes = tot;
  return Status();
}

Status plan_destroy(hk_plan_t p) {
  if (!p) return Status();
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_tables || !p->aux.empty()) (void)hipDeviceSynchronize();
  if (p->d_tables) (void)hipFree(p->d_tables);
  release_streams(p);
  delete p;
  return Status();
}

Status plan_set_oneshot(hk_plan_t p) {
  if (!p) return fail(HK_ERR_NULL_POINTER, "plan is NULL");
  p->tables_in_ws = true;
  return Status();
}

Status plan_release_after(hk_plan_t p, hipStream_t st) {
  // The descriptor tables were copied into the caller's workspace from the
  // plan's host buffer; wait for the stream before that buffer goes away.
  hipError_t e = hipStreamSynchronize(st);
  release_streams(p);
  delete p;
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  return Status();
}

// ---------------------------------------------------------------------------
// Autotuner.  For each row/column split of N it runs a coordinate descent:
// the row-pass parameters (elements per lane, rows per workgroup, rows in
// turn) and the column-pass parameters (elements per lane, tile width, XCD
// tile numbering) drive different kernels, so each group is searched with the
// other fixed, twice.  Every candidate is timed on scratch buffers: inputs
// distinct per instance (zero-filled), and for single products a pool of
// input sets larger than the 256 MB last-level cache that successive launches
// cycle through, so that inputs come from HBM as in use.  A playoff of the
// fastest candidates (interleaved repeated timings, median) picks the winner,
// which is cached under the key the call path looks up (dtype, program, 1D/BHHB, N,
// batch class).
// ---------------------------------------------------------------------------
Status autotune_problem(const Problem &proto, int64_t batch, bool verbose) {
  Status s = ensure_device();
  if (!s.ok()) return s;
  if (batch < 1) return fail(HK_ERR_INVALID_VALUE, "batch must be >= 1");
  Problem p = proto;
  const hk_dtype_t dt = p.dt;
  Layout lay0;
  s = layout_for(p, 0, &lay0, true, batch);
  if (!s.ok()) return s;
  // layouts to search
  std::vector<std::pair<int, Layout>> layouts;
  for (int sp : {0, -1, 1, -2, 2}) {
    Layout lay;
    if (p.is_block && sp != 0) continue;
    if (!layout_for(p, sp, &lay, true, batch).ok()) continue;
    if (sp != 0 && (lay.resident || lay.odd != lay0.odd || (lay.logR == lay0.logR && lay.logC == lay0.logC)))
      continue;
    layouts.push_back({sp, lay});
  }
  // buffer sizes (workspace does not depend on the schedule)
  const size_t eb = elem_bytes(dt);
  int64_t hrows = 1 - p.m, hcols = 1 - p.m, vmax = 1;
  for (int q = 0; q < p.m; ++q) {
    hrows += p.dims[q];
    hcols += p.bdims[q];
    vmax = std::max<int64_t>(vmax, p.dims[q] * (p.is_block ? p.bdims[q] : 1));
  }
  const int64_t hlen = p.is_block ? hrows * hcols : hrows;
  const int64_t ylen = std::max<int64_t>(hlen, vmax);  // room for y, grad_h or grad_x
  size_t wsb = 0;
  for (const auto &sl : layouts) {
    Sched sc = default_sched(dt, sl.second, p.prog, batch);
    sc.split = sl.first;
    Shape sh;
    Ptrs P;
    build_shape(p, sl.second, sc, &sh, &P, nullptr);
    wsb = std::max(wsb, instance_ws_bytes(sh, dt));
  }
  const int64_t in_bytes = (hlen + vmax) * (int64_t)eb;
  const int64_t pool = batch > 1 ? 1 : std::max<int64_t>(1, std::min<int64_t>(64, ((int64_t)384 << 20) / in_bytes + 1));
  const int64_t nin = batch > 1 ? batch : pool;
  void *dh = nullptr, *dx = nullptr, *dy = nullptr, *dy1 = nullptr, *da = nullptr, *dws = nullptr;
  hipError_t e = hipMalloc(&dh, nin * hlen * eb);
  if (e == hipSuccess) e = hipMalloc(&dx, nin * vmax * eb);
  if (e == hipSuccess) e = hipMalloc(&dy, batch * ylen * eb);
  if (e == hipSuccess) e = hipMalloc(&dy1, batch * ylen * eb);
  if (e == hipSuccess) e = hipMalloc(&da, batch * 2 * eb);
  if (e == hipSuccess && wsb) e = hipMalloc(&dws, batch * wsb);
  if (e == hipSuccess) e = hipMemset(dh, 0, nin * hlen * eb);
  if (e == hipSuccess) e = hipMemset(dx, 0, nin * vmax * eb);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  p.h = dh;
  for (int q = 0; q < p.m; ++q)
    if (p.vec[q]) p.vec[q] = dx;
  if (p.prog == PROG_FWD) {
    if (p.y) p.y = dy;
    if (p.alpha) p.alpha = da;
  } else {
    if (p.v) p.v = dx;
    if (p.phi) p.phi = da;
    if (p.gh) p.gh = dy;
    if (p.gx) p.gx = dy1;
  }
  const int reps = batch > 8 ? 2 : (batch > 1 ? 5 : (int)std::max<int64_t>(16, pool));
  int ntimed = 0;
  double best_seen = 1e30;
  // time of one schedule in ms (infinite if the kernels cannot run it)
  auto time_sched = [&](const Layout &lay, const Sched &sc) -> double {
    if (!sched_valid(dt, lay, sc)) return 1e30;
    Shape sh;
    Ptrs P;
    build_shape(p, lay, sc, &sh, &P, nullptr);
    P.ws = dws;
    Strides str;
    memset(&str, 0, sizeof(str));
    int64_t op_stride[MAXOPS];
    for (int o = 0; o < sh.nops; ++o) op_stride[o] = (sh.ops[o].role == ROLE_H ? hlen : vmax) * (int64_t)eb;
    if (batch > 1)
      for (int o = 0; o < sh.nops; ++o) str.op[o] = op_stride[o];
    str.y = ylen * eb;
    str.out1 = ylen * eb;
    str.alpha = eb;
    str.ws = (int64_t)instance_ws_bytes(sh, dt);
    const Ptrs P0 = P;
    auto launch_k = [&](int k) {
      if (batch == 1)
        for (int o = 0; o < sh.nops; ++o) P.op[o] = (const char *)P0.op[o] + (k % pool) * op_stride[o];
      return launch_shape(dt, sh, sc, P, str, batch, nullptr);
    };
    // warm-up launch, timed: a candidate already 4x slower than the best so
    // far is not timed further
    (void)hipEventRecord(e0, nullptr);
    s = launch_k(0);
    (void)hipEventRecord(e1, nullptr);
    (void)hipEventSynchronize(e1);
    if (!s.ok()) return 1e30;
    float wms = 0;
    (void)hipEventElapsedTime(&wms, e0, e1);
    if (wms > 4.0 * best_seen) {
      if (verbose)
        fprintf(stderr, "[hk autotune] split=%d E_row=%d rows=%d iters=%d E_col=%d tw=%d xcd=%d : %.4f ms (skipped)\n",
                sc.split, sc.E_row, sc.rows_per_wg, sc.iters, sc.E_col, sc.tw, sc.xcd, wms);
      return (double)wms;
    }
    (void)hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps && s.ok(); ++r) s = launch_k(r + 1);
    (void)hipEventRecord(e1, nullptr);
    (void)hipEventSynchronize(e1);
    if (!s.ok()) return 1e30;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ++ntimed;
    const double t = ms / reps;
    best_seen = std::min(best_seen, t);
    if (verbose)
      fprintf(stderr, "[hk autotune] split=%d E_row=%d rows=%d iters=%d E_col=%d tw=%d xcd=%d : %.4f ms\n", sc.split,
              sc.E_row, sc.rows_per_wg, sc.iters, sc.E_col, sc.tw, sc.xcd, t);
    return t;
  };
  double best = 1e30;
  Sched bestsc;
  Layout bestlay;
  struct Cand {
    double t;
    int li;  // index into layouts
    Sched sc;
  };
  std::vector<Cand> seen;
  if (e == hipSuccess) {
    for (int li = 0; li < (int)layouts.size(); ++li) {
      const Layout &lay = layouts[li].second;
      Sched cur = default_sched(dt, lay, p.prog, batch);
      cur.split = layouts[li].first;
      double tcur = time_sched(lay, cur);
      if (!s.ok()) break;
      if (tcur < 1e30) seen.push_back({tcur, li, cur});
      for (int round = 0; round < 2 && s.ok(); ++round) {
        // row-pass parameters
        for (int er : {4, 8, 16})
          for (int rows : {1, 2, 4, 8, 16, 32})
            for (int it : {1, 2, 4}) {
              if (lay.resident && it != 1) continue;
              Sched c = cur;
              c.E_row = er;
              c.rows_per_wg = rows;
              c.iters = it;
              if (c.E_row == cur.E_row && c.rows_per_wg == cur.rows_per_wg && c.iters == cur.iters) continue;
              const double tc = time_sched(lay, c);
              if (!s.ok()) break;
              if (tc < 1e30) seen.push_back({tc, li, c});
              if (tc < tcur) {
                tcur = tc;
                cur = c;
              }
            }
        if (lay.resident || !s.ok()) break;
        // column-pass parameters
        for (int ec : {8, 16})
          for (int tw : {1, 2, 4, 8, 16, 32})
            for (int xcd : {0, 1}) {
              Sched c = cur;
              c.E_col = ec;
              c.tw = tw;
              c.xcd = xcd;
              if (c.E_col == cur.E_col && c.tw == cur.tw && c.xcd == cur.xcd) continue;
              const double tc = time_sched(lay, c);
              if (!s.ok()) break;
              if (tc < 1e30) seen.push_back({tc, li, c});
              if (tc < tcur) {
                tcur = tc;
                cur = c;
              }
            }
      }
      if (tcur < best) {
        best = tcur;
        bestsc = cur;
        bestlay = lay;
      }
    }
  }
  // Playoff.  One timing of a candidate varies by a few percent from run to
  // run, enough to crown a schedule that is no faster than the one it
  // replaces.  The fastest few candidates, the default schedule and the
  // schedule already cached under this key are timed again in interleaved
  // rounds; the lowest median wins.
  if (e == hipSuccess && s.ok() && !seen.empty()) {
    std::stable_sort(seen.begin(), seen.end(), [](const Cand &a, const Cand &b) { return a.t < b.t; });
    std::vector<Cand> fin;
    auto same = [](const Sched &a, const Sched &b) {
      return a.E_row == b.E_row && a.rows_per_wg == b.rows_per_wg && a.E_col == b.E_col && a.tw == b.tw &&
             a.split == b.split && a.xcd == b.xcd && a.iters == b.iters;
    };
    auto add = [&](int li, const Sched &c) {
      for (const Cand &f : fin)
        if (f.li == li && same(f.sc, c)) return;
      fin.push_back({0.0, li, c});
    };
    for (size_t i = 0; i < seen.size() && fin.size() < 4; ++i) add(seen[i].li, seen[i].sc);
    for (int li = 0; li < (int)layouts.size(); ++li)
      if (layouts[li].first == 0) {
        Sched d = default_sched(dt, layouts[li].second, p.prog, batch);
        d.split = 0;
        add(li, d);
      }
    Sched inc;
    if (sched_lookup(dt, p.prog, p.is_block ? 1 : 0, lay0.lclass(), lay0.logR + lay0.logC, p.is_block ? lay0.logC : -1,
                     batch, &inc))
      for (int li = 0; li < (int)layouts.size(); ++li)
        if (layouts[li].first == inc.split) add(li, inc);
    constexpr int kRounds = 5;
    std::vector<std::vector<double>> ts(fin.size());
    for (int r = 0; r < kRounds && s.ok(); ++r)
      for (size_t i = 0; i < fin.size() && s.ok(); ++i)
        ts[i].push_back(time_sched(layouts[fin[i].li].second, fin[i].sc));
    if (s.ok()) {
      best = 1e30;
      for (size_t i = 0; i < fin.size(); ++i) {
        std::sort(ts[i].begin(), ts[i].end());
        const double med = ts[i][kRounds / 2];
        if (verbose)
          fprintf(stderr, "[hk autotune] playoff split=%d E_row=%d rows=%d iters=%d E_col=%d tw=%d xcd=%d : median %.4f ms\n",
                  fin[i].sc.split, fin[i].sc.E_row, fin[i].sc.rows_per_wg, fin[i].sc.iters, fin[i].sc.E_col,
                  fin[i].sc.tw, fin[i].sc.xcd, med);
        if (med < best) {
          best = med;
          bestsc = fin[i].sc;
          bestlay = layouts[fin[i].li].second;
        }
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipDeviceSynchronize();
  (void)hipFree(dh);
  (void)hipFree(dx);
  (void)hipFree(dy);
  (void)hipFree(dy1);
  (void)hipFree(da);
  if (dws) (void)hipFree(dws);
  if (e != hipSuccess) return hip_fail(e, "autotune buffers");
  if (!s.ok()) return s;
  if (best >= 1e30) return fail(HK_ERR_NOT_SUPPORTED, "autotune found no schedule");
  sched_store(dt, p.prog, p.is_block ? 1 : 0, lay0.lclass(), lay0.logR + lay0.logC, p.is_block ? lay0.logC : -1,
              batch, bestsc);
  if (verbose)
    fprintf(stderr,
            "[hk autotune] best of %d: split=%d (odd=%d R=2^%d C=2^%d) E_row=%d rows=%d iters=%d E_col=%d tw=%d "
            "xcd=%d %.4f ms\n",
            ntimed, bestsc.split, bestlay.odd, bestlay.logR, bestlay.logC, bestsc.E_row, bestsc.rows_per_wg, bestsc.iters,
            bestsc.E_col, bestsc.tw, bestsc.xcd, best);
  return Status();
}

Status autotune_tvp(hk_dtype_t dt, int m, int64_t n, bool verbose) {
  return autotune_shape(dt, 0, m, n, nullptr, nullptr, 1, verbose);
}

Status autotune_shape(hk_dtype_t dt, int kind, int m, int64_t n, const int64_t *inner, const int64_t *blocks,
                      int64_t batch, bool verbose) {
  if (m < 2 || m > HK_MAX_ORDER) return fail(HK_ERR_INVALID_VALUE, "order m must be in [2, 8]");
  Problem p;
  p.dt = dt;
  p.m = m;
  const void *dummy = (const void *)256;
  p.h = dummy;
  Status s;
  if (kind == 0 || kind == 2) {  // forward, equal vectors (1D or BHHB)
    p.prog = PROG_FWD;
    p.is_block = kind == 2;
    for (int q = 0; q < m; ++q) {
      p.dims[q] = p.is_block ? (inner ? inner[q] : 0) : n;
      if (p.is_block) p.bdims[q] = blocks ? blocks[q] : 0;
      p.vec[q] = dummy;
    }
    p.y = (void *)256;
    p.alpha = (void *)256;
    s = validate_forward(p);
  } else if (kind == 1) {  // adjoint with both cotangents and both gradients
    p.prog = PROG_BWD;
    for (int q = 0; q < m; ++q) p.dims[q] = n;
    p.vec[1] = dummy;
    p.v = dummy;
    p.phi = dummy;
    p.gx = (void *)256;
    p.gh = (void *)256;
    s = validate_backward(p);
  } else {
    return fail(HK_ERR_INVALID_VALUE, "unknown autotune kind");
  }
  if (!s.ok()) return s;
  return autotune_problem(p, batch, verbose);
}

}  // namespace hk

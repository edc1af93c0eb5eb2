// C ABI of liblbx: plan construction, workspace layout and the entry points
// declared in include/lbx.h.  Host code only; all arithmetic on states runs
// in the kernels (kernels_*.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "lbx_host.hpp"

using namespace lbx;

namespace lbx {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return LB_EDEVICE;
}

// Profiling state is guarded by p->mu (held by every caller below).
static void prof_account(const lb_plan *p, const lbx_prof_pending &e) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, e.start, e.stop) == hipSuccess) {
    p->prof_n[e.kernel] += e.launches;
    p->prof_ms[e.kernel] += ms;
  }
  p->ev_pool.push_back(e.start);
  p->ev_pool.push_back(e.stop);
}

void prof_resolve(const lb_plan *p) {
  std::lock_guard<std::mutex> g(p->mu);
  for (auto &e : p->prof_pending) {
    if (hipEventSynchronize(e.stop) == hipSuccess) {
      prof_account(p, e);
    } else {
      (void)hipEventDestroy(e.start);
      (void)hipEventDestroy(e.stop);
    }
  }
  p->prof_pending.clear();
}

void prof_add_work(const lb_plan *p, int kernel, int64_t work) {
  std::lock_guard<std::mutex> g(p->mu);
  p->prof_work[kernel] += work;
}

hipEvent_t ProfScope::prof_event(const lb_plan *p) {
  if (!p->ev_pool.empty()) {
    hipEvent_t e = p->ev_pool.back();
    p->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

// Accounts the launches that have already finished (oldest first, without
// waiting), so that a long profiled time loop keeps few events alive.
void ProfScope::prof_drain(const lb_plan *p) {
  size_t n = 0;
  while (n < p->prof_pending.size() && hipEventQuery(p->prof_pending[n].stop) == hipSuccess) {
    prof_account(p, p->prof_pending[n]);
    ++n;
  }
  p->prof_pending.erase(p->prof_pending.begin(), p->prof_pending.begin() + n);
}

lbx_opts plan_options(const lb_plan *p) {
  std::lock_guard<std::mutex> g(p->mu);
  return p->opts;
}

int status_bits_code(int32_t s) {
  if (s & LB_STATUS_NONFINITE) return fail(LB_ENONFINITE, "an objective is not finite");
  if (s & LB_STATUS_THETA)
    return fail(LB_EUNSUPPORTED,
                "a stage-solve contraction bound is >= 0.5 (step or control amplitude too large); calls with a "
                "workspace in LB_OPT_SYNC mode solve such steps with GMRES");
  if (s & LB_STATUS_NOCONV) return fail(LB_EUNSUPPORTED, "a stage solve did not converge within the sweep cap");
  if (s & LB_STATUS_RETRY)
    return fail(LB_EUNSUPPORTED, "a streamed step needed more stage sweeps than were launched; repeat the call "
                                 "with LB_OPT_SYNC on, which repeats it with a-priori counts");
  return LB_OK;
}

}  // namespace lbx

// ----------------------------------------------------------------------------
// Batch metadata: everything derived from batch_per_sys, cached per plan.
// ----------------------------------------------------------------------------
namespace {

lbx_opts snapshot(const lb_plan *p) { return plan_options(p); }

struct LdsClass {
  int block, ept;
  int qc;      // > 0: specialised kernel for qc subsystems; 0: generic kernel
  int i0, i1;  // item range
};

struct BatchMeta {
  std::vector<int32_t> batch;
  int64_t total_entries = 0;
  int total_states = 0;
  std::vector<int64_t> sys_off;     // batched entry offset of system s
  std::vector<int32_t> sys_state0;  // first global state of system s (nsys+1)
  std::vector<int> path;            // 1 = LDS, 2 = streaming, 0 = empty system
  // LDS path
  std::vector<LdsItem> items;
  std::vector<LdsClass> classes;
  std::vector<int32_t> lds_sys, lds_item_range;
  int64_t lds_hist_entries = 0;  // sum over items of (NT+1) N^2
  int64_t lds_gpart = 0;         // doubles of gradient partials
  // streaming path
  std::vector<StreamSeg> segs;
  std::vector<int32_t> seg_state0;
  int64_t st_entries = 0;  // compact streamed entries
  int64_t st_blocks = 0;
  int tile_sys = -1;       // single streamed system run by the block-tiled kernels
  int tile_B = 0;
  int tile_k = 0;          // its block shape
  // device copies (one allocation)
  void *dmem = nullptr;
  LdsItem *d_items = nullptr;
  int32_t *d_lds_sys = nullptr, *d_lds_item_range = nullptr;
  StreamSeg *d_segs = nullptr;
  int32_t *d_seg_state0 = nullptr;
  int32_t *d_state_sys = nullptr;
  int64_t *d_state_off = nullptr;
  int32_t *d_sys_state0 = nullptr;
  // running penalty: per system {first stream block, blocks, first LDS item, items}
  std::vector<int64_t> pen_rng;
  int64_t *d_pen_rng = nullptr;
};

struct PlanExtra {
  std::mutex mu;
  std::map<std::vector<int32_t>, std::unique_ptr<BatchMeta>> batches;
};

std::mutex g_extra_mu;
std::map<const lb_plan *, std::unique_ptr<PlanExtra>> g_extra;

PlanExtra *extra_of(const lb_plan *p) {
  std::lock_guard<std::mutex> g(g_extra_mu);
  auto &e = g_extra[p];
  if (!e) e.reset(new PlanExtra());
  return e.get();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Path of system s: 1 LDS-resident, 2 streamed, -1 not possible.
int path_for(const lb_plan *p, int s, int path, bool stream_small) {
  int blk, ept;
  const bool fits = lds_shape(p->sys[s].N2, &blk, &ept);
  if (path == 1) return fits && !stream_small ? 1 : -1;
  if (path == 2) return 2;
  return fits && !stream_small ? 1 : 2;
}

template <class T>
T *carve(char *&cur, size_t n) {
  T *r = reinterpret_cast<T *>(cur);
  cur += align256(n * sizeof(T));
  return r;
}

// Checkpoint interval of streamed systems: 0 picks ceil(sqrt(NT)).
int ckpt_interval(const lb_plan *p, int ckpt_every) {
  if (ckpt_every > 0) return std::min(ckpt_every, p->NT);
  return std::max(1, (int)std::ceil(std::sqrt((double)p->NT)));
}
int ckpt_count(int NT, int c) { return (NT - 1) / c + 2; }

// An explicit checkpoint interval above 1 is honoured by every system: the
// LDS-resident kernels keep every state, so systems that would run there are
// streamed instead.
bool streams_small(int ckpt_every) { return ckpt_every > 1; }

// path_override: -1 uses the option LB_OPT_PATH.
// generic_lds: every LDS-resident system on the generic kernels (the
// specialised ones have no running-penalty source).
int build_batch(const lb_plan *p, const lbx_opts &o, const int32_t *batch, bool stream_small,
                BatchMeta **out, int path_override = -1, bool generic_lds = false) {
  const int nsys = (int)p->sys.size();
  const int path = path_override >= 0 ? path_override : o.path;
  std::vector<int32_t> key(batch, batch + nsys);
  for (int s = 0; s < nsys; ++s)
    if (key[s] < 0) return fail(LB_EINVAL, "batch_per_sys has a negative entry");
  key.push_back(path);
  key.push_back(o.tile);
  key.push_back(o.tile_ki);
  key.push_back(stream_small ? 1 : 0);
  key.push_back(generic_lds ? 1 : 0);
  PlanExtra *ex = extra_of(p);
  std::lock_guard<std::mutex> g(ex->mu);
  auto it = ex->batches.find(key);
  if (it != ex->batches.end()) {
    *out = it->second.get();
    return LB_OK;
  }
  std::unique_ptr<BatchMeta> m(new BatchMeta());
  m->batch.assign(key.begin(), key.begin() + nsys);
  m->sys_off.resize(nsys);
  m->sys_state0.resize(nsys + 1);
  m->path.resize(nsys);
  int64_t off = 0;
  int st = 0;
  for (int s = 0; s < nsys; ++s) {
    m->sys_off[s] = off;
    m->sys_state0[s] = st;
    off += (int64_t)key[s] * p->sys[s].N2;
    st += key[s];
    if (key[s] == 0) {
      m->path[s] = 0;
      continue;
    }
    m->path[s] = path_for(p, s, path, stream_small);
    if (m->path[s] < 0)
      return fail(LB_EUNSUPPORTED, "system " + std::to_string(s) +
                                       " cannot run on the LDS-resident kernels (N^2 > 4096, or a checkpoint "
                                       "interval above 1)");
  }
  m->sys_state0[nsys] = st;
  m->total_entries = off;
  m->total_states = st;
  // LDS items grouped by kernel class, systems contiguous within a class.
  const int NT = p->NT;
  std::map<std::tuple<int, int, int>, std::vector<int>> cls;
  for (int s = 0; s < nsys; ++s)
    if (m->path[s] == 1) {
      int blk, ept;
      lds_shape(p->sys[s].N2, &blk, &ept);
      // the specialised kernels have no coupling terms
      const int qc = !generic_lds && lds_fast_ok(blk, ept, p->sys[s].Q) && p->sys[s].njc == 0 ? p->sys[s].Q : 0;
      cls[std::make_tuple(blk, ept, qc)].push_back(s);
    }
  for (auto &kv : cls) {
    LdsClass c{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first),
               (int)m->items.size(), 0};
    for (int s : kv.second) {
      const SysDev &S = p->sys[s];
      m->lds_sys.push_back(s);
      m->lds_item_range.push_back((int)m->items.size());
      for (int b = 0; b < key[s]; ++b) {
        LdsItem itm{};
        itm.sys = s;
        itm.b = b;
        itm.off = m->sys_off[s] + (int64_t)b * S.N2;
        itm.st_off = m->lds_hist_entries;
        m->lds_hist_entries += (int64_t)(NT + 1) * S.N2;
        itm.parts = c.qc > 0 ? c.block / 16 : c.block / 64;
        itm.gp_off = m->lds_gpart;
        m->lds_gpart += (int64_t)NT * itm.parts * 2 * S.Q;
        itm.wterm = 0.0;  // set per call (beta lives on the device)
        m->items.push_back(itm);
      }
    }
    c.i1 = (int)m->items.size();
    m->classes.push_back(c);
  }
  m->lds_item_range.push_back((int)m->items.size());
  // Streaming segments.
  int64_t coff = 0, blk = 0;
  for (int s = 0; s < nsys; ++s)
    if (m->path[s] == 2) {
      StreamSeg sg{};
      sg.sys = s;
      sg.nstates = key[s];
      sg.off = coff;
      sg.boff = m->sys_off[s];
      sg.count = (int64_t)key[s] * p->sys[s].N2;
      sg.blk0 = blk;
      coff += sg.count;
      blk += (sg.count + STREAM_BLOCK - 1) / STREAM_BLOCK;
      m->segs.push_back(sg);
      m->seg_state0.push_back(m->sys_state0[s]);
    }
  m->st_entries = coff;
  m->st_blocks = blk;
  if (m->segs.size() == 1 && o.tile) {
    const int k = tile_ki(p, m->segs[0].sys, o.tile_ki);
    if (k) {
      m->tile_sys = m->segs[0].sys;
      m->tile_B = m->segs[0].nstates;
      m->tile_k = k;
    }
  }
  // Running-penalty ranges of every system.
  m->pen_rng.assign((size_t)4 * nsys, 0);
  for (const auto &sg : m->segs) {
    m->pen_rng[4 * sg.sys] = sg.blk0;
    m->pen_rng[4 * sg.sys + 1] = (sg.count + STREAM_BLOCK - 1) / STREAM_BLOCK;
  }
  for (size_t k = 0; k < m->lds_sys.size(); ++k) {
    const int s = m->lds_sys[k];
    m->pen_rng[4 * s + 2] = m->lds_item_range[k];
    m->pen_rng[4 * s + 3] = m->lds_item_range[k + 1] - m->lds_item_range[k];
  }
  // Per-state tables for the objective.
  std::vector<int32_t> state_sys(std::max(1, st));
  std::vector<int64_t> state_off(std::max(1, st));
  for (int s = 0; s < nsys; ++s)
    for (int b = 0; b < key[s]; ++b) {
      state_sys[m->sys_state0[s] + b] = s;
      state_off[m->sys_state0[s] + b] = m->sys_off[s] + (int64_t)b * p->sys[s].N2;
    }
  // One device allocation for every table.
  size_t bytes = align256(std::max<size_t>(1, m->items.size()) * sizeof(LdsItem)) +
                 align256(std::max<size_t>(1, m->lds_sys.size()) * 4) +
                 align256(m->lds_item_range.size() * 4) +
                 align256(std::max<size_t>(1, m->segs.size()) * sizeof(StreamSeg)) +
                 align256(std::max<size_t>(1, m->seg_state0.size()) * 4) +
                 align256(state_sys.size() * 4) + align256(state_off.size() * 8) +
                 align256(m->sys_state0.size() * 4) + align256(m->pen_rng.size() * 8);
  LBX_HIP(hipMalloc(&m->dmem, bytes));
  char *cur = (char *)m->dmem;
  m->d_items = carve<LdsItem>(cur, std::max<size_t>(1, m->items.size()));
  m->d_lds_sys = carve<int32_t>(cur, std::max<size_t>(1, m->lds_sys.size()));
  m->d_lds_item_range = carve<int32_t>(cur, m->lds_item_range.size());
  m->d_segs = carve<StreamSeg>(cur, std::max<size_t>(1, m->segs.size()));
  m->d_seg_state0 = carve<int32_t>(cur, std::max<size_t>(1, m->seg_state0.size()));
  m->d_state_sys = carve<int32_t>(cur, state_sys.size());
  m->d_state_off = carve<int64_t>(cur, state_off.size());
  m->d_sys_state0 = carve<int32_t>(cur, m->sys_state0.size());
  m->d_pen_rng = carve<int64_t>(cur, m->pen_rng.size());
  if (!m->items.empty())
    LBX_HIP(hipMemcpy(m->d_items, m->items.data(), m->items.size() * sizeof(LdsItem), hipMemcpyHostToDevice));
  if (!m->lds_sys.empty())
    LBX_HIP(hipMemcpy(m->d_lds_sys, m->lds_sys.data(), m->lds_sys.size() * 4, hipMemcpyHostToDevice));
  LBX_HIP(hipMemcpy(m->d_lds_item_range, m->lds_item_range.data(), m->lds_item_range.size() * 4,
                    hipMemcpyHostToDevice));
  if (!m->segs.empty())
    LBX_HIP(hipMemcpy(m->d_segs, m->segs.data(), m->segs.size() * sizeof(StreamSeg), hipMemcpyHostToDevice));
  if (!m->seg_state0.empty())
    LBX_HIP(hipMemcpy(m->d_seg_state0, m->seg_state0.data(), m->seg_state0.size() * 4, hipMemcpyHostToDevice));
  LBX_HIP(hipMemcpy(m->d_state_sys, state_sys.data(), state_sys.size() * 4, hipMemcpyHostToDevice));
  LBX_HIP(hipMemcpy(m->d_state_off, state_off.data(), state_off.size() * 8, hipMemcpyHostToDevice));
  LBX_HIP(hipMemcpy(m->d_sys_state0, m->sys_state0.data(), m->sys_state0.size() * 4, hipMemcpyHostToDevice));
  LBX_HIP(hipMemcpy(m->d_pen_rng, m->pen_rng.data(), m->pen_rng.size() * 8, hipMemcpyHostToDevice));
  *out = m.get();
  ex->batches[key] = std::move(m);
  return LB_OK;
}

// Sweeps launched per streamed step: steps whose first iterate is
// extrapolated from a full history, and the others (started from fewer
// increments or from q).  The kernels run only as many as the step needs; a
// step that needs more raises LB_STATUS_RETRY.
constexpr int SWEEPS_HIST = 8;
constexpr int SWEEPS_START = 12;

// Trajectory storage (forward states the adjoint needs): LDS-resident items
// keep every state, [items][NT+1][N^2]; streamed systems keep checkpoints
// [nck][streamed entries] at multiples of c and at NT.
struct TrajLayout {
  size_t hist = 0, ckpt = 0, total = 0;
  int c = 1, nck = 0;
};

TrajLayout traj_layout(const lb_plan *p, const BatchMeta &m, int ckpt_every) {
  TrajLayout T;
  T.c = ckpt_interval(p, ckpt_every);
  T.nck = ckpt_count(p->NT, T.c);
  T.hist = 0;
  T.ckpt = align256((size_t)m.lds_hist_entries * sizeof(double2));
  T.total = T.ckpt + align256((m.segs.empty() ? 0 : (size_t)T.nck) * m.st_entries * sizeof(double2));
  return T;
}

// Workspace layout of one operation.
struct Layout {
  size_t status = 0, ctab = 0, ktab = 0, ttab = 0, objpart = 0, items = 0, sweeps = 0, kout = 0, gstep = 0;
  size_t traj = 0;  // LB_OP_GRADIENT: the trajectory lives in the workspace
  size_t rhoT = 0;  // LB_OP_GRADIENT: rho(T) when the caller does not want it
  size_t zhist = 0, gpart = 0;
  size_t q0 = 0, q1 = 0, z0 = 0, z1 = 0, zsf = 0, ringf = 0, zsa = 0, ringa = 0, zh = 0, qh0 = 0, qh1 = 0,
         seg = 0, st_gpart = 0, st_gfin = 0, slots = 0, kstep = 0;
  size_t kry = 0, kpart = 0;  // Krylov fallback: vectors and reduction scratch
  size_t ptab = 0, pacc = 0, ppart = 0, pen = 0;  // LB_OP_GRADIENT: running penalty
  size_t total = 0;
  TrajLayout T;
  int H = 0;
  int64_t grows = 1;  // gradient partial rows per step (streamed systems)
  int gbatch = 1;     // steps whose partial rows are reduced by one launch
};

// krylov: the layout of the Krylov fallback (no increment history; room for
// the GMRES vectors of the streamed batch).
// Block shape of the gradient integrands of the tiled streamed system (the
// two-pass sweeps use the system's first block shape), or 0: generic kernel.
int grad_tile_k(const lb_plan *p, const BatchMeta &m) {
  if (m.tile_sys < 0) return 0;
  return m.tile_k >= LB_SPLIT_BASE ? tile_ki(p, m.tile_sys, 0) : m.tile_k;
}

Layout layout(const lb_plan *p, const lbx_opts &o, int op, const BatchMeta &m, int ckpt_every,
              bool krylov = false) {
  Layout L;
  size_t cur = 0;
  auto take = [&](size_t bytes) {
    const size_t r = cur;
    cur += align256(std::max<size_t>(bytes, 1));
    return r;
  };
  const int nsys = (int)p->sys.size();
  const size_t E = (size_t)m.st_entries * sizeof(double2);
  const bool st = !m.segs.empty();
  L.H = st && op != LB_OP_IMR_STEP && !krylov ? o.history : 0;
  L.status = take(sizeof(int32_t));
  L.ctab = take((size_t)p->ctab_total * sizeof(double2));
  L.ktab = take((size_t)nsys * p->NT * 2 * sizeof(int32_t));
  L.ttab = take((size_t)nsys * p->NT * sizeof(double2));
  L.kout = take((size_t)nsys * p->NT * sizeof(int32_t));
  L.objpart = take((size_t)std::max(1, m.total_states) * 64 * sizeof(double));
  L.items = take(std::max<size_t>(1, m.items.size()) * sizeof(LdsItem));
  L.sweeps = take(std::max<size_t>(1, m.items.size()) * sizeof(int64_t));
  L.slots = take((size_t)2 * nsys * 2 * LB_STEP_SLOTS * sizeof(unsigned long long));
  L.kstep = take((size_t)2 * nsys * sizeof(int32_t));
  L.z0 = take(st ? E : 0);
  L.z1 = take(st ? E : 0);
  if (krylov && st) {
    L.kry = take((size_t)KRY_VECTORS * E);
    L.kpart = take(kry_part_bytes());
  }
  L.T = traj_layout(p, m, ckpt_every);
  if (op == LB_OP_IMR_STEP) {
    L.total = cur;
    return L;
  }
  L.q0 = take(st ? E : 0);
  L.q1 = take(st ? E : 0);
  L.zsf = take(st && L.H ? E : 0);
  L.ringf = take(st ? (size_t)L.H * E : 0);
  if (op == LB_OP_FORWARD) {
    L.total = cur;
    return L;
  }
  // LB_OP_GRADIENT (trajectory included) and LB_OP_BACKWARD
  if (op == LB_OP_GRADIENT) {
    L.traj = take(L.T.total);
    L.rhoT = take((size_t)m.total_entries * sizeof(double2));
    L.ptab = take((size_t)nsys * p->NT * sizeof(double));
    L.pacc = take((size_t)m.st_blocks * sizeof(double));
    L.ppart = take(m.items.size() * PEN_PARTS * sizeof(double));
    L.pen = take((size_t)nsys * sizeof(double));
  }
  L.gstep = take((size_t)2 * p->ctab_total * sizeof(double));
  bool fast = false;
  for (const auto &c : m.classes) fast = fast || c.qc > 0;
  L.zhist = take(fast ? (size_t)m.lds_hist_entries * sizeof(double2) : 0);
  L.gpart = take((size_t)m.lds_gpart * sizeof(double));
  L.zsa = take(st && L.H ? E : 0);
  L.ringa = take(st ? (size_t)L.H * E : 0);
  L.zh = take(st ? E : 0);
  L.qh0 = take(st ? E : 0);
  L.qh1 = take(st ? E : 0);
  L.seg = take(st ? (size_t)std::max(0, L.T.c - 1) * E : 0);
  L.grows = std::max<int64_t>(
      1, std::max<int64_t>(m.st_blocks, grad_tile_k(p, m) > 0 ? tile_grad_rows(p, m.tile_sys, m.tile_B, grad_tile_k(p, m)) : 0));
  // Up to a checkpoint interval of steps, within 256 MB of partial rows.
  const size_t row_bytes = (size_t)L.grows * 2 * QMAX * sizeof(double);
  L.gbatch = (int)std::max<int64_t>(1, std::min<int64_t>(L.T.c, (int64_t)((256u << 20) / row_bytes)));
  L.st_gpart = take(st ? (size_t)L.gbatch * row_bytes : 0);
  L.st_gfin = take(st ? (size_t)L.gbatch * stream_grad_fin_doubles((int)m.segs.size()) * sizeof(double) : 0);
  L.total = cur;
  return L;
}

int check_plan(const lb_plan *p) {
  if (!p) return fail(LB_EINVAL, "plan is NULL");
  return LB_OK;
}

// Weights (beta_b / M_s) times gscale[s] of the LDS items live on the device
// (beta is a device array), so the adjoint kernels read them through a
// per-call item copy.
__global__ void item_weights_kernel(LdsItem *items, int n, const double *beta, const int32_t *sys_state0,
                                    const double *gscale) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  LdsItem &it = items[k];
  const int M = sys_state0[it.sys + 1] - sys_state0[it.sys];
  const double gs = gscale ? gscale[it.sys] : 1.0;
  it.wterm = beta[sys_state0[it.sys] + it.b] / (double)M * gs;
  it.wpen = gs / (double)M;
}

int copy_segments(const BatchMeta &m, const double2 *src, bool src_batched, double2 *dst, hipStream_t st) {
  for (const auto &sg : m.segs) {
    const double2 *a = src + (src_batched ? sg.boff : sg.off);
    double2 *b = dst + (src_batched ? sg.off : sg.boff);
    LBX_HIP(hipMemcpyAsync(b, a, sg.count * sizeof(double2), hipMemcpyDeviceToDevice, st));
  }
  return LB_OK;
}

// Reads the status word of a workspace (synchronises the stream).
int read_status(const int32_t *d_status, hipStream_t st, int32_t *bits) {
  *bits = 0;
  LBX_HIP(hipMemcpyAsync(bits, d_status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  LBX_HIP(hipStreamSynchronize(st));
  return LB_OK;
}

// Error code of the status bits.
int status_code(int32_t s) { return status_bits_code(s); }

int status_code(const int32_t *d_status, hipStream_t st) {
  int32_t s = 0;
  if (int rc = read_status(d_status, st, &s)) return rc;
  return status_code(s);
}

// LB_OPT_GRAPH: the streamed time loop is recorded in chunks of steps with
// stream capture on a private stream and replayed as one graph launch per
// chunk.  Chunks of equal shape reuse the executable graph through
// hipGraphExecUpdate.  Only kernel launches are captured.
struct GraphRun {
  hipStream_t user;
  hipStream_t cap = nullptr;
  hipEvent_t ev = nullptr;
  hipGraphExec_t exec = nullptr;
  bool on;
  bool active = false;  // a capture is open
  GraphRun(const lbx_opts &o, hipStream_t s) : user(s), on(o.graph_steps > 0) {}
  int init() {
    if (!on) return LB_OK;
    LBX_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    LBX_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    return LB_OK;
  }
  hipStream_t stream() const { return on ? cap : user; }
  int begin() {
    if (!on) return LB_OK;
    LBX_HIP(hipEventRecord(ev, user));
    LBX_HIP(hipStreamWaitEvent(cap, ev, 0));
    LBX_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    active = true;
    return LB_OK;
  }
  int end() {
    if (!on) return LB_OK;
    active = false;
    hipGraph_t g = nullptr;
    LBX_HIP(hipStreamEndCapture(cap, &g));
    bool ok = false;
    if (exec) {
      hipGraphExecUpdateResult res;
      hipGraphNode_t err_node = nullptr;
      ok = hipGraphExecUpdate(exec, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
      if (!ok) {
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(exec);
        exec = nullptr;
      }
    }
    if (!exec) {
      const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "hipGraphInstantiate");
      }
    }
    (void)hipGraphDestroy(g);
    LBX_HIP(hipGraphLaunch(exec, cap));
    LBX_HIP(hipEventRecord(ev, cap));
    LBX_HIP(hipStreamWaitEvent(user, ev, 0));
    return LB_OK;
  }
  ~GraphRun() {
    if (!on) return;
    if (active) {  // an error left the capture open: close and drop it
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(cap, &g);
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (cap) {
      (void)hipStreamSynchronize(cap);
      (void)hipStreamDestroy(cap);
    }
    if (ev) (void)hipEventDestroy(ev);
  }
};

// Everything one call's streamed steps need.
struct StreamCtx {
  const lb_plan *p;
  const lbx_opts *o;
  const BatchMeta *m;
  const Layout *L;
  char *w;
  bool prof;
  // a-priori mode (the retry of a call): per-step counts known on the host
  // (kst[j], every launched sweep runs, every step starts from q)
  const std::vector<int32_t> *kst = nullptr;
  mutable int64_t seq = 0;  // steps launched by the call (parity of the maxima slots)
  StepArgs base() const {
    StepArgs A{};
    A.sysv = p->d_sys;
    A.Etab = p->d_E;
    A.desc = p->d_desc;
    A.ctab = (const double2 *)(w + L->ctab);
    A.ttab = (const double2 *)(w + L->ttab);
    A.NT = p->NT;
    A.nsys = (int)p->sys.size();
    A.z0 = (double2 *)(w + L->z0);
    A.z1 = (double2 *)(w + L->z1);
    A.slots = (unsigned long long *)(w + L->slots);
    A.kstep = (int32_t *)(w + L->kstep);
    A.kout = prof ? (int32_t *)(w + L->kout) : nullptr;
    A.status = (int32_t *)(w + L->status);
    A.tol = o->tol;
    A.kcap = 64;
    A.B = m->tile_B;
    A.segs = m->d_segs;
    A.nseg = (int)m->segs.size();
    A.nblk = m->st_blocks;
    return A;
  }
};

// History of one streamed pass: the start iterate of the next step and the
// ring of converged increments; n counts the steps taken in the pass.
struct PassHist {
  double2 *zs = nullptr;
  double2 *ring = nullptr;
  int H = 0;
  int n = 0;
};

// One implicit-midpoint step of every streamed system, q -> out at step j:
// the sweep launches of the stage solve (each runs only if the step needs it).
// Restarted GMRES on the stage system of step j of the whole streamed batch
// (App. A eq. linsystem_primal; eq. linsystem_adjoint when adj), right
// preconditioned by W = (1 - h D)^{-1}, from y = q (z = W q, the start of the
// splitting iteration).  Classical Gram-Schmidt twice per Arnoldi step;
// complex Givens rotations on the host.  Ends when the true residual
// ||q - A z|| is at most KRY_RTOL ||q|| (or, after KRY_RESTARTS cycles,
// KRY_ACCEPT ||q||), then writes out = 2 z - q and zh = z like the last
// sweep.  Synchronises the stream at every Arnoldi step.
constexpr double KRY_RTOL = 1e-15;
constexpr double KRY_ACCEPT = 1e-13;
constexpr int KRY_RESTARTS = 60;

int krylov_step(const StreamCtx &c, int j, bool adj, const double2 *q, double2 *out, double2 *zh, hipStream_t st) {
  typedef std::complex<double> cd;
  const lb_plan *p = c.p;
  const BatchMeta &m = *c.m;
  const Layout &L = *c.L;
  const int64_t E = m.st_entries;
  if (!L.kry) return fail(LB_EINVAL, "internal: Krylov step without its workspace");
  double2 *V = (double2 *)(c.w + L.kry);
  double2 *Y = V + (int64_t)(KRY_M + 1) * E;
  double2 *U = V + (int64_t)(KRY_M + 2) * E;
  double2 *part = (double2 *)(c.w + L.kpart);
  double2 *dres = part + (size_t)1024 * KRY_MAXV;
  const KryArgs A{p->d_sys, p->d_E, p->d_desc, (const double2 *)(c.w + L.ctab), m.d_segs, (int)m.segs.size(),
                  m.st_blocks, j};
  double2 hbuf[KRY_MAXV];
  auto dots = [&](const double2 *Vb, int n, const double2 *x, cd *res) -> int {
    if (int rc = launch_kry_dots(Vb, E, n, x, E, part, dres, st)) return rc;
    LBX_HIP(hipMemcpyAsync(hbuf, dres, n * sizeof(double2), hipMemcpyDeviceToHost, st));
    LBX_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) res[i] = cd(hbuf[i].x, hbuf[i].y);
    return LB_OK;
  };
  auto norm = [&](const double2 *x, double *r) -> int {
    cd v;
    if (int rc = dots(x, 1, x, &v)) return rc;
    *r = std::sqrt(std::max(0.0, v.real()));
    return LB_OK;
  };
  // B x into y (q - B x when q is given)
  auto bapply = [&](const double2 *x, const double2 *qq, double2 *y) -> int {
    if (int rc = launch_kry_weight(A, adj, x, U, st)) return rc;
    return launch_kry_apply(A, adj, U, qq, y, st);
  };
  auto axpy = [&](int n, const cd *cf, double s, double2 *x) -> int {
    KryCoef k{};
    k.n = n;
    for (int i = 0; i < n; ++i) k.c[i] = make_double2(cf[i].real(), cf[i].imag());
    return launch_kry_axpy(V, E, k, s, x, E, st);
  };
  int rc;
  double qn;
  if ((rc = norm(q, &qn))) return rc;
  LBX_HIP(hipMemcpyAsync(Y, q, (size_t)E * sizeof(double2), hipMemcpyDeviceToDevice, st));
  for (int cyc = 0;; ++cyc) {
    double beta;
    if ((rc = bapply(Y, q, V)) || (rc = norm(V, &beta))) return rc;
    if (beta <= KRY_RTOL * qn) break;
    if (cyc == KRY_RESTARTS) {
      if (beta <= KRY_ACCEPT * qn) break;
      return fail(LB_EUNSUPPORTED, "step " + std::to_string(j) + ": the Krylov stage solve did not converge (" +
                                       "relative residual " + std::to_string(beta / qn) + ")");
    }
    if ((rc = axpy(0, nullptr, 1.0 / beta, V))) return rc;
    cd H[KRY_M + 1][KRY_M], sn[KRY_M], g[KRY_M + 1];
    double cr[KRY_M];
    for (int i = 0; i <= KRY_M; ++i) g[i] = 0.0;
    g[0] = beta;
    int kd = 0;
    for (int k = 0; k < KRY_M; ++k) {
      double2 *W = V + (int64_t)(k + 1) * E;
      cd h1[KRY_MAXV], h2[KRY_MAXV];
      if ((rc = bapply(V + (int64_t)k * E, nullptr, W))) return rc;
      if ((rc = dots(V, k + 1, W, h1)) || (rc = axpy(k + 1, h1, 1.0, W))) return rc;
      if ((rc = dots(V, k + 1, W, h2)) || (rc = axpy(k + 1, h2, 1.0, W))) return rc;
      double hn;
      if ((rc = norm(W, &hn))) return rc;
      for (int i = 0; i <= k; ++i) H[i][k] = h1[i] + h2[i];
      // earlier rotations, then the one that removes H[k+1][k] = hn
      for (int i = 0; i < k; ++i) {
        const cd x = H[i][k], y = H[i + 1][k];
        H[i][k] = cr[i] * x + sn[i] * y;
        H[i + 1][k] = -std::conj(sn[i]) * x + cr[i] * y;
      }
      const cd a = H[k][k];
      const double ta = std::abs(a), r = std::hypot(ta, hn);
      if (r == 0.0) {  // breakdown with a zero column: the space is exhausted
        kd = k;
        break;
      }
      if (ta == 0.0) {
        cr[k] = 0.0;
        sn[k] = 1.0;
        H[k][k] = hn;
      } else {
        cr[k] = ta / r;
        sn[k] = (a / ta) * hn / r;
        H[k][k] = (a / ta) * r;
      }
      g[k + 1] = -std::conj(sn[k]) * g[k];
      g[k] = cr[k] * g[k];
      kd = k + 1;
      if (hn > 0.0)
        if ((rc = axpy(0, nullptr, 1.0 / hn, W))) return rc;
      if (std::abs(g[k + 1]) <= KRY_RTOL * qn || hn == 0.0) break;
    }
    // y = R^{-1} g; Y += sum y_i V_i
    cd yv[KRY_MAXV];
    for (int i = kd - 1; i >= 0; --i) {
      cd sacc = g[i];
      for (int l = i + 1; l < kd; ++l) sacc -= H[i][l] * yv[l];
      yv[i] = sacc / H[i][i];
    }
    for (int i = 0; i < kd; ++i) yv[i] = -yv[i];
    if (kd > 0)
      if ((rc = axpy(kd, yv, 1.0, Y))) return rc;
  }
  return launch_kry_finish(A, adj, Y, q, out, zh, st);
}

// gq0, gq1, gpart (block-tiled adjoint steps): the forward states q^j, q^{j+1}
// and the partial-sum rows of the gradient integrands the last sweep forms.
int stream_step(const StreamCtx &c, int j, bool adj, const double2 *q, double2 *out, PassHist &ph, double2 *zh,
                hipStream_t st, const double2 *gq0 = nullptr, const double2 *gq1 = nullptr,
                double *gpart = nullptr) {
  if (c.kst && (*c.kst)[j] < 0) {  // Krylov fallback step
    ph.n++;
    return krylov_step(c, j, adj, q, out, zh, st);
  }
  StepArgs A = c.base();
  A.j = j;
  A.q = q;
  A.out = out;
  A.zh = zh;
  A.gq0 = gq0;
  A.gq1 = gq1;
  A.gpart = gpart;
  A.par = (int)(c.seq++ & 1);
  const int H = c.kst ? 0 : ph.H;
  A.H = H;
  A.n = ph.n;
  A.m = H > 0 ? std::min(ph.n + 1, H) : 0;
  A.zstart = (H > 0 && ph.n > 0) ? ph.zs : nullptr;
  A.znext = H > 0 ? ph.zs : nullptr;
  A.ring = ph.ring;
  A.ring_stride = c.m->st_entries;
  if (c.kst) {
    A.apriori = 1;
    A.L = std::max(2, (*c.kst)[j]);
  } else if (c.o->sweeps > 0) {
    A.L = c.o->sweeps;
  } else {
    A.L = (H > 0 && ph.n >= H) ? SWEEPS_HIST : SWEEPS_START;
  }
  ProfScope ps(c.p, c.prof, LB_KERNEL_SWEEP, st);  // one timed unit per step
  for (int kk = 0; kk < A.L; ++kk)
    if (int rc = launch_sweep(c.p, A, kk, adj, c.m->tile_sys, c.m->tile_k, st)) return rc;
  ph.n++;
  return LB_OK;
}

// A-priori sweep counts from q of every step (the largest over the streamed
// systems), read on the host: the counts of a call repeated after
// LB_STATUS_RETRY.  With `krylov` a step whose contraction bound is >= 0.5
// for any streamed system gets -1 (solved by krylov_step); otherwise such a
// step is an error.  Synchronises the stream.
int apriori_counts(const lb_plan *p, const BatchMeta &m, const int32_t *d_ktab, std::vector<int32_t> &kst,
                   hipStream_t st, bool krylov = false) {
  const size_t n = p->sys.size() * (size_t)p->NT * 2;
  std::vector<int32_t> k(n);
  LBX_HIP(hipMemcpyAsync(k.data(), d_ktab, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  LBX_HIP(hipStreamSynchronize(st));
  kst.assign(p->NT, 1);
  for (const auto &sg : m.segs)
    for (int j = 0; j < p->NT; ++j) {
      const int kj = k[((size_t)sg.sys * p->NT + j) * 2 + 1];
      if (kj < 1) {
        if (!krylov)
          return fail(LB_EUNSUPPORTED, "system " + std::to_string(sg.sys) + " step " + std::to_string(j) +
                                           ": the stage-solve contraction bound is >= 0.5 (step or control "
                                           "amplitude too large)");
        kst[j] = -1;
      } else if (kst[j] >= 0) {
        kst[j] = std::max(kst[j], kj);
      }
    }
  return LB_OK;
}

struct NoHook {
  int operator()(int, const double2 *, hipStream_t) const { return LB_OK; }
};

// Streamed forward steps j0..j1-1.  slot(j) returns the buffer that receives
// q^j (j > j0); q^{j0} is `qstart`.  hook(j, q^j, stream) runs before step j.
// Each call starts a fresh history.
template <class Slot, class Hook = NoHook>
int stream_forward(const StreamCtx &c, int j0, int j1, const double2 *qstart, Slot slot, hipStream_t user,
                   Hook hook = Hook()) {
  GraphRun gr(*c.o, user);
  if (int rc = gr.init()) return rc;
  const hipStream_t st = gr.stream();
  const int chunk = gr.on ? c.o->graph_steps : std::max(1, j1 - j0);
  PassHist ph;
  ph.H = c.L->H;
  ph.zs = (double2 *)(c.w + c.L->zsf);
  ph.ring = (double2 *)(c.w + c.L->ringf);
  const double2 *cur = qstart;
  for (int c0 = j0; c0 < j1; c0 += chunk) {
    const int c1 = std::min(j1, c0 + chunk);
    if (int rc = gr.begin()) return rc;
    for (int j = c0; j < c1; ++j) {
      if (int rc = hook(j, cur, st)) return rc;
      double2 *out = slot(j + 1);
      if (int rc = stream_step(c, j, false, cur, out, ph, nullptr, st)) return rc;
      cur = out;
    }
    if (int rc = gr.end()) return rc;
  }
  return LB_OK;
}

// Adds the entry-sweeps of one LDS-resident pass to the profile (read back
// from the kernels: a synchronisation, only while profiling).
int lds_profile_work(const lb_plan *p, const BatchMeta &m, int kernel, const int64_t *slots, hipStream_t st) {
  if (!slots || m.items.empty()) return LB_OK;
  std::vector<int64_t> sw(m.items.size());
  LBX_HIP(hipMemcpyAsync(sw.data(), slots, sw.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  LBX_HIP(hipStreamSynchronize(st));
  int64_t work = 0;
  for (size_t i = 0; i < m.items.size(); ++i) work += sw[i] * p->sys[m.items[i].sys].N2;
  prof_add_work(p, kernel, work);
  return LB_OK;
}

// Adds the entry-sweeps of the streamed steps of a call (kout) to the profile.
int stream_profile_work(const lb_plan *p, const BatchMeta &m, const int32_t *kout, hipStream_t st) {
  if (m.segs.empty()) return LB_OK;
  const size_t n = p->sys.size() * (size_t)p->NT;
  std::vector<int32_t> k(n);
  LBX_HIP(hipMemcpyAsync(k.data(), kout, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  LBX_HIP(hipStreamSynchronize(st));
  int64_t work = 0;
  for (const auto &sg : m.segs) {
    int64_t ks = 0;
    for (int j = 0; j < p->NT; ++j) ks += k[(size_t)sg.sys * p->NT + j];
    work += ks * sg.count;
  }
  prof_add_work(p, LB_KERNEL_SWEEP, work);
  return LB_OK;
}

// Start of a call: status word, maxima slots and profiling counters cleared.
int call_begin(const lb_plan *p, const Layout &L, char *w, bool prof, hipStream_t st) {
  if (int rc = launch_fill_zero(w + L.status, 4, st)) return rc;
  if (int rc = launch_slots_clear((unsigned long long *)(w + L.slots), (int)p->sys.size(), st)) return rc;
  if (prof)
    if (int rc = launch_fill_zero(w + L.kout, p->sys.size() * (size_t)p->NT * sizeof(int32_t), st)) return rc;
  return LB_OK;
}

// End of an attempt: profiling read-back, then (LB_OPT_SYNC) the status bits.
int call_end(const lb_plan *p, const lbx_opts &o, const BatchMeta &m, const Layout &L, char *w, bool prof,
             hipStream_t st, int32_t *bits) {
  *bits = 0;
  if (prof) {
    if (int rc = stream_profile_work(p, m, (const int32_t *)(w + L.kout), st)) return rc;
    prof_resolve(p);
  }
  if (o.sync) return read_status((const int32_t *)(w + L.status), st, bits);
  return LB_OK;
}

// A call's batch metadata and workspace layout: the usual ones, or those of
// the Krylov fallback (every system streamed, GMRES vectors, no history).
struct CallPlan {
  BatchMeta *m = nullptr;
  Layout L;
};

// Runs attempt(o, plan, kst, bits) (kst NULL: device-side counts).  In
// LB_OPT_SYNC mode:
// * a step whose stage-solve contraction bound is >= 0.5 (LB_STATUS_THETA)
//   makes the call run once more in the Krylov fallback: fallback(&plan)
//   gives its metadata and layout, steps with the bound below 0.5 run their
//   a-priori sweep counts and the others restarted GMRES;
// * a step that needed more sweeps than were launched (LB_STATUS_RETRY)
//   makes the call run once more with the a-priori counts of every step.
// The result is the status of the last run.
template <class Attempt, class Fallback>
int run_call(const lb_plan *p, const lbx_opts &o, const CallPlan &cp, size_t ws_bytes, char *w, hipStream_t st,
             Attempt attempt, Fallback fallback) {
  int32_t bits = 0;
  int rc = attempt(o, cp, nullptr, &bits);
  if (rc || !o.sync) return rc;
  if (bits & LB_STATUS_THETA) {
    CallPlan fp;
    if ((rc = fallback(&fp))) return rc;
    if (ws_bytes < fp.L.total)
      return fail(LB_ENOMEM, "workspace too small for the Krylov fallback of this call (size it with "
                             "lb_workspace_bytes)");
    std::vector<int32_t> kst;
    // the tables of the first run (same offsets in both layouts)
    if ((rc = apriori_counts(p, *fp.m, (const int32_t *)(w + cp.L.ktab), kst, st, true))) return rc;
    lbx_opts of = o;
    of.graph_steps = 0;  // the Krylov steps synchronise
    bits = 0;
    if ((rc = attempt(of, fp, &kst, &bits))) return rc;
    return status_code(bits);
  }
  if ((bits & LB_STATUS_RETRY) && !(bits & LB_STATUS_NONFINITE)) {
    std::vector<int32_t> kst;
    if ((rc = apriori_counts(p, *cp.m, (const int32_t *)(w + cp.L.ktab), kst, st))) return rc;
    bits = 0;
    if ((rc = attempt(o, cp, &kst, &bits))) return rc;
  }
  return status_code(bits);
}

// Work of one call spread over the plan's side streams: each side stream it
// uses first waits for what `st` holds at begin(), and `st` waits for all of
// them at join() (also on the way out of an error).
struct Fork {
  const lb_plan *p;
  hipStream_t st;
  bool on;
  hipEvent_t start = nullptr;
  bool used[4] = {};
  Fork(const lb_plan *p_, hipStream_t s, bool want) : p(p_), st(s), on(want && p_->naux > 0) {}
  int begin() {
    if (!on) return LB_OK;
    LBX_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    LBX_HIP(hipEventRecord(start, st));
    return LB_OK;
  }
  // The stream of item k.
  int stream(int k, hipStream_t *out) {
    if (!on) {
      *out = st;
      return LB_OK;
    }
    const int i = k % p->naux;
    if (!used[i]) {
      LBX_HIP(hipStreamWaitEvent(p->aux[i], start, 0));
      used[i] = true;
    }
    *out = p->aux[i];
    return LB_OK;
  }
  int join() {
    if (!on) return LB_OK;
    on = false;
    int rc = LB_OK;
    for (int i = 0; i < p->naux; ++i)
      if (used[i]) {
        hipEvent_t e;
        hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (r == hipSuccess) r = hipEventRecord(e, p->aux[i]);
        if (r == hipSuccess) r = hipStreamWaitEvent(st, e, 0);
        (void)hipEventDestroy(e);
        if (r != hipSuccess && rc == LB_OK) rc = hip_fail(r, "side-stream join");
      }
    (void)hipEventDestroy(start);
    return rc;
  }
  ~Fork() { (void)join(); }
};

// Running penalty of one gradient call (null when gamma1 = 0): the merit
// functional, its target, the weight table and the accumulators.
struct Penalty {
  int kind;
  const double2 *rhotar;
  const double *ptab;
  double *acc, *part;
};

int run_forward(const lb_plan *p, const lbx_opts &o, const BatchMeta &m, const Layout &L, char *w,
                const double *alpha, const double2 *rho0, double2 *rhoT, char *traj, bool prof,
                const std::vector<int32_t> *kst, hipStream_t st, const Penalty *pen = nullptr) {
  double2 *ctab = (double2 *)(w + L.ctab);
  int32_t *ktab = (int32_t *)(w + L.ktab);
  double2 *ttab = (double2 *)(w + L.ttab);
  int32_t *status = (int32_t *)(w + L.status);
  int rc;
  if ((rc = launch_control_table(p, 0, (int)p->sys.size(), alpha, ctab, 0, ktab, ttab, o.tol, st))) return rc;
  // LDS-resident systems: one persistent launch per kernel class, each on a
  // side stream of its own beside the streamed systems.
  double2 *hist = traj ? (double2 *)(traj + L.T.hist) : nullptr;
  int64_t *slots = prof ? (int64_t *)(w + L.sweeps) : nullptr;
  Fork fk(p, st, m.classes.size() > 1 || (!m.classes.empty() && !m.segs.empty()));
  if ((rc = fk.begin())) return rc;
  for (size_t ci = 0; ci < m.classes.size(); ++ci) {
    const auto &c = m.classes[ci];
    hipStream_t cs;
    if ((rc = fk.stream((int)ci, &cs))) return rc;
    ProfScope ps(p, prof, LB_KERNEL_LDS_FORWARD, cs);
    rc = c.qc > 0 ? launch_lds_forward_fast(p, m.d_items + c.i0, c.i1 - c.i0, c.block, c.ept, c.qc, ctab, ttab,
                                            o.tol, rho0, rhoT, hist, slots ? slots + c.i0 : nullptr, status, cs)
                  : launch_lds_forward(p, m.d_items + c.i0, c.i1 - c.i0, c.block, c.ept, ctab, ktab, rho0, rhoT,
                                       hist, slots ? slots + c.i0 : nullptr, status, cs);
    if (rc) return rc;
    if (pen) {
      if (!hist) return fail(LB_EINVAL, "internal: running penalty without a state history");
      if ((rc = launch_penalty_lds(p, pen->kind, m.d_items + c.i0, c.i1 - c.i0, hist, pen->rhotar, pen->ptab,
                                   pen->part + (size_t)c.i0 * PEN_PARTS, cs)))
        return rc;
    }
  }
  if (m.segs.empty()) {
    if ((rc = fk.join())) return rc;
    return lds_profile_work(p, m, LB_KERNEL_LDS_FORWARD, slots, st);
  }
  // Streamed systems: the sweeps of every step over all of them.
  StreamCtx sc{p, &o, &m, &L, w, prof, kst};
  double2 *q0 = (double2 *)(w + L.q0), *q1 = (double2 *)(w + L.q1);
  const size_t E = (size_t)m.st_entries;
  double2 *ck = traj ? (double2 *)(traj + L.T.ckpt) : nullptr;
  double2 *start = ck ? ck : q0;
  if ((rc = copy_segments(m, rho0, true, start, st))) return rc;
  const int NT = p->NT, c = L.T.c;
  const double2 *last_out = start;
  auto slot = [&](int j) -> double2 * {
    double2 *r;
    if (ck && (j % c == 0 || j == NT)) r = ck + (size_t)(j == NT ? L.T.nck - 1 : j / c) * E;
    else r = (last_out == q0) ? q1 : q0;
    last_out = r;
    return r;
  };
  const int nseg = (int)m.segs.size();
  auto hook = [&](int j, const double2 *q, hipStream_t s) -> int {
    return pen ? launch_penalty_accum(p, pen->kind, m.d_segs, nseg, m.st_blocks, j, q, pen->rhotar, pen->ptab,
                                      pen->acc, s)
               : LB_OK;
  };
  if (pen && (rc = launch_fill_zero(pen->acc, (size_t)m.st_blocks * sizeof(double), st))) return rc;
  if ((rc = stream_forward(sc, 0, NT, start, slot, st, hook))) return rc;
  if ((rc = fk.join()) || (rc = lds_profile_work(p, m, LB_KERNEL_LDS_FORWARD, slots, st))) return rc;
  return copy_segments(m, last_out, false, rhoT, st);
}

// Adjoint pass and gradient of every system from a forward trajectory.
int run_backward(const lb_plan *p, const lbx_opts &o, const BatchMeta &m, const Layout &L, char *w, int kind,
                 const double *alpha, const char *traj, const double2 *rhotar, const double *beta, double gamma2,
                 const double *gscale, double *grad, bool prof, const std::vector<int32_t> *kst,
                 hipStream_t st, const Penalty *pen = nullptr) {
  int rc;
  double2 *ctab = (double2 *)(w + L.ctab);
  int32_t *ktab = (int32_t *)(w + L.ktab);
  double2 *ttab = (double2 *)(w + L.ttab);
  int32_t *status = (int32_t *)(w + L.status);
  double *gstep = (double *)(w + L.gstep);
  if ((rc = launch_fill_zero(gstep, (size_t)2 * p->ctab_total * sizeof(double), st))) return rc;
  // LDS-resident adjoint: each kernel class on a side stream of its own beside
  // the streamed systems; its gradient rows are reduced after the join.
  LdsItem *items = (LdsItem *)(w + L.items);
  double *gpart = (double *)(w + L.gpart);
  int64_t *slots = prof ? (int64_t *)(w + L.sweeps) : nullptr;
  Fork fk(p, st, m.classes.size() > 1 || (!m.classes.empty() && !m.segs.empty()));
  if (!m.items.empty()) {
    const double2 *hist = (const double2 *)(traj + L.T.hist);
    LBX_HIP(hipMemcpyAsync(items, m.d_items, m.items.size() * sizeof(LdsItem), hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(item_weights_kernel, dim3(((int)m.items.size() + 127) / 128), dim3(128), 0, st, items,
                       (int)m.items.size(), beta, m.d_sys_state0, gscale);
    LBX_HIP(hipGetLastError());
    if ((rc = fk.begin())) return rc;
    for (size_t ci = 0; ci < m.classes.size(); ++ci) {
      const auto &c = m.classes[ci];
      hipStream_t cs;
      if ((rc = fk.stream((int)ci, &cs))) return rc;
      ProfScope ps(p, prof, LB_KERNEL_LDS_ADJOINT, cs);
      if (pen && c.qc > 0) return fail(LB_EINVAL, "internal: running penalty on the specialised LDS kernels");
      rc = c.qc > 0 ? launch_lds_adjoint_fast(p, items + c.i0, c.i1 - c.i0, c.block, c.ept, c.qc, kind, ctab, ttab,
                                              o.tol, rhotar, hist, (double2 *)(w + L.zhist), gpart,
                                              slots ? slots + c.i0 : nullptr, status, cs)
                    : launch_lds_adjoint(p, items + c.i0, c.i1 - c.i0, c.block, c.ept, kind, ctab, ktab, rhotar,
                                         hist, pen ? pen->ptab : nullptr, gpart, slots ? slots + c.i0 : nullptr,
                                         status, cs);
      if (rc) return rc;
    }
  }
  auto lds_tail = [&]() -> int {
    if (m.items.empty()) return LB_OK;
    if (int r = fk.join()) return r;
    if (int r = lds_profile_work(p, m, LB_KERNEL_LDS_ADJOINT, slots, st)) return r;
    return launch_lds_grad_reduce(p, m.d_lds_item_range, (int)m.lds_sys.size(), m.d_lds_sys, items, gpart, gstep,
                                  st);
  };
  // Streamed adjoint with checkpoint recomputation.
  if (!m.segs.empty()) {
    StreamCtx sc{p, &o, &m, &L, w, prof, kst};
    const size_t E = (size_t)m.st_entries;
    const int NT = p->NT, c = L.T.c;
    double2 *ck = (double2 *)(traj + L.T.ckpt);
    double2 *seg = (double2 *)(w + L.seg);
    double2 *qh[2] = {(double2 *)(w + L.qh0), (double2 *)(w + L.qh1)};
    double2 *zh = (double2 *)(w + L.zh);
    double *sgp = (double *)(w + L.st_gpart), *sgf = (double *)(w + L.st_gfin);
    const int64_t gstride = L.grows * 2 * QMAX;  // doubles per step slot
    int pend = 0, jtop = 0;
    int64_t rows = 0;
    const int nseg = (int)m.segs.size();
    const int gk = grad_tile_k(p, m);
    // the last sweep of a block-tiled adjoint step forms its gradient integrands
    const bool fuse = o.fuse_grad && gk > 0 && m.tile_sys >= 0 && tile_grad_fusable(p, m.tile_sys, m.tile_k);
    if ((rc = launch_terminal(p, kind, m.d_segs, nseg, m.st_blocks, ck + (size_t)(L.T.nck - 1) * E, rhotar, beta,
                              m.d_seg_state0, gscale, qh[0], st)))
      return rc;
    PassHist ah;  // the adjoint's history runs across segments
    ah.H = L.H;
    ah.zs = (double2 *)(w + L.zsa);
    ah.ring = (double2 *)(w + L.ringa);
    int cur = 0;
    const int nsegs_t = (NT + c - 1) / c;
    for (int sgi = nsegs_t - 1; sgi >= 0; --sgi) {
      const int j0 = sgi * c, j1 = std::min(NT, j0 + c);
      auto slot = [&](int j) -> double2 * {
        if (j == j0) return ck + (size_t)(j0 / c) * E;
        if (j == j1) return ck + (size_t)(j1 == NT ? L.T.nck - 1 : j1 / c) * E;
        return seg + (size_t)(j - j0 - 1) * E;
      };
      // Recompute q^{j0+1} .. q^{j1-1} from the checkpoint.
      if (j1 - j0 > 1)
        if ((rc = stream_forward(sc, j0, j1 - 1, slot(j0), slot, st))) return rc;
      GraphRun gr(o, st);
      if ((rc = gr.init())) return rc;
      const hipStream_t ast = gr.stream();
      const int chunk = gr.on ? o.graph_steps : c;
      for (int ce = j1; ce > j0; ce -= chunk) {
        const int cb = std::max(j0, ce - chunk);
        if ((rc = gr.begin())) return rc;
        for (int j = ce - 1; j >= cb; --j) {
          // Partial rows of the pending steps go to successive slots and are
          // reduced together (every gbatch steps and at the end of a chunk).
          if (pend == 0) jtop = j;
          double *gp = sgp + (size_t)pend * gstride;
          const bool fj = fuse && !(kst && (*kst)[j] < 0);  // not a Krylov step
          if (fj) {
            if ((rc = stream_step(sc, j, true, qh[cur], qh[cur ^ 1], ah, nullptr, ast, slot(j), slot(j + 1), gp)))
              return rc;
            rows = tile_grad_rows(p, m.tile_sys, m.tile_B, gk);
          } else {
            // The last sweep also writes the stage vector zh = qh^{j+1} + delta
            // = (qh^j + qh^{j+1})/2.
            if ((rc = stream_step(sc, j, true, qh[cur], qh[cur ^ 1], ah, zh, ast))) return rc;
            ProfScope ps(p, prof, LB_KERNEL_STREAM_GRAD, ast, m.st_entries);
            rc = gk > 0 ? launch_tile_grad(p, m.tile_sys, m.tile_B, gk, zh, slot(j), slot(j + 1), gp, &rows, ast)
                        : launch_stream_grad(p, m.d_segs, nseg, m.st_blocks, zh, slot(j), slot(j + 1), gp, ast);
            if (rc) return rc;
          }
          if (++pend == L.gbatch || j == cb) {
            if ((rc = launch_stream_grad_finalize(p, m.d_segs, nseg, jtop, pend, sgp, gstride, sgf, gstep, rows,
                                                  ast)))
              return rc;
            pend = 0;
          }
          // Source of the running penalty at q^j (App. B); none at j = 0,
          // where it would not reach the gradient.
          if (pen && j > 0)
            if ((rc = launch_penalty_source(p, pen->kind, m.d_segs, nseg, m.st_blocks, j, slot(j), pen->rhotar,
                                            pen->ptab, gscale, qh[cur ^ 1], ast)))
              return rc;
          cur ^= 1;
        }
        if ((rc = gr.end())) return rc;
      }
    }
  }
  if ((rc = lds_tail())) return rc;
  return launch_grad_contract(p, gstep, alpha, gamma2, gscale, grad, st);
}

}  // namespace

// ----------------------------------------------------------------------------
// Plan
// ----------------------------------------------------------------------------
extern "C" int lb_plan_create(const lb_system_desc *desc, int32_t nsys, lb_plan **out) {
  if (!out) return fail(LB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!desc || nsys <= 0) return fail(LB_EINVAL, "no systems");
  std::unique_ptr<lb_plan> p(new lb_plan());
  std::vector<double> E;
  std::vector<uint64_t> dg;
  std::vector<double> car;
  int64_t tab = 0, aoff = 0, coff = 0, ctoff = 0;
  for (int s = 0; s < nsys; ++s) {
    const lb_system_desc &d = desc[s];
    const std::string who = "system " + std::to_string(s) + ": ";
    if (d.Q < 1 || d.Q > QMAX) return fail(LB_EINVAL, who + "Q must be in 1..12");
    if (!d.nlev || !d.detuning || !d.selfkerr || !d.crosskerr || !d.T1 || !d.T2 || !d.carrier)
      return fail(LB_EINVAL, who + "NULL parameter array");
    if (d.Ns < 3) return fail(LB_EINVAL, who + "Ns must be >= 3");
    if (d.Nf < 1) return fail(LB_EINVAL, who + "Nf must be >= 1");
    if (!(d.T > 0.0) || !std::isfinite(d.T)) return fail(LB_EINVAL, who + "T must be finite and > 0");
    if (d.NT < 1) return fail(LB_EINVAL, who + "NT must be >= 1");
    if (s > 0 && d.NT != desc[0].NT) return fail(LB_EINVAL, who + "all systems of a plan must share NT");
    SysDev S{};
    S.Q = d.Q;
    int64_t N = 1;
    for (int q = 0; q < d.Q; ++q) {
      if (d.nlev[q] < 1 || d.nlev[q] > LB_LIMIT_NLEV) return fail(LB_EINVAL, who + "nlev must be in 1..31");
      S.nlev[q] = d.nlev[q];
      N *= d.nlev[q];
      if (N > (1 << 20)) return fail(LB_EUNSUPPORTED, who + "N too large");
    }
    for (int q = 0; q < d.Q * d.Q; ++q)
      if (!std::isfinite(d.crosskerr[q])) return fail(LB_EINVAL, who + "non-finite cross-Kerr");
    for (int q = 0; q < d.Q; ++q) {
      if (!std::isfinite(d.detuning[q]) || !std::isfinite(d.selfkerr[q]))
        return fail(LB_EINVAL, who + "non-finite detuning or self-Kerr");
      if (std::isnan(d.T1[q]) || std::isnan(d.T2[q])) return fail(LB_EINVAL, who + "NaN T1/T2");
      for (int f = 0; f < d.Nf; ++f)
        if (!std::isfinite(d.carrier[q * d.Nf + f])) return fail(LB_EINVAL, who + "non-finite carrier");
    }
    S.N = (int32_t)N;
    S.N2 = N * N;
    S.NT = d.NT;
    S.Ns = d.Ns;
    S.Nf = d.Nf;
    S.nalpha = 2 * d.Q * d.Ns * d.Nf;
    int64_t stride = 1;
    for (int q = d.Q - 1; q >= 0; --q) {
      S.stride[q] = (int32_t)stride;
      stride *= d.nlev[q];
    }
    S.T = d.T;
    S.dt = d.T / d.NT;
    S.h = 0.5 * S.dt;
    S.dtau = d.T / (d.Ns - 2);
    double theta_jump = 0.0, gmax = 0.0;
    for (int q = 0; q < d.Q; ++q) {
      const int nl = d.nlev[q];
      S.g1[q] = (std::isfinite(d.T1[q]) && d.T1[q] > 0) ? 1.0 / d.T1[q] : 0.0;
      S.g2[q] = (std::isfinite(d.T2[q]) && d.T2[q] > 0) ? 1.0 / d.T2[q] : 0.0;
      double cs = 0.0;
      for (int n = 0; n < nl; ++n) {
        const double v = (n > 0 ? std::sqrt((double)n) : 0.0) + (n + 1 < nl ? std::sqrt((double)(n + 1)) : 0.0);
        cs = std::max(cs, v);
      }
      S.csum[q] = cs;
      theta_jump += S.g1[q] * (nl - 1);
      gmax += S.g1[q] * (nl - 1) + 0.5 * S.g2[q] * (nl - 1) * (nl - 1);
    }
    // Jaynes-Cummings pairs (Sec. II), p > q, with their share of the
    // contraction bound: a pair's row and column terms each sum to at most
    // |g| max over digits of (sqrt(n_p) sqrt(n_q+1) + sqrt(n_p+1) sqrt(n_q)).
    S.njc = 0;
    if (d.jc) {
      for (int pp = 0; pp < d.Q; ++pp)
        for (int qq = 0; qq < pp; ++qq) {
          const double g = d.jc[pp * d.Q + qq];
          if (!std::isfinite(g)) return fail(LB_EINVAL, who + "non-finite Jaynes-Cummings coupling");
          if (g == 0.0) continue;
          const double dr = d.rotfreq ? d.rotfreq[pp] - d.rotfreq[qq] : 0.0;
          if (!std::isfinite(dr)) return fail(LB_EINVAL, who + "non-finite rotation frequency");
          const int k = S.njc++;
          S.jp[k] = (int8_t)pp;
          S.jq[k] = (int8_t)qq;
          S.jg[k] = TWO_PI * g;
          S.jd[k] = TWO_PI * dr;
          const int lp = d.nlev[pp], lq = d.nlev[qq];
          double rmax = 0.0;
          for (int np = 0; np < lp; ++np)
            for (int nq = 0; nq < lq; ++nq) {
              double v = 0.0;
              if (np > 0 && nq + 1 < lq) v += std::sqrt((double)np * (nq + 1));
              if (np + 1 < lp && nq > 0) v += std::sqrt((double)(np + 1) * nq);
              rmax = std::max(rmax, v);
            }
          theta_jump += 2.0 * std::fabs(S.jg[k]) * rmax;
        }
    }
    S.theta_jump = S.h * theta_jump;
    // Energies of H_sys (Sec. II), rad/ns, and digit tables.
    double emin = 1e300, emax = -1e300;
    for (int64_t i = 0; i < N; ++i) {
      int dig[QMAX];
      int64_t rem = i;
      uint64_t packed = 0;
      for (int q = d.Q - 1; q >= 0; --q) {
        dig[q] = (int)(rem % d.nlev[q]);
        rem /= d.nlev[q];
      }
      double e = 0.0;
      for (int q = 0; q < d.Q; ++q) {
        packed |= (uint64_t)dig[q] << (DIGIT_BITS * q);
        const double n = dig[q];
        e += d.detuning[q] * n - 0.5 * d.selfkerr[q] * n * (n - 1.0);
        for (int r = q + 1; r < d.Q; ++r) e -= d.crosskerr[q * d.Q + r] * n * dig[r];
      }
      e *= TWO_PI;
      E.push_back(e);
      dg.push_back(packed);
      emin = std::min(emin, e);
      emax = std::max(emax, e);
    }
    S.hDmax = S.h * ((emax - emin) + gmax);
    S.tab_off = tab;
    tab += N;
    S.carrier_off = coff;
    for (int q = 0; q < d.Q * d.Nf; ++q) car.push_back(d.carrier[q]);
    coff += (int64_t)d.Q * d.Nf;
    S.alpha_off = aoff;
    aoff += S.nalpha;
    S.ctab_off = ctoff;
    ctoff += (int64_t)d.NT * d.Q;
    p->sys.push_back(S);
  }
  p->NT = desc[0].NT;
  p->ctab_total = ctoff;
  if (hipGetDevice(&p->device) != hipSuccess) return fail(LB_EDEVICE, "no HIP device");
  auto cleanup = [&](int rc) {
    (void)hipFree(p->d_sys);
    (void)hipFree(p->d_E);
    (void)hipFree(p->d_desc);
    (void)hipFree(p->d_carrier);
    return rc;
  };
  hipError_t e;
  if ((e = hipMalloc(&p->d_sys, p->sys.size() * sizeof(SysDev))) != hipSuccess ||
      (e = hipMalloc(&p->d_E, E.size() * sizeof(double))) != hipSuccess ||
      (e = hipMalloc(&p->d_desc, dg.size() * sizeof(uint64_t))) != hipSuccess ||
      (e = hipMalloc(&p->d_carrier, car.size() * sizeof(double))) != hipSuccess)
    return cleanup(hip_fail(e, "hipMalloc(plan tables)"));
  if ((e = hipMemcpy(p->d_sys, p->sys.data(), p->sys.size() * sizeof(SysDev), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->d_E, E.data(), E.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->d_desc, dg.data(), dg.size() * sizeof(uint64_t), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->d_carrier, car.data(), car.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMemcpy(plan tables)"));
  for (auto &a : p->aux) {
    if (hipStreamCreateWithFlags(&a, hipStreamNonBlocking) != hipSuccess) {
      a = nullptr;
      break;
    }
    p->naux++;
  }
  *out = p.release();
  return LB_OK;
}

extern "C" void lb_plan_destroy(lb_plan *p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> g(g_extra_mu);
    auto it = g_extra.find(p);
    if (it != g_extra.end()) {
      for (auto &kv : it->second->batches) (void)hipFree(kv.second->dmem);
      g_extra.erase(it);
    }
  }
  (void)hipFree(p->d_sys);
  (void)hipFree(p->d_E);
  (void)hipFree(p->d_desc);
  (void)hipFree(p->d_carrier);
  for (auto &e : p->prof_pending) {
    (void)hipEventSynchronize(e.stop);
    (void)hipEventDestroy(e.start);
    (void)hipEventDestroy(e.stop);
  }
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  for (int i = 0; i < p->naux; ++i) (void)hipStreamDestroy(p->aux[i]);
  delete p;
}

extern "C" int lb_plan_info(const lb_plan *p, int32_t sys, int32_t *N, int32_t *nalpha, int32_t *NT) {
  if (int rc = check_plan(p)) return rc;
  if (sys < 0 || sys >= (int)p->sys.size()) return fail(LB_EINVAL, "sys out of range");
  if (N) *N = p->sys[sys].N;
  if (nalpha) *nalpha = p->sys[sys].nalpha;
  if (NT) *NT = p->NT;
  return LB_OK;
}

extern "C" int lb_plan_set_option(lb_plan *p, int32_t option, double value) {
  if (int rc = check_plan(p)) return rc;
  std::lock_guard<std::mutex> g(p->mu);
  lbx_opts &o = p->opts;
  if (option == LB_OPT_PATH) {
    if (value != 0 && value != 1 && value != 2) return fail(LB_EINVAL, "LB_OPT_PATH must be 0, 1 or 2");
    o.path = (int)value;
    return LB_OK;
  }
  if (option == LB_OPT_TILE) {
    if (value != 0 && value != 1 && value != 2) return fail(LB_EINVAL, "LB_OPT_TILE must be 0, 1 or 2");
    o.tile = (int)value;
    return LB_OK;
  }
  if (option == LB_OPT_TILE_KI) {
    if (value < 0 || value > LB_SPLIT_BASE + LB_LIMIT_QMAX || value != (int)value)
      return fail(LB_EINVAL, "LB_OPT_TILE_KI must be 0..99 (block shape) or 101..111 (two-pass split)");
    o.tile_ki = (int)value;
    return LB_OK;
  }
  if (option == LB_OPT_GRAPH) {
    if (value < 0 || value > 100000 || value != (int)value) return fail(LB_EINVAL, "LB_OPT_GRAPH must be 0..100000");
    o.graph_steps = (int)value;
    return LB_OK;
  }
  if (option == LB_OPT_PROFILE) {
    o.profile = value != 0.0;
    return LB_OK;
  }
  if (option == LB_OPT_SOLVE_TOL) {
    if (!(value > 0.0 && value < 1.0)) return fail(LB_EINVAL, "LB_OPT_SOLVE_TOL must be in (0, 1)");
    o.tol = value;
    return LB_OK;
  }
  if (option == LB_OPT_HISTORY) {
    if (value < 0 || value > 6 || value != (int)value) return fail(LB_EINVAL, "LB_OPT_HISTORY must be 0..6");
    o.history = (int)value;
    return LB_OK;
  }
  if (option == LB_OPT_SWEEPS) {
    if (value != 0 && (value < 2 || value > 64 || value != (int)value))
      return fail(LB_EINVAL, "LB_OPT_SWEEPS must be 0 or 2..64");
    o.sweeps = (int)value;
    return LB_OK;
  }
  if (option == LB_OPT_FUSE_GRAD) {
    o.fuse_grad = value != 0.0;
    return LB_OK;
  }
  if (option == LB_OPT_SYNC) {
    o.sync = value != 0.0;
    return LB_OK;
  }
  return fail(LB_EINVAL, "unknown option");
}

extern "C" int lb_workspace_bytes(const lb_plan *p, int32_t op, const int32_t *batch_per_sys, int32_t ckpt_every,
                                  size_t *bytes) {
  if (int rc = check_plan(p)) return rc;
  if (!batch_per_sys || !bytes) return fail(LB_EINVAL, "NULL argument");
  if (op < LB_OP_IMR_STEP || op > LB_OP_BACKWARD) return fail(LB_EINVAL, "unknown op");
  if (ckpt_every < 0) return fail(LB_EINVAL, "ckpt_every must be >= 0");
  const lbx_opts o = snapshot(p);
  BatchMeta *m;
  // imr_step always streams; only the trajectory-keeping operations honour ckpt_every.
  const bool small = op != LB_OP_IMR_STEP && streams_small(ckpt_every);
  if (int rc = build_batch(p, o, batch_per_sys, small, &m, op == LB_OP_IMR_STEP ? 2 : -1)) return rc;
  const int ck = op == LB_OP_IMR_STEP ? 1 : ckpt_every;
  *bytes = layout(p, o, op, *m, ck).total;
  // room for the generic LDS kernels of a call with a running penalty
  if (op == LB_OP_GRADIENT) {
    BatchMeta *mg;
    if (int rc = build_batch(p, o, batch_per_sys, small, &mg, -1, true)) return rc;
    *bytes = std::max(*bytes, layout(p, o, op, *mg, ck).total);
  }
  // room for the Krylov fallback (every system streamed)
  BatchMeta *mf;
  if (int rc = build_batch(p, o, batch_per_sys, op != LB_OP_IMR_STEP, &mf, 2)) return rc;
  *bytes = std::max(*bytes, layout(p, o, op, *mf, ck, true).total);
  return LB_OK;
}

extern "C" int lb_trajectory_bytes(const lb_plan *p, const int32_t *batch_per_sys, int32_t ckpt_every,
                                   size_t *bytes) {
  if (int rc = check_plan(p)) return rc;
  if (!batch_per_sys || !bytes) return fail(LB_EINVAL, "NULL argument");
  if (ckpt_every < 0) return fail(LB_EINVAL, "ckpt_every must be >= 0");
  const lbx_opts o = snapshot(p);
  BatchMeta *m;
  if (int rc = build_batch(p, o, batch_per_sys, streams_small(ckpt_every), &m)) return rc;
  *bytes = traj_layout(p, *m, ckpt_every).total;
  // the layout of a trajectory written by the Krylov fallback
  BatchMeta *mf;
  if (int rc = build_batch(p, o, batch_per_sys, true, &mf, 2)) return rc;
  *bytes = std::max(*bytes, traj_layout(p, *mf, ckpt_every).total);
  return LB_OK;
}

extern "C" int lb_status(const lb_plan *p, const void *ws, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (!ws) return noalloc_status(p, (hipStream_t)stream);
  return status_code((const int32_t *)ws, (hipStream_t)stream);
}

// ----------------------------------------------------------------------------
// Entry points
// ----------------------------------------------------------------------------
extern "C" int control_table(const lb_plan *p, int32_t sys, const double *alpha, void *table, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (sys < 0 || sys >= (int)p->sys.size()) return fail(LB_EINVAL, "sys out of range");
  if (!alpha || !table) return fail(LB_EINVAL, "NULL argument");
  const lbx_opts o = snapshot(p);
  // alpha is this system's block; the kernel adds alpha_off, so shift it back.
  const double *abase = alpha - p->sys[sys].alpha_off;
  return launch_control_table(p, sys, 1, abase, (double2 *)table, p->sys[sys].ctab_off, nullptr, nullptr, o.tol,
                              (hipStream_t)stream);
}

extern "C" int lindblad_apply(const lb_plan *p, int32_t sys, double t, const double *alpha, const void *x,
                              void *y, int32_t B, int32_t adjoint, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (sys < 0 || sys >= (int)p->sys.size()) return fail(LB_EINVAL, "sys out of range");
  if (B < 0) return fail(LB_EINVAL, "B must be >= 0");
  if (B == 0) return LB_OK;
  if (!alpha || !x || !y) return fail(LB_EINVAL, "NULL argument");
  if (!std::isfinite(t)) return fail(LB_EINVAL, "t must be finite");
  const size_t bytes = (size_t)B * p->sys[sys].N2 * sizeof(double2);
  const char *xa = (const char *)x, *ya = (const char *)y;
  if (xa < ya + bytes && ya < xa + bytes) return fail(LB_EINVAL, "x and y overlap");
  const lbx_opts o = snapshot(p);
  return launch_apply(p, sys, t, alpha, (const double2 *)x, (double2 *)y, B, adjoint != 0, o.tile, o.tile_ki,
                      (hipStream_t)stream);
}

extern "C" int imr_step(const lb_plan *p, int32_t sys, int32_t j, const double *alpha, const void *q_in,
                        void *q_out, int32_t B, int32_t adjoint, void *ws, size_t ws_bytes, void *stream) {
  if (int rc = check_plan(p)) return rc;
  const int nsys = (int)p->sys.size();
  if (sys < 0 || sys >= nsys) return fail(LB_EINVAL, "sys out of range");
  if (j < 0 || j >= p->NT) return fail(LB_EINVAL, "step index out of range");
  if (B < 0) return fail(LB_EINVAL, "B must be >= 0");
  if (B == 0) return LB_OK;
  if (!alpha || !q_in || !q_out || !ws) return fail(LB_EINVAL, "NULL argument");
  {
    const uintptr_t a = (uintptr_t)q_in, c = (uintptr_t)q_out;
    const size_t bytes = (size_t)B * p->sys[sys].N2 * sizeof(double2);
    if (a < c + bytes && c < a + bytes) return fail(LB_EINVAL, "q_in and q_out overlap");
  }
  const lbx_opts o = snapshot(p);
  hipStream_t st = (hipStream_t)stream;
  std::vector<int32_t> batch(nsys, 0);
  batch[sys] = B;
  CallPlan cp;
  int rc = build_batch(p, o, batch.data(), false, &cp.m, 2);
  if (rc) return rc;
  cp.L = layout(p, o, LB_OP_IMR_STEP, *cp.m, 1);
  if (ws_bytes < cp.L.total) return fail(LB_ENOMEM, "workspace too small");
  char *w = (char *)ws;
  const bool prof = o.profile;
  const double *abase = alpha - p->sys[sys].alpha_off;
  auto attempt = [&](const lbx_opts &oo, const CallPlan &c, const std::vector<int32_t> *kst, int32_t *bits) -> int {
    const lbx_opts &o = oo;
    const Layout &L = c.L;
    BatchMeta *m = c.m;
    double2 *ctab = (double2 *)(w + L.ctab);
    int rc = call_begin(p, L, w, prof, st);
    if (!rc)
      rc = launch_control_table(p, sys, 1, abase, ctab, 0, (int32_t *)(w + L.ktab), (double2 *)(w + L.ttab), o.tol,
                                st);
    // (the tables are written at the system's own offsets, where the sweep
    // kernels read them)
    StreamCtx sc{p, &o, m, &L, w, prof, kst};
    PassHist ph;  // a single step starts from q
    if (!rc) rc = stream_step(sc, j, adjoint != 0, (const double2 *)q_in, (double2 *)q_out, ph, nullptr, st);
    if (rc) return rc;
    return call_end(p, o, *m, L, w, prof, st, bits);
  };
  auto fallback = [&](CallPlan *f) -> int {
    f->m = cp.m;
    f->L = layout(p, o, LB_OP_IMR_STEP, *cp.m, 1, true);
    return LB_OK;
  };
  return run_call(p, o, cp, ws_bytes, w, st, attempt, fallback);
}

extern "C" int forward_solve(const lb_plan *p, const double *alpha, const void *rho0, void *rhoT,
                             const int32_t *batch_per_sys, void *traj, int32_t ckpt_every, void *ws, size_t ws_bytes,
                             void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (!alpha || !rho0 || !rhoT || !batch_per_sys || !ws) return fail(LB_EINVAL, "NULL argument");
  if (ckpt_every < 0) return fail(LB_EINVAL, "ckpt_every must be >= 0");
  const lbx_opts o = snapshot(p);
  CallPlan cp;
  const bool small = traj && streams_small(ckpt_every);
  if (int rc = build_batch(p, o, batch_per_sys, small, &cp.m)) return rc;
  if (cp.m->total_entries == 0) return LB_OK;
  const int ck = traj ? ckpt_every : 1;
  cp.L = layout(p, o, LB_OP_FORWARD, *cp.m, ck);
  if (ws_bytes < cp.L.total) return fail(LB_ENOMEM, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  const bool prof = o.profile;
  auto attempt = [&](const lbx_opts &oo, const CallPlan &c, const std::vector<int32_t> *kst, int32_t *bits) -> int {
    int rc = call_begin(p, c.L, w, prof, st);
    if (!rc)
      rc = run_forward(p, oo, *c.m, c.L, w, alpha, (const double2 *)rho0, (double2 *)rhoT, (char *)traj, prof, kst,
                       st);
    if (rc) return rc;
    return call_end(p, oo, *c.m, c.L, w, prof, st, bits);
  };
  auto fallback = [&](CallPlan *f) -> int {
    if (int rc = build_batch(p, o, batch_per_sys, true, &f->m, 2)) return rc;
    f->L = layout(p, o, LB_OP_FORWARD, *f->m, ck, true);
    return LB_OK;
  };
  return run_call(p, o, cp, ws_bytes, w, st, attempt, fallback);
}

extern "C" int objective(const lb_plan *p, int32_t kind, const void *rhoT, const void *rhotar, const double *beta,
                         const int32_t *batch_per_sys, double gamma2, const double *alpha, double *G, double *J,
                         void *ws, size_t ws_bytes, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (kind != LB_J_FROB && kind != LB_J_TR && kind != LB_J_NM) return fail(LB_EINVAL, "unknown merit functional");
  if (!rhoT || !rhotar || !beta || !batch_per_sys || !alpha || !G || !ws) return fail(LB_EINVAL, "NULL argument");
  if (!std::isfinite(gamma2)) return fail(LB_EINVAL, "gamma2 must be finite");
  const lbx_opts o = snapshot(p);
  BatchMeta *m;
  if (int rc = build_batch(p, o, batch_per_sys, false, &m)) return rc;
  const Layout L = layout(p, o, LB_OP_FORWARD, *m, 1);
  if (ws_bytes < L.total) return fail(LB_ENOMEM, "workspace too small");
  char *w = (char *)ws;
  hipStream_t st = (hipStream_t)stream;
  int32_t *status = (int32_t *)(w + L.status);
  if (int rc = launch_fill_zero(status, 4, st)) return rc;
  if (int rc = launch_objective(p, kind, (const double2 *)rhoT, (const double2 *)rhotar, beta, m->d_state_sys,
                                m->d_state_off, m->d_sys_state0, m->total_states, gamma2, alpha, nullptr,
                                (double *)(w + L.objpart), J, G, status, st))
    return rc;
  if (o.sync) return status_code(status, st);
  return LB_OK;
}

extern "C" int adjoint_backward(const lb_plan *p, int32_t kind, const double *alpha, const void *traj,
                                int32_t ckpt_every, const void *rhotar, const double *beta,
                                const int32_t *batch_per_sys, double gamma2, const double *gscale, double *grad,
                                void *ws, size_t ws_bytes, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (kind != LB_J_FROB && kind != LB_J_TR && kind != LB_J_NM) return fail(LB_EINVAL, "unknown merit functional");
  if (!alpha || !traj || !rhotar || !beta || !batch_per_sys || !grad || !ws) return fail(LB_EINVAL, "NULL argument");
  if (ckpt_every < 0) return fail(LB_EINVAL, "ckpt_every must be >= 0");
  if (!std::isfinite(gamma2)) return fail(LB_EINVAL, "gamma2 must be finite");
  const lbx_opts o = snapshot(p);
  CallPlan cp;
  if (int rc = build_batch(p, o, batch_per_sys, streams_small(ckpt_every), &cp.m)) return rc;
  cp.L = layout(p, o, LB_OP_BACKWARD, *cp.m, ckpt_every);
  if (ws_bytes < cp.L.total) return fail(LB_ENOMEM, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  const bool prof = o.profile;
  auto attempt = [&](const lbx_opts &oo, const CallPlan &c, const std::vector<int32_t> *kst, int32_t *bits) -> int {
    const Layout &L = c.L;
    int rc = call_begin(p, L, w, prof, st);
    // The controls (and their tables) are rebuilt for this call.
    if (!rc)
      rc = launch_control_table(p, 0, (int)p->sys.size(), alpha, (double2 *)(w + L.ctab), 0,
                                (int32_t *)(w + L.ktab), (double2 *)(w + L.ttab), oo.tol, st);
    if (!rc)
      rc = run_backward(p, oo, *c.m, L, w, kind, alpha, (const char *)traj, (const double2 *)rhotar, beta, gamma2,
                        gscale, grad, prof, kst, st);
    if (rc) return rc;
    return call_end(p, oo, *c.m, L, w, prof, st, bits);
  };
  // A trajectory that forward_solve wrote in its Krylov fallback has the
  // fallback's layout; this call meets the same bound and falls back too.
  auto fallback = [&](CallPlan *f) -> int {
    if (int rc = build_batch(p, o, batch_per_sys, true, &f->m, 2)) return rc;
    f->L = layout(p, o, LB_OP_BACKWARD, *f->m, ckpt_every, true);
    return LB_OK;
  };
  return run_call(p, o, cp, ws_bytes, w, st, attempt, fallback);
}

extern "C" int adjoint_gradient(const lb_plan *p, int32_t kind, const double *alpha, const void *rho0,
                                const void *rhotar, const double *beta, const int32_t *batch_per_sys, double gamma2,
                                double gamma1, double penalty_a, int32_t ckpt_every, double *G, double *grad,
                                void *rhoT_out, void *ws, size_t ws_bytes, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (kind != LB_J_FROB && kind != LB_J_TR && kind != LB_J_NM) return fail(LB_EINVAL, "unknown merit functional");
  if (!alpha || !rho0 || !rhotar || !beta || !batch_per_sys || !G || !grad || !ws)
    return fail(LB_EINVAL, "NULL argument");
  if (ckpt_every < 0) return fail(LB_EINVAL, "ckpt_every must be >= 0");
  if (!std::isfinite(gamma2)) return fail(LB_EINVAL, "gamma2 must be finite");
  if (!std::isfinite(gamma1)) return fail(LB_EINVAL, "gamma1 must be finite");
  const bool penal = gamma1 != 0.0;
  if (penal && !(penalty_a > 0.0 && std::isfinite(penalty_a)))
    return fail(LB_EINVAL, "penalty_a must be positive and finite");
  const lbx_opts o = snapshot(p);
  CallPlan cp;
  if (int rc = build_batch(p, o, batch_per_sys, streams_small(ckpt_every), &cp.m, -1, penal)) return rc;
  cp.L = layout(p, o, LB_OP_GRADIENT, *cp.m, ckpt_every);
  if (ws_bytes < cp.L.total) return fail(LB_ENOMEM, "workspace too small");
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  const bool prof = o.profile;
  auto attempt = [&](const lbx_opts &oo, const CallPlan &c, const std::vector<int32_t> *kst, int32_t *bits) -> int {
    const lbx_opts &o = oo;
    const Layout &L = c.L;
    BatchMeta *m = c.m;
    char *traj = w + L.traj;
    // rho(T) goes to the caller's buffer, or to the workspace.
    double2 *rhoT = rhoT_out ? (double2 *)rhoT_out : (double2 *)(w + L.rhoT);
    const Penalty pn{kind, (const double2 *)rhotar, (const double *)(w + L.ptab), (double *)(w + L.pacc),
                     (double *)(w + L.ppart)};
    const Penalty *pen = penal ? &pn : nullptr;
    double *penv = penal ? (double *)(w + L.pen) : nullptr;
    int rc = call_begin(p, L, w, prof, st);
    if (!rc && pen) rc = launch_penalty_table(p, gamma1, penalty_a, (double *)(w + L.ptab), st);
    if (!rc) rc = run_forward(p, o, *m, L, w, alpha, (const double2 *)rho0, rhoT, traj, prof, kst, st, pen);
    if (!rc && pen)
      rc = launch_penalty_final(p, kind, m->d_pen_rng, pn.acc, pn.part, pn.ptab, m->d_sys_state0, penv, st);
    if (!rc)
      rc = launch_objective(p, kind, rhoT, (const double2 *)rhotar, beta, m->d_state_sys, m->d_state_off,
                            m->d_sys_state0, m->total_states, gamma2, alpha, penv, (double *)(w + L.objpart),
                            nullptr, G, (int32_t *)(w + L.status), st);
    if (!rc)
      rc = run_backward(p, o, *m, L, w, kind, alpha, traj, (const double2 *)rhotar, beta, gamma2, nullptr, grad,
                        prof, kst, st, pen);
    if (rc) return rc;
    return call_end(p, o, *m, L, w, prof, st, bits);
  };
  auto fallback = [&](CallPlan *f) -> int {
    if (int rc = build_batch(p, o, batch_per_sys, true, &f->m, 2)) return rc;
    f->L = layout(p, o, LB_OP_GRADIENT, *f->m, ckpt_every, true);
    return LB_OK;
  };
  return run_call(p, o, cp, ws_bytes, w, st, attempt, fallback);
}

extern "C" int lb_profile_read(const lb_plan *p, int32_t kernel, int64_t *launches, double *total_ms, int32_t reset) {
  if (int rc = check_plan(p)) return rc;
  if (kernel < 0 || kernel >= LB_KERNEL_COUNT) return fail(LB_EINVAL, "unknown kernel family");
  prof_resolve(p);
  std::lock_guard<std::mutex> g(p->mu);
  if (launches) *launches = p->prof_n[kernel];
  if (total_ms) *total_ms = p->prof_ms[kernel];
  if (reset) {
    p->prof_n[kernel] = 0;
    p->prof_ms[kernel] = 0.0;
    p->prof_work[kernel] = 0;
  }
  return LB_OK;
}

extern "C" int lb_profile_work(const lb_plan *p, int32_t kernel, int64_t *entry_sweeps) {
  if (int rc = check_plan(p)) return rc;
  if (kernel < 0 || kernel >= LB_KERNEL_COUNT) return fail(LB_EINVAL, "unknown kernel family");
  if (!entry_sweeps) return fail(LB_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(p->mu);
  *entry_sweeps = p->prof_work[kernel];
  return LB_OK;
}

extern "C" int sweep_counts(const lb_plan *p, const double *alpha, int32_t *counts, void *stream) {
  if (int rc = check_plan(p)) return rc;
  if (!alpha || !counts) return fail(LB_EINVAL, "NULL argument");
  const lbx_opts o = snapshot(p);
  hipStream_t st = (hipStream_t)stream;
  const size_t nk = p->sys.size() * (size_t)p->NT * 2;
  void *tmp = nullptr;
  LBX_HIP(hipMalloc(&tmp, align256(p->ctab_total * sizeof(double2)) + nk * sizeof(int32_t)));
  double2 *ctab = (double2 *)tmp;
  int32_t *ktab = (int32_t *)((char *)tmp + align256(p->ctab_total * sizeof(double2)));
  int rc = launch_control_table(p, 0, (int)p->sys.size(), alpha, ctab, 0, ktab, nullptr, o.tol, st);
  if (rc == LB_OK) {
    hipError_t e = hipMemcpyAsync(counts, ktab, nk * sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = hip_fail(e, "sweep_counts copy");
  }
  (void)hipFree(tmp);
  return rc;
}

// ----------------------------------------------------------------------------
// Autotuner: times the kernel configurations of the streamed systems of a
// batch on the caller's workspace and keeps the fastest in the plan.
// ----------------------------------------------------------------------------
namespace {

// Mean time of `reps` first steps (forward, no history) with the options o.
int time_steps(const lb_plan *p, const lbx_opts &o, const BatchMeta &m, const Layout &L, char *w, int reps,
               hipStream_t st, float *ms) {
  StreamCtx sc{p, &o, &m, &L, w, false, nullptr};
  double2 *q0 = (double2 *)(w + L.q0), *q1 = (double2 *)(w + L.q1);
  hipEvent_t a, b;
  LBX_HIP(hipEventCreate(&a));
  LBX_HIP(hipEventCreate(&b));
  int rc = LB_OK;
  PassHist ph;  // H = 0: every step starts from q
  for (int r = 0; r < 2 && !rc; ++r) rc = stream_step(sc, 0, false, q0, q1, ph, nullptr, st);
  if (!rc) (void)hipEventRecord(a, st);
  for (int r = 0; r < reps && !rc; ++r) rc = stream_step(sc, 0, false, (r & 1) ? q1 : q0, (r & 1) ? q0 : q1, ph, nullptr, st);
  if (!rc) {
    (void)hipEventRecord(b, st);
    const hipError_t e = hipEventSynchronize(b);
    if (e != hipSuccess) rc = hip_fail(e, "autotune timing");
    else (void)hipEventElapsedTime(ms, a, b);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

}  // namespace

extern "C" int lb_autotune(lb_plan *p, const double *alpha, const int32_t *batch_per_sys, void *ws, size_t ws_bytes,
                           void *stream, int32_t *result) {
  if (int rc = check_plan(p)) return rc;
  if (!alpha || !batch_per_sys || !ws || !result) return fail(LB_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  lbx_opts o = snapshot(p);
  BatchMeta *m;
  if (int rc = build_batch(p, o, batch_per_sys, false, &m)) return rc;
  result[0] = o.tile;
  result[1] = o.tile_ki;
  result[2] = o.graph_steps;
  if (m->segs.empty()) return LB_OK;
  // The workspace must hold the forward layout of every candidate (the
  // generic and tiled layouts are the same size).
  const Layout L = layout(p, o, LB_OP_FORWARD, *m, 1);
  if (ws_bytes < L.total) return fail(LB_ENOMEM, "workspace too small");
  int rc = launch_control_table(p, 0, (int)p->sys.size(), alpha, (double2 *)(w + L.ctab), 0, (int32_t *)(w + L.ktab),
                                (double2 *)(w + L.ttab), o.tol, st);
  if (rc) return rc;
  const size_t E = (size_t)m->st_entries * sizeof(double2);
  if ((rc = launch_fill_trial((double2 *)(w + L.q0), m->st_entries, st)) ||
      (rc = launch_fill_trial((double2 *)(w + L.q1), m->st_entries, st)))
    return rc;
  if ((rc = launch_slots_clear((unsigned long long *)(w + L.slots), (int)p->sys.size(), st))) return rc;
  // Kernel family and block shape.
  std::vector<std::pair<int, int>> cand = {{0, 0}};
  if (m->segs.size() == 1) {
    const int sys = m->segs[0].sys;
    for (int ki : {44, 43, 34, 42, 33, 66, 55, 32, 23})
      if (tile_ki(p, sys, ki) == ki) cand.push_back({1, ki});
    // two-pass splits with at least 9 rows and columns on both sides
    for (int ka = 1; ka < p->sys[sys].Q; ++ka) {
      SplitGeo g;
      if (split_geo(p, sys, LB_SPLIT_BASE + ka, &g) && g.NA >= 9 && p->sys[sys].N / g.NA >= 9)
        cand.push_back({1, LB_SPLIT_BASE + ka});
    }
  }
  const int reps = m->st_entries > (1 << 22) ? 6 : 20;
  float best = 1e30f;
  int bt = o.tile, bk = o.tile_ki;
  lbx_opts oc = o;
  oc.graph_steps = 0;
  for (const auto &c : cand) {
    oc.tile = c.first;
    oc.tile_ki = c.second;
    BatchMeta *mc;
    if ((rc = build_batch(p, oc, batch_per_sys, false, &mc))) return rc;
    float ms = 0.f;
    if ((rc = time_steps(p, oc, *mc, L, w, reps, st, &ms))) return rc;
    if (ms < best) {
      best = ms;
      bt = c.first;
      bk = c.second;
    }
  }
  {
    std::lock_guard<std::mutex> g(p->mu);
    p->opts.tile = bt;
    p->opts.tile_ki = bk;
  }
  result[0] = bt;
  result[1] = bk;
  result[2] = o.graph_steps;
  return LB_OK;
}

extern "C" const char *lb_last_error(void) { return g_err.c_str(); }

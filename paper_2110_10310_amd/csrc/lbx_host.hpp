// Host-side plan structure and kernel launchers shared by the library's
// translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "lbx.h"
#include "lbx_device.hpp"

struct lbx_prof_pending {
  int kernel;
  int launches;  // kernel launches bracketed by the two events
  hipEvent_t start, stop;
};

// Options of a plan (lb_plan_set_option); every call works on a copy taken
// when it starts, so options may change while other calls are running.
struct lbx_opts {
  int path = 0;                          // LB_OPT_PATH
  int tile = 1;                          // LB_OPT_TILE
  int tile_ki = 0;                       // LB_OPT_TILE_KI (0: default block)
  int graph_steps = 0;                   // LB_OPT_GRAPH (0: launch directly)
  int history = 5;                       // LB_OPT_HISTORY
  int sweeps = 0;                        // LB_OPT_SWEEPS (0: built-in)
  bool fuse_grad = false;                // LB_OPT_FUSE_GRAD
  bool profile = false;                  // LB_OPT_PROFILE
  bool sync = true;                      // LB_OPT_SYNC
  double tol = 1.1102230246251565e-16;   // LB_OPT_SOLVE_TOL (2^-53)
};

struct lb_plan {
  std::vector<lbx::SysDev> sys;   // host copy of the per-system constants
  lbx::SysDev *d_sys = nullptr;   // device copy
  double *d_E = nullptr;          // energies of H_sys per basis index [rad/ns]
  uint64_t *d_desc = nullptr;     // packed subsystem digits per basis index
  double *d_carrier = nullptr;    // carriers [GHz], per system [Q][Nf]
  int32_t NT = 0;                 // common number of steps
  int64_t ctab_total = 0;         // sum over systems of NT*Q
  int device = 0;
  mutable std::mutex mu;          // guards opts and the profiling state
  lbx_opts opts;
  // LB_OPT_PROFILE: per-kernel-family launch counts and durations.
  mutable int64_t prof_n[LB_KERNEL_COUNT] = {};
  mutable double prof_ms[LB_KERNEL_COUNT] = {};
  mutable int64_t prof_work[LB_KERNEL_COUNT] = {};  // entries x sweeps (x steps for STREAM_GRAD)
  mutable std::vector<lbx_prof_pending> prof_pending;
  mutable std::vector<hipEvent_t> ev_pool;  // recycled profiling events
  // side streams (default priority) on which a call runs its LDS-resident
  // kernel classes beside the streamed systems
  hipStream_t aux[4] = {};
  int naux = 0;
};

namespace lbx {

// Work item of the LDS-resident persistent kernels: one state of one system.
struct LdsItem {
  int32_t sys;
  int32_t b;          // state index within its system
  int64_t off;        // first entry of the state in the batched buffers
  int64_t st_off;     // first entry of this item's state history (NT+1 states)
  int64_t gp_off;     // first double of this item's gradient partials [NT][parts][2Q]
  double wterm;       // beta_b / M_s (terminal condition weight)
  int32_t parts;      // gradient partial sums per step written by this item's block
  int32_t pad;
  double wpen;        // 1 / M_s (running-penalty source weight, times the table entry)
};

// Segment of the streaming kernels: all states of one system.
struct StreamSeg {
  int32_t sys;
  int32_t nstates;
  int64_t off;        // first entry in the compact work buffers of streamed states
  int64_t boff;       // first entry in the caller's batched buffers
  int64_t count;      // nstates * N^2
  int64_t blk0;       // first block of the segment in a launch
};

constexpr int STREAM_BLOCK = 256;

// HIP-event timing of `launches` consecutive launches of one kernel family
// when the plan's profiling is on.  Bracketing a run of back-to-back launches
// (the sweeps of one step) keeps the events' own cost from inflating short
// kernels.
struct ProfScope {
  const lb_plan *p;
  int kernel;
  int launches;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(const lb_plan *p_, bool on, int k, hipStream_t s, int64_t work = 0, int n = 1)
      : p(p_), kernel(k), launches(n), st(s) {
    if (!on) return;
    std::lock_guard<std::mutex> g(p->mu);
    p->prof_work[k] += work;
    a = prof_event(p);
    if (a) (void)hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!a) return;
    std::lock_guard<std::mutex> g(p->mu);
    hipEvent_t b = prof_event(p);
    if (!b) return;
    (void)hipEventRecord(b, st);
    p->prof_pending.push_back({kernel, launches, a, b});
    if (p->prof_pending.size() >= 2048) prof_drain(p);
  }
  // both called with p->mu held
  static hipEvent_t prof_event(const lb_plan *p);
  static void prof_drain(const lb_plan *p);
};

// Waits for every profiled launch, accumulates its time and recycles its events.
void prof_resolve(const lb_plan *p);
void prof_add_work(const lb_plan *p, int kernel, int64_t work);

// Thread-local error message helpers.
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define LBX_HIP(call)                                   \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return lbx::hip_fail(_e, #call); \
  } while (0)

// Status bits that kernels raise in the status word of a call's workspace.
constexpr int LB_STATUS_THETA = 1;      // a stage-solve contraction bound >= 0.5
constexpr int LB_STATUS_NOCONV = 2;     // a stage solve hit the sweep cap
constexpr int LB_STATUS_NONFINITE = 4;  // an objective is not finite
constexpr int LB_STATUS_RETRY = 8;      // a streamed step needed more sweeps than were launched

// Slots per system and step parity for the grid-wide maxima of sweep 0.
constexpr int LB_STEP_SLOTS = 64;

// Arguments of one sweep launch (kernels_step.hip), passed by value.
struct StepArgs {
  const SysDev *sysv;
  const double *Etab;
  const uint64_t *desc;
  const double2 *ctab;      // control table (rad/ns) of every system
  const double2 *ttab;      // [nsys][NT] (theta, theta / (1 - theta))
  int64_t cshift, tshift;   // the tables hold entries from these indices on (0: all)
  int NT, nsys;
  int j;                    // step index: controls at t_j + dt/2
  int n, m, H;              // steps already taken in this pass; history used; ring length
  int par;                  // parity of the step (selects its maxima slots)
  int L;                    // sweeps launched for this step
  int apriori;              // 1: every launched sweep runs (counts known on the host)
  const double2 *q;         // q^j (adjoint: qh^{j+1})
  double2 *out;             // q^{j+1} (adjoint: qh^j)
  const double2 *zstart;    // first iterate q + delta0, or NULL (delta0 = 0)
  double2 *z0, *z1;         // sweep iterates
  double2 *znext;           // first iterate of the next step, or NULL
  double2 *zh;              // stage vector q + delta (adjoint), or NULL
  double2 *ring;            // H increment buffers, ring_stride entries apart
  int64_t ring_stride;
  unsigned long long *slots;  // [2][nsys][2][LB_STEP_SLOTS] maxima (bits of doubles)
  int32_t *kstep;           // [2][nsys] sweeps of the step (by parity)
  int32_t *kout;            // sweeps taken are added to [nsys][NT], or NULL
  int32_t *status;          // status word (LB_STATUS_*)
  double tol;
  int kcap;                 // most sweeps after the first
  int sys, B;               // tiled: the system and its states
  int64_t units;            // tiled: units of the launch (set by the launcher)
  const StreamSeg *segs;    // generic: segments
  int nseg;
  int64_t nblk;             // generic: units (STREAM_BLOCK entries each)
  // two-pass sweep (tile_k >= LB_SPLIT_BASE): pass A takes subsystems
  // split_q..Q-1 (products of levels split_na), pass B the others
  int split_q;
  int64_t split_na, split_sp;
  // block-tiled adjoint step: when gpart is set, its last sweep also forms
  // the step's gradient integrands from the forward states gq0 = q^j and
  // gq1 = q^{j+1}, one row of 2 QMAX partial sums per unit
  const double2 *gq0, *gq1;
  double *gpart;
};

// Whether the last sweep of a block-tiled adjoint step of this system and
// block shape can form the step's gradient integrands (StepArgs::gpart).
bool tile_grad_fusable(const lb_plan *p, int sys, int tile_k);

// Block shapes at or above this code select the two-pass sweep and apply of
// one system, split after (code - LB_SPLIT_BASE) least significant subsystems.
constexpr int LB_SPLIT_BASE = 100;
struct SplitGeo {
  int q0;       // pass A: subsystems q0..Q-1 (the least significant digits)
  int64_t NA;   // product of their levels
  int64_t SP;   // spectator columns of a pass-B set (lowest column digits; divides NA)
};
// The split of system sys for code k (false when k is not a valid split).
bool split_geo(const lb_plan *p, int sys, int k, SplitGeo *g);
// lindblad_apply of B states with the two-pass kernels; y holds the partial
// sum between the passes.
int launch_split_apply(const lb_plan *p, int sys, int B, bool adj, double t, const double *alpha,
                       const double2 *x, double2 *y, const SplitGeo &g, hipStream_t st);

// A copy of the plan's options (taken when a call starts).
lbx_opts plan_options(const lb_plan *p);
// Error code of LB_STATUS_* bits (LB_OK when none is set).
int status_bits_code(int32_t bits);
// Waits for `st` and returns the status of the last imr_step_noalloc call
// on the current device.
int noalloc_status(const lb_plan *p, hipStream_t st);

// Sweep kk of one step: the block-tiled kernel of system tile_sys in block
// shape tile_k (10 KR + KC) when tile_sys >= 0, else the generic one.
int launch_sweep(const lb_plan *p, StepArgs &A, int kk, bool adj, int tile_sys, int tile_k, hipStream_t st);
// Clears the maxima slots of both parities of nsys systems.
int launch_slots_clear(unsigned long long *slots, int nsys, hipStream_t st);

// ---- Krylov stage solve of the streamed batch (steps with theta >= 0.5) ----
constexpr int KRY_M = 10;             // restart length of GMRES
constexpr int KRY_MAXV = KRY_M + 1;   // Krylov vectors of one cycle
constexpr int KRY_VECTORS = KRY_M + 3;  // basis, solution and one work vector
struct KryArgs {
  const SysDev *sysv;
  const double *Etab;
  const uint64_t *desc;
  const double2 *ctab;  // controls at the systems' offsets
  const StreamSeg *segs;
  int nseg;
  int64_t nblk;
  int j;  // step
};
struct KryCoef {
  int n;
  double2 c[KRY_MAXV];
};
// u = W x (W = (1 - h D)^{-1}, conjugated for the adjoint).
int launch_kry_weight(const KryArgs &A, bool adj, const double2 *x, double2 *u, hipStream_t st);
// y = u - h M u (M^+ for the adjoint), or q minus that when q is not NULL.
int launch_kry_apply(const KryArgs &A, bool adj, const double2 *u, const double2 *q, double2 *y, hipStream_t st);
// Device scratch of launch_kry_dots.
size_t kry_part_bytes();
// out[i] = <V_i, x> for i < n (V_i at V + i*stride), E entries.
int launch_kry_dots(const double2 *V, int64_t stride, int n, const double2 *x, int64_t E, double2 *part,
                    double2 *out, hipStream_t st);
// x = s x - sum_i c_i V_i.
int launch_kry_axpy(const double2 *V, int64_t stride, const KryCoef &c, double s, double2 *x, int64_t E,
                    hipStream_t st);
// z = W y, out = 2 z - q, zh = z (zh may be NULL).
int launch_kry_finish(const KryArgs &A, bool adj, const double2 *y, const double2 *q, double2 *out, double2 *zh,
                      hipStream_t st);

// ---- launchers (each returns LB_OK or an error code) ----

// Zeroes `bytes` (a multiple of 4) with a kernel.
int launch_fill_zero(void *ptr, size_t bytes, hipStream_t st);
int launch_fill_trial(double2 *ptr, int64_t n, hipStream_t st);

// Control table of systems s0..s0+nsys-1; entry (s, j, q) goes to
// ctab[ctab_off(s) - ctab_shift + j*Q + q].  ktab ([s][j][2] a-priori sweep
// counts) and ttab ([s][j] = (theta, theta / (1 - theta))) may be NULL.
int launch_control_table(const lb_plan *p, int s0, int nsys, const double *alpha, double2 *ctab,
                         int64_t ctab_shift, int32_t *ktab, double2 *ttab, double tol, hipStream_t st);

// y = M(t) x or M(t)^+ x; tile_opt / ki_opt are LB_OPT_TILE / LB_OPT_TILE_KI.
int launch_apply(const lb_plan *p, int sys, double t, const double *alpha, const double2 *x,
                 double2 *y, int B, bool adj, int tile_opt, int ki_opt, hipStream_t st);

// Gradient integrands of one step from the adjoint stage vector zh and the
// forward states q0 = q^j, q1 = q^{j+1} (per-block partial rows).
int launch_stream_grad(const lb_plan *p, const StreamSeg *d_segs, int nseg, int64_t nblk,
                       const double2 *zh, const double2 *q0, const double2 *q1, double *gpart,
                       hipStream_t st);

// Two-pass fixed-order sum of the stream_grad partials of nsteps steps into
// gstep: slot z (partial rows at gpart + z slot_stride) holds step jtop - z;
// gfin is scratch of nsteps stream_grad_fin_doubles(nseg) doubles.
size_t stream_grad_fin_doubles(int nseg);
int launch_stream_grad_finalize(const lb_plan *p, const StreamSeg *d_segs, int nseg, int jtop,
                                int nsteps, const double *gpart, int64_t slot_stride, double *gfin,
                                double *gstep, int64_t rows, hipStream_t st);

// Generic LDS-resident kernels: a-priori sweep counts from ktab; sweeps
// (nullable) receives each item's total; status collects LB_STATUS_* bits.
int launch_lds_forward(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                       const double2 *ctab, const int32_t *ktab, const double2 *rho0,
                       double2 *rhoT, double2 *states, int64_t *sweeps, int32_t *status, hipStream_t st);

// ptab (nullable): the running-penalty table of launch_penalty_table; the
// adjoint then adds the source term of every step j >= 1.
int launch_lds_adjoint(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                       int kind, const double2 *ctab, const int32_t *ktab, const double2 *rhotar,
                       const double2 *states, const double *ptab, double *gpart, int64_t *sweeps,
                       int32_t *status, hipStream_t st);

int launch_lds_grad_reduce(const lb_plan *p, const int32_t *d_item_range, int nsys_lds,
                           const int32_t *d_sys_ids, const LdsItem *d_items, const double *gpart,
                           double *gstep, hipStream_t st);

// G (nullable) and J (nullable) per system / state; status (nullable)
// receives LB_STATUS_NONFINITE when a G is not finite.  pen (nullable,
// DEVICE [nsys]) is added to G: the running penalty.
int launch_objective(const lb_plan *p, int kind, const double2 *rhoT, const double2 *rhotar,
                     const double *beta, const int32_t *d_state_sys, const int64_t *d_state_off,
                     const int32_t *d_sys_state0, int nstates, double gamma2, const double *alpha,
                     const double *pen, double *partial, double *J, double *G, int32_t *status,
                     hipStream_t st);

// Running penalty (Sec. III eq. optimproblem, gamma1 term), integrated by
// the left rectangle rule on the time grid.
//   ptab[s][j] = gamma1 dt_s beta_s(j dt_s), beta(t) = exp(-((t - T)/a)^2) / a,
// for every system s and step j < NT.  Per merit functional the value of
// one entry is v = |q - t|^2 / 2 (J_Frob) or Re conj(t) q (J_Tr, J_Nm), and
//   pen_s = (1/M_s) sum_i sum_j ptab[s][j] J(q_i^j),  J_Tr = 1 - sum v.
constexpr int PEN_PARTS = 32;  // partial sums per LDS-resident state
int launch_penalty_table(const lb_plan *p, double gamma1, double a, double *ptab, hipStream_t st);
// acc[b] += ptab[sys][j] * (sum of v over the entries of stream block b), q
// holding q^j of the streamed states (compact layout).
int launch_penalty_accum(const lb_plan *p, int kind, const StreamSeg *d_segs, int nseg, int64_t nblk, int j,
                         const double2 *q, const double2 *rhotar, const double *ptab, double *acc,
                         hipStream_t st);
// part[item][c] = sum over the steps of chunk c of ptab[sys][j] * (sum of v
// over q^j), from the state history of each LDS-resident item.
int launch_penalty_lds(const lb_plan *p, int kind, const LdsItem *d_items, int nitems, const double2 *hist,
                       const double2 *rhotar, const double *ptab, double *part, hipStream_t st);
// pen[s] from the accumulators; rng[s] = {first stream block, blocks, first
// LDS item, items} of system s.
int launch_penalty_final(const lb_plan *p, int kind, const int64_t *d_rng, const double *acc,
                         const double *part, const double *ptab, const int32_t *d_sys_state0, double *pen,
                         hipStream_t st);
// Adjoint source of step j on the streamed states:
//   qh += ptab[sys][j] gscale[sys] / M (dJ/d(conj q) at q = q^j).
int launch_penalty_source(const lb_plan *p, int kind, const StreamSeg *d_segs, int nseg, int64_t nblk, int j,
                          const double2 *q, const double2 *rhotar, const double *ptab, const double *gscale,
                          double2 *qh, hipStream_t st);

// Terminal condition of the streamed states; gscale (nullable, DEVICE
// [nsys]) weights each system's objective.
int launch_terminal(const lb_plan *p, int kind, const StreamSeg *d_segs, int nseg, int64_t nblk,
                    const double2 *rhoT, const double2 *rhotar, const double *beta,
                    const int32_t *d_seg_state0, const double *gscale, double2 *qh, hipStream_t st);

int launch_grad_contract(const lb_plan *p, const double *gstep, const double *alpha,
                         double gamma2, const double *gscale, double *grad, hipStream_t st);

// LDS path: block size and entries per thread for a state of n2 entries;
// returns false when the state does not fit the LDS-resident kernels.
bool lds_shape(int64_t n2, int *block, int *ept);

// Block-tiled kernels (kernels_tile.hip).  tile_ki returns the block shape
// 10*KR + KC of an eligible system (equal-level subsystems with an
// instantiated shape; ki_opt selects among them, 0 the default) or 0.
int tile_ki(const lb_plan *p, int sys, int ki_opt);
// Multi-pass apply kernels: number of passes of the system's plan, 0 if not
// eligible; launch_split runs them (mode 0: apply).
int split_kl(const lb_plan *p, int sys);
int launch_split(const lb_plan *p, int sys, int B, int mode, bool adj, const double *alpha, double t,
                 const double2 *ctab, int j, const double2 *zin, const double2 *qin, double2 *out,
                 double2 *zout, hipStream_t st);
// lindblad_apply of an eligible system (multi-pass when tile_opt is 2 and the
// system has a pass plan).
int launch_tile_apply(const lb_plan *p, int sys, int B, bool adj, const double *alpha, double t,
                      const double2 *x, double2 *y, int tile_opt, int ki_opt, hipStream_t st);
// Block-tiled gradient integrands of one step in block shape k (partial rows:
// tile_grad_rows).
int64_t tile_grad_rows(const lb_plan *p, int sys, int B, int k);
int launch_tile_grad(const lb_plan *p, int sys, int B, int k, const double2 *zh, const double2 *q0,
                     const double2 *q1, double *gpart, int64_t *rows, hipStream_t st);

// Specialised LDS-resident kernels (kernels_lds_fast.hip) for Q subsystems.
bool lds_fast_ok(int block, int ept, int Q);
// They pick the number of sweeps of every step a posteriori (see
// extra_sweeps) and, when `sweeps` is not NULL, write each item's total.
int launch_lds_forward_fast(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                            int Q, const double2 *ctab, const double2 *ttab, double tol, const double2 *rho0,
                            double2 *rhoT, double2 *states, int64_t *sweeps, int32_t *status, hipStream_t st);
// The adjoint stores each step's converged stage vector in zhist (laid out
// like the state history) and a second launch forms the gradient integrands.
int launch_lds_adjoint_fast(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                            int Q, int kind, const double2 *ctab, const double2 *ttab, double tol,
                            const double2 *rhotar, const double2 *states, double2 *zhist,
                            double *gpart, int64_t *sweeps, int32_t *status, hipStream_t st);

}  // namespace lbx

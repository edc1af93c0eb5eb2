// Host-side plan structure and kernel launchers shared by the library's
// translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lbx.h"
#include "lbx_device.hpp"

struct lbx_prof_pending {
  int kernel;
  int launches;  // kernel launches bracketed by the two events
  hipEvent_t start, stop;
};

struct lb_plan {
  std::vector<lbx::SysDev> sys;   // host copy of the per-system constants
  lbx::SysDev *d_sys = nullptr;   // device copy
  double *d_E = nullptr;          // energies of H_sys per basis index [rad/ns]
  uint64_t *d_desc = nullptr;     // packed subsystem digits per basis index
  double *d_carrier = nullptr;    // carriers [GHz], per system [Q][Nf]
  int32_t NT = 0;                 // common number of steps
  int64_t ctab_total = 0;         // sum over systems of NT*Q
  int path = 0;                   // LB_OPT_PATH
  int tile = 1;                   // LB_OPT_TILE
  int tile_ki = 0;                // LB_OPT_TILE_KI (0: default block)
  int graph_steps = 0;            // LB_OPT_GRAPH (0: launch directly)
  mutable bool capturing = false; // inside a stream capture: no profiling events
  double tol = 1.1102230246251565e-16;  // LB_OPT_SOLVE_TOL (2^-53)
  int device = 0;
  // LB_OPT_PROFILE: per-kernel-family launch counts and durations.
  bool profile = false;
  mutable int64_t prof_n[LB_KERNEL_COUNT] = {};
  mutable double prof_ms[LB_KERNEL_COUNT] = {};
  mutable int64_t prof_work[LB_KERNEL_COUNT] = {};  // entries x sweeps (x steps for STREAM_GRAD)
  mutable std::vector<lbx_prof_pending> prof_pending;
  mutable std::vector<hipEvent_t> ev_pool;  // recycled profiling events
  mutable int64_t *d_sweeps = nullptr;  // per-item sweep totals of the LDS kernels (profiling)
  mutable size_t sweeps_cap = 0;
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
  ProfScope(const lb_plan *p_, int k, hipStream_t s, int64_t work = 0, int n = 1)
      : p(p_), kernel(k), launches(n), st(s) {
    if (!p->profile || p->capturing) return;
    p->prof_work[k] += work;
    a = prof_event(p);
    if (a) (void)hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = prof_event(p);
    if (!b) return;
    (void)hipEventRecord(b, st);
    p->prof_pending.push_back({kernel, launches, a, b});
    if (p->prof_pending.size() >= 2048) prof_drain(p);
  }
  static hipEvent_t prof_event(const lb_plan *p);
  static void prof_drain(const lb_plan *p);
};

// Waits for every profiled launch, accumulates its time and recycles its events.
void prof_resolve(const lb_plan *p);

// Thread-local error message helpers.
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define LBX_HIP(call)                                   \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return lbx::hip_fail(_e, #call); \
  } while (0)

// ---- launchers (each returns LB_OK or an error code) ----

// Control table of systems s0..s0+nsys-1; entry (s, j, q) goes to
// ctab[ctab_off(s) - ctab_shift + j*Q + q].  ktab ([s][j][2] a-priori sweep
// counts) and ttab ([s][j] = (theta, theta / (1 - theta))) may be NULL.
int launch_control_table(const lb_plan *p, int s0, int nsys, const double *alpha, double2 *ctab,
                         int64_t ctab_shift, int32_t *ktab, double2 *ttab, hipStream_t st);

int launch_apply(const lb_plan *p, int sys, double t, const double *alpha, const double2 *x,
                 double2 *y, int B, bool adj, hipStream_t st);

// Sweep kk of the stage solve of every streamed segment at step j.  Each
// segment runs its own system's count K = ktab[sys][j][1] (kfix > 0: K =
// kfix for all) and skips sweeps kk >= K; sweep kk reads q (kk = 0), z0 (kk
// odd) or z1 (kk even) and writes z1 / z0, or `out` on its last sweep, which
// with want_zh also writes the converged stage vector z = q + delta into
// the z buffer it does not read.
int launch_sweep(const lb_plan *p, const StreamSeg *d_segs, int nseg, int64_t nblk, int j, int kk,
                 int kfix, bool adj, const double2 *ctab, const int32_t *ktab, const double2 *qin,
                 double2 *z0, double2 *z1, double2 *out, bool want_zh, hipStream_t st);

// Gradient integrands of step j; each segment's stage vector is in z0 or z1
// as its last adjoint sweep (ktab) left it.
int launch_stream_grad(const lb_plan *p, const StreamSeg *d_segs, int nseg, int64_t nblk,
                       const double2 *z0, const double2 *z1, const int32_t *ktab, int j,
                       const double2 *q0, const double2 *q1, double *gpart, hipStream_t st);

// Two-pass fixed-order sum of the stream_grad partials of nsteps steps into
// gstep: slot z (partial rows at gpart + z slot_stride) holds step jtop - z;
// gfin is scratch of nsteps stream_grad_fin_doubles(nseg) doubles.
size_t stream_grad_fin_doubles(int nseg);
int launch_stream_grad_finalize(const lb_plan *p, const StreamSeg *d_segs, int nseg, int jtop,
                                int nsteps, const double *gpart, int64_t slot_stride, double *gfin,
                                double *gstep, int64_t rows, hipStream_t st);

int launch_lds_forward(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                       const double2 *ctab, const int32_t *ktab, const double2 *rho0,
                       double2 *rhoT, double2 *states, hipStream_t st);

int launch_lds_adjoint(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                       int kind, const double2 *ctab, const int32_t *ktab, const double2 *rhotar,
                       const double2 *states, double *gpart, hipStream_t st);

int launch_lds_grad_reduce(const lb_plan *p, const int32_t *d_item_range, int nsys_lds,
                           const int32_t *d_sys_ids, const LdsItem *d_items, const double *gpart,
                           double *gstep, hipStream_t st);

int launch_objective(const lb_plan *p, int kind, const double2 *rhoT, const double2 *rhotar,
                     const double *beta, const int32_t *d_state_sys, const int64_t *d_state_off,
                     const int32_t *d_sys_state0, int nstates, double gamma2, const double *alpha,
                     double *partial, double *J, double *G, hipStream_t st);

int launch_terminal(const lb_plan *p, int kind, const StreamSeg *d_segs, int nseg, int64_t nblk,
                    const double2 *rhoT, const double2 *rhotar, const double *beta,
                    const int32_t *d_seg_state0, double2 *qh, hipStream_t st);

int launch_grad_contract(const lb_plan *p, const double *gstep, const double *alpha,
                         double gamma2, double *grad, hipStream_t st);

// LDS path: block size and entries per thread for a state of n2 entries;
// returns false when the state does not fit the LDS-resident kernels.
bool lds_shape(int64_t n2, int *block, int *ept);

// Block-tiled streaming kernels (kernels_tile.hip).  tile_nl returns the
// common level count of an eligible system (equal-level subsystems whose
// (NL, Q) has an instantiated block shape or, with LB_OPT_TILE 2, a pass
// plan) or 0.
int tile_nl(const lb_plan *p, int sys);
int tile_ki(const lb_plan *p, int sys);  // block shape 10*KR + KC, 0 if not eligible
// mode 0: y = M x (alpha, t); mode 1: sweep (q + delta); mode 2: last sweep (q + 2 delta),
// with the controls of step j from ctab.
// Two-pass split kernels (kernels_tile.hip): number of low subsystems of the
// split of system sys, 0 if not eligible; launch_split runs both passes.
// launch_tile uses them when LB_OPT_TILE is 2 and the system is eligible.
int split_kl(const lb_plan *p, int sys);
int launch_split(const lb_plan *p, int sys, int B, int mode, bool adj, const double *alpha, double t,
                 const double2 *ctab, int j, const double2 *zin, const double2 *qin, double2 *out,
                 double2 *zout, hipStream_t st);
int launch_tile(const lb_plan *p, int sys, int B, int mode, bool adj, const double *alpha, double t,
                const double2 *ctab, int j, const double2 *zin, const double2 *qin, double2 *out,
                double2 *zout, hipStream_t st);
// Block-tiled gradient integrands of one step (partial rows: tile_grad_rows).
int64_t tile_grad_rows(const lb_plan *p, int sys, int B);
int launch_tile_grad(const lb_plan *p, int sys, int B, const double2 *zh, const double2 *q0,
                     const double2 *q1, double *gpart, int64_t *rows, hipStream_t st);

// Specialised LDS-resident kernels (kernels_lds_fast.hip) for Q subsystems.
bool lds_fast_ok(int block, int ept, int Q);
// They pick the number of sweeps of every step a posteriori (see
// extra_sweeps) and, when `sweeps` is not NULL, write each item's total.
int launch_lds_forward_fast(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                            int Q, const double2 *ctab, const double2 *ttab, const double2 *rho0,
                            double2 *rhoT, double2 *states, int64_t *sweeps, hipStream_t st);
// The adjoint stores each step's converged stage vector in zhist (laid out
// like the state history) and a second launch forms the gradient integrands.
int launch_lds_adjoint_fast(const lb_plan *p, const LdsItem *d_items, int nitems, int block, int ept,
                            int Q, int kind, const double2 *ctab, const double2 *ttab,
                            const double2 *rhotar, const double2 *states, double2 *zhist,
                            double *gpart, int64_t *sweeps, hipStream_t st);

}  // namespace lbx

// imr_step_noalloc: one implicit-midpoint step (App. A eqs. IMR and
// linsystem_primal; App. B eq. linsystem_adjoint) like imr_step, for callers
// that cannot allocate device memory (graph capture, allocation-free serving
// loops).  Its scratch memory (status word, the step's controls, the maxima
// slots and counts, the segment table and the two sweep iterates) is a
// file-scope device array of LB_NOALLOC_SCRATCH_BYTES on every device the
// library runs on; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.  The array keeps the
// last call's contents; calls that overlap on one device race on it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <map>
#include <mutex>
#include <string>

#include "lbx_host.hpp"
#include "tile_unit.hpp"

namespace lbx {

static_assert(LB_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
__device__ __align__(256) unsigned char scratch[LB_NOALLOC_SCRATCH_BYTES];

namespace {

// Layout of the scratch array: a table region, then the two iterates.
constexpr size_t NA_STATUS = 0;                           // int32
constexpr size_t NA_CTAB = 256;                           // QMAX complex controls of the step
constexpr size_t NA_TTAB = NA_CTAB + 256;                 // (theta, theta / (1 - theta))
constexpr size_t NA_KTAB = NA_TTAB + 256;                 // a-priori counts (LDS start, q start)
constexpr size_t NA_SEG = NA_KTAB + 256;                  // one StreamSeg
constexpr size_t NA_KSTEP = NA_SEG + 256;                 // [2][nsys] counts
constexpr size_t NA_SLOTS = NA_KSTEP + 2 * LB_NOALLOC_MAX_SYSTEMS * 4;
constexpr size_t NA_TABLES = NA_SLOTS + (size_t)2 * LB_NOALLOC_MAX_SYSTEMS * 2 * LB_STEP_SLOTS * 8;
constexpr size_t NA_Z0 = ((NA_TABLES + (1u << 20) - 1) / (1u << 20)) * (1u << 20);
static_assert(NA_Z0 + 2 * (size_t)LB_NOALLOC_MAX_ENTRIES * 16 <= LB_NOALLOC_SCRATCH_BYTES, "scratch layout");

std::mutex g_na_mu;
std::map<int, char *> g_na_ptr;  // scratch address per device

// Address of the scratch array on the current device (looked up once per device).
int scratch_ptr(char **out) {
  int dev = 0;
  LBX_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_na_mu);
  auto it = g_na_ptr.find(dev);
  if (it != g_na_ptr.end()) {
    *out = it->second;
    return LB_OK;
  }
  void *ptr = nullptr;
  LBX_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  g_na_ptr[dev] = (char *)ptr;
  *out = (char *)ptr;
  return LB_OK;
}

// Controls of step j of system sys (rad/ns) from the system's own parameters
// `alpha` (nalpha of that system), the contraction bound theta and
// the a-priori counts (control_table_kernel for one step), the segment of the
// states and zeroed status word, slots and counts.  One workgroup.
__global__ __launch_bounds__(256) void noalloc_setup_kernel(const SysDev *__restrict__ sysv, int sys, int nsys,
                                                            int j, const double *__restrict__ alpha,
                                                            const double *__restrict__ carrier, double tol,
                                                            StreamSeg seg, char *__restrict__ w) {
  const SysDev &S = sysv[sys];
  const int tid = threadIdx.x;
  unsigned long long *slots = (unsigned long long *)(w + NA_SLOTS);
  for (int k = tid; k < 2 * nsys * 2 * LB_STEP_SLOTS; k += 256) slots[k] = 0ull;
  int32_t *kstep = (int32_t *)(w + NA_KSTEP);
  for (int k = tid; k < 2 * nsys; k += 256) kstep[k] = 0;
  if (tid != 0) return;
  *(int32_t *)(w + NA_STATUS) = 0;
  *(StreamSeg *)(w + NA_SEG) = seg;
  double2 *ctab = (double2 *)(w + NA_CTAB);
  const double t = ((double)j + 0.5) * S.dt;
  double theta = S.theta_jump;
  for (int q = 0; q < S.Q; ++q) {
    const double2 d = control_value(S, alpha, carrier + S.carrier_off, q, t);
    ctab[q] = d;
    theta += S.h * 2.0 * hypot(d.x, d.y) * S.csum[q];
  }
  *(double2 *)(w + NA_TTAB) = make_double2(theta, theta < 1.0 ? theta / (1.0 - theta) : 0.0);
  int kst = -1;
  if (theta <= 0.0) {
    kst = 1;
  } else if (theta < 0.5) {
    const double e0 = S.hDmax + theta;
    kst = e0 <= tol ? 1 : (int)ceil((log(tol) - log(e0)) / log(theta));
    kst = kst < 1 ? 1 : kst;
  }
  ((int32_t *)(w + NA_KTAB))[1] = kst;
}

// kst > 0: repeat the step with that a-priori count (every launched sweep runs).
int launch_noalloc(const lb_plan *p, const lbx_opts &o, int sys, int j, const double *alpha, const double2 *q_in,
                   double2 *q_out, int B, bool adj, int kst, char *w, hipStream_t st) {
  const SysDev &S = p->sys[sys];
  StreamSeg seg{};
  seg.sys = sys;
  seg.nstates = B;
  seg.off = 0;
  seg.boff = 0;
  seg.count = (int64_t)B * S.N2;
  seg.blk0 = 0;
  hipLaunchKernelGGL(noalloc_setup_kernel, dim3(1), dim3(256), 0, st, p->d_sys, sys, (int)p->sys.size(), j, alpha,
                     p->d_carrier, o.tol, seg, w);
  LBX_HIP(hipGetLastError());
  const int tk = o.tile ? tile_ki(p, sys, o.tile_ki) : 0;
  StepArgs A{};
  A.sysv = p->d_sys;
  A.Etab = p->d_E;
  A.desc = p->d_desc;
  A.ctab = (const double2 *)(w + NA_CTAB);
  A.cshift = S.ctab_off + (int64_t)j * S.Q;
  A.ttab = (const double2 *)(w + NA_TTAB);
  A.tshift = (int64_t)sys * p->NT + j;
  A.NT = p->NT;
  A.nsys = (int)p->sys.size();
  A.j = j;
  A.q = q_in;
  A.out = q_out;
  A.z0 = (double2 *)(w + NA_Z0);
  A.z1 = A.z0 + LB_NOALLOC_MAX_ENTRIES;
  A.slots = (unsigned long long *)(w + NA_SLOTS);
  A.kstep = (int32_t *)(w + NA_KSTEP);
  A.status = (int32_t *)(w + NA_STATUS);
  A.tol = o.tol;
  A.kcap = 64;
  A.B = B;
  A.segs = (const StreamSeg *)(w + NA_SEG);
  A.nseg = 1;
  A.nblk = (seg.count + STREAM_BLOCK - 1) / STREAM_BLOCK;
  if (kst > 0) {
    A.apriori = 1;
    A.L = kst > 2 ? kst : 2;
  } else {
    A.L = o.sweeps > 0 ? o.sweeps : 12;
  }
  for (int kk = 0; kk < A.L; ++kk)
    if (int rc = launch_sweep(p, A, kk, adj, tk ? sys : -1, tk, st)) return rc;
  return LB_OK;
}

}  // namespace

int noalloc_status(const lb_plan *p, hipStream_t st) {
  (void)p;
  char *w = nullptr;
  if (int rc = scratch_ptr(&w)) return rc;
  int32_t bits = 0;
  LBX_HIP(hipMemcpyAsync(&bits, w + NA_STATUS, sizeof(bits), hipMemcpyDeviceToHost, st));
  LBX_HIP(hipStreamSynchronize(st));
  return status_bits_code(bits);
}

}  // namespace lbx

using namespace lbx;

extern "C" int imr_step_noalloc(const lb_plan *p, int32_t sys, int32_t j, const double *alpha, const void *q_in,
                                void *q_out, int32_t B, int32_t adjoint, void *stream) {
  if (!p) return fail(LB_EINVAL, "plan is NULL");
  const int nsys = (int)p->sys.size();
  if (sys < 0 || sys >= nsys) return fail(LB_EINVAL, "sys out of range");
  if (j < 0 || j >= p->NT) return fail(LB_EINVAL, "step index out of range");
  if (B < 0) return fail(LB_EINVAL, "B must be >= 0");
  if (B == 0) return LB_OK;
  if (!alpha || !q_in || !q_out) return fail(LB_EINVAL, "NULL argument");
  const int64_t entries = (int64_t)B * p->sys[sys].N2;
  if (entries > LB_NOALLOC_MAX_ENTRIES)
    return fail(LB_EINVAL, "imr_step_noalloc: B*N^2 = " + std::to_string(entries) + " exceeds the scratch limit of " +
                               std::to_string((long long)LB_NOALLOC_MAX_ENTRIES) + " entries");
  if (nsys > LB_NOALLOC_MAX_SYSTEMS)
    return fail(LB_EINVAL, "imr_step_noalloc: the plan has more than " + std::to_string(LB_NOALLOC_MAX_SYSTEMS) +
                               " systems");
  {
    const uintptr_t a = (uintptr_t)q_in, c = (uintptr_t)q_out;
    const size_t bytes = (size_t)entries * sizeof(double2);
    if (a < c + bytes && c < a + bytes) return fail(LB_EINVAL, "q_in and q_out overlap");
  }
  const lbx_opts o = plan_options(p);
  hipStream_t st = (hipStream_t)stream;
  char *w = nullptr;
  if (int rc = scratch_ptr(&w)) return rc;
  if (int rc = launch_noalloc(p, o, sys, j, alpha, (const double2 *)q_in, (double2 *)q_out, B, adjoint != 0, 0, w,
                              st))
    return rc;
  if (!o.sync) return LB_OK;
  int32_t bits = 0;
  LBX_HIP(hipMemcpyAsync(&bits, w + NA_STATUS, sizeof(bits), hipMemcpyDeviceToHost, st));
  LBX_HIP(hipStreamSynchronize(st));
  if ((bits & LB_STATUS_RETRY) && !(bits & (LB_STATUS_THETA | LB_STATUS_NONFINITE))) {
    // repeat with the a-priori count of the step (read from the scratch)
    int32_t k[2] = {0, 0};
    LBX_HIP(hipMemcpyAsync(k, w + NA_KTAB, sizeof(k), hipMemcpyDeviceToHost, st));
    LBX_HIP(hipStreamSynchronize(st));
    if (k[1] < 1) return fail(LB_EUNSUPPORTED, "the stage-solve contraction bound of this step is >= 0.5");
    if (int rc = launch_noalloc(p, o, sys, j, alpha, (const double2 *)q_in, (double2 *)q_out, B, adjoint != 0, k[1],
                                w, st))
      return rc;
    LBX_HIP(hipMemcpyAsync(&bits, w + NA_STATUS, sizeof(bits), hipMemcpyDeviceToHost, st));
    LBX_HIP(hipStreamSynchronize(st));
  }
  return status_bits_code(bits);
}

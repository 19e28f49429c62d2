// C ABI of the pseudo-spectral DNS library (declarations and contracts in include/psdns.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace psdns {
Ops ops_n8(int);
Ops ops_n16(int);
Ops ops_n32(int);
Ops ops_n64(int);
Ops ops_n128(int);
Ops ops_n256(int);
Ops ops_n512(int);
Ops ops_n1024(int);
Ops ops_general(int);
int general_x_lines(int n, int precision);
}  // namespace psdns

using namespace psdns;

namespace {

thread_local std::string g_err = "no error";

psdns_status fail(psdns_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

psdns_status hip_fail(hipError_t e, const char* what) {
  return fail(PSDNS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                           \
  do {                                          \
    hipError_t e_ = (call);                     \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// largest retained |k_i|: (N-1)/3 for the 2/3 rule, else the largest k with 9 k^2 < 2 N^2
int kmax_of(int n, int dealias) {
  if (dealias != PSDNS_DEALIAS_PHASE_SPHERE) return (n - 1) / 3;
  int k = 0;
  while (9LL * (k + 1) * (k + 1) < 2LL * n * n) ++k;
  return k;
}

// whether the plan's steps run on the general kernels (mixed radix)
bool general_plan(const psdns_plan_params* p) { return !is_pow2(p->n); }

bool valid_params(const psdns_plan_params* p, std::string* why) {
  if (!p) {
    *why = "params is NULL";
    return false;
  }
  const int n = p->n;
  int rest = n;
  for (int f : {2, 3, 5, 7, 11, 13})
    while (rest % f == 0) rest /= f;
  if (n < 8 || n > 1024 || n % 2 != 0 || rest != 1) {
    *why = "n must be even, in [8, 1024], with prime factors among 2, 3, 5, 7, 11, 13; got " + std::to_string(n);
    return false;
  }
  if (p->dealias != PSDNS_DEALIAS_TWO_THIRDS && p->dealias != PSDNS_DEALIAS_PHASE_SPHERE) {
    *why = "dealias must be PSDNS_DEALIAS_TWO_THIRDS or PSDNS_DEALIAS_PHASE_SPHERE, got " + std::to_string(p->dealias);
    return false;
  }
  if (p->n_scalars < 0 || p->n_scalars > PSDNS_MAX_SCALARS) {
    *why = "n_scalars must be in [0, " + std::to_string(PSDNS_MAX_SCALARS) + "], got " + std::to_string(p->n_scalars);
    return false;
  }
  if (p->precision != 32 && p->precision != 64) {
    *why = "precision must be 32 or 64, got " + std::to_string(p->precision);
    return false;
  }
  {
    // the column passes address one field (one z plane for the y-pass arrays) with
    // 32-bit byte offsets from a per-field buffer base
    const long long k = kmax_of(n, p->dealias), m = 2 * k + 1, px = (k + 1 + 15) / 16 * 16;
    const double field_bytes = (double)n * m * px * (p->precision == 32 ? 8 : 16);
    if (field_bytes >= 4294967296.0) {
      *why = "one transposed field would exceed 4 GiB";
      return false;
    }
  }
  if (p->batch < 1 || p->batch > 65535) {
    *why = "batch must be in [1, 65535], got " + std::to_string(p->batch);
    return false;
  }
  return true;
}

Ops ops_pow2(int n, int prec) {
  switch (n) {
    case 8: return ops_n8(prec);
    case 16: return ops_n16(prec);
    case 32: return ops_n32(prec);
    case 64: return ops_n64(prec);
    case 128: return ops_n128(prec);
    case 256: return ops_n256(prec);
    case 512: return ops_n512(prec);
    default: return ops_n1024(prec);
  }
}

// The step kernels of a plan: the tuned ones of its N, or the general ones.  A power-of-two
// plan with the phase-shift dealiasing steps on the tuned kernels (their phase-shift stage,
// one schedule) and takes its initial fields, statistics and state conversions from the
// general kernels, whose layouts are the same.
Ops ops_for(const psdns_plan_params* p) {
  const int n = p->n, prec = p->precision;
  if (!is_pow2(n)) return ops_general(prec);
  Ops t = ops_pow2(n, prec);
  if (p->dealias != PSDNS_DEALIAS_PHASE_SPHERE) return t;
  Ops o = ops_general(prec);
  o.nsched = 1;
  o.sched[0] = t.sched[0];
  o.sched[0].rhs_stage = t.rhs_phase;
  o.rhs_mixed = nullptr;
  return o;
}


// blocks per slot of the moments kernels (fixed, so their partial sums have a fixed order)
int moment_blocks(int n) {
  const long long lines = (long long)n * n;
  return (int)(lines < 1024 ? lines : 1024);
}

int shell_count(int K) { return (int)std::lround(std::sqrt(3.0) * K) + 1; }

// doubles per slot of the psdns_spectra record
int spectra_record(int ns, int S) { return ns * (1 + S) + 8 + 4 * S + 16 + 3 * S; }

struct Layout {
  Geom g;
  size_t csize;  // bytes per complex
  size_t off_dyn, off_fband, off_part, off_stat, off_ystage, off_acc, off_abuf, off_bbuf, off_akeep, ws_bytes,
      st_bytes;
  long long part_len, stat_len;
  int nbm, rec;
};

Layout make_layout(const psdns_plan_params* p) {
  Layout L{};
  Geom& g = L.g;
  g.N = p->n;
  g.K = kmax_of(p->n, p->dealias);
  g.sphere = p->dealias == PSDNS_DEALIAS_PHASE_SPHERE;
  g.M = 2 * g.K + 1;
  g.KX = g.K + 1;
  g.PX = (g.KX + 15) / 16 * 16;
  g.S = p->n_scalars;
  g.F = 3 + g.S;
  g.FA = 5 + 2 * g.S;
  g.FB = 6 + 3 * g.S;
  g.batch = p->batch;
  g.st_field = (long long)g.M * g.M * g.PX;
  g.a_field = (long long)g.N * g.M * g.PX;
  g.b_field = (long long)g.N * g.N * g.PX;
  // x-pass partial maxima: at most one per line whatever the schedule (the step sets
  // the count of the schedule in use)
  g.nblk_x = g.N * g.N;
  g.ns = shell_count(g.K);
  L.nbm = moment_blocks(g.N);
  L.rec = spectra_record(g.ns, g.S);
  L.csize = p->precision == 32 ? 8 : 16;
  const size_t B = (size_t)g.batch;
  const long long n_init = ((long long)g.M * g.M * g.KX + 255) / 256;
  const long long n_max = (long long)B * g.nblk_x;
  L.part_len = n_init > n_max ? n_init : n_max;
  size_t off = 0;
  L.off_dyn = off;
  off = align_up(off + B * sizeof(DynDev), 256);
  L.off_fband = off;
  off = align_up(off + B * (size_t)kStochCand * 12 * sizeof(double), 256);
  L.off_part = off;
  off = align_up(off + (size_t)L.part_len * sizeof(double), 256);
  L.off_stat = off;
  L.stat_len = (long long)B * g.ns * (2 + 3 * g.S) + 2LL * B * L.nbm * (3 * 6 + 1);
  off = align_up(off + (size_t)L.stat_len * sizeof(double), 256);
  L.off_ystage = off;
  off = align_up(off + B * g.F * (size_t)g.st_field * L.csize, 256);
  L.off_acc = off;
  off = align_up(off + B * g.F * (size_t)g.st_field * L.csize, 256);
  L.off_abuf = off;
  off = align_up(off + B * g.FA * (size_t)g.a_field * L.csize, 256);
  L.off_bbuf = off;
  off = align_up(off + B * g.FB * (size_t)g.b_field * L.csize, 256);
  L.off_akeep = off;
  if (g.sphere) off = align_up(off + B * g.F * (size_t)g.a_field * L.csize, 256);
  L.ws_bytes = off;
  L.st_bytes = B * g.F * (size_t)g.st_field * L.csize;
  return L;
}

const char* kKernelNames[KID_COUNT] = {"forcing_amplitude", "z_inverse",        "y_inverse",
                                       "x_pass",            "step_dt",          "y_forward",
                                       "z_forward_update",  "aux",              "z_forward_update_inverse",
                                       "step"};

// Event pairs around launches; records may nest (a step around its kernels), so end()
// closes the innermost open record of its kind.
struct EventTimer : Timer {
  struct Rec {
    int kid;
    hipEvent_t a, b;
    bool closed;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipError_t err = hipSuccess;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) err = r;
    return e;
  }
  void begin(int kid, hipStream_t s) override {
    Rec r{kid, get(), get(), false};
    if (r.a) {
      const hipError_t e = hipEventRecord(r.a, s);
      if (e != hipSuccess) err = e;
    }
    recs.push_back(r);
  }
  void end(int kid, hipStream_t s) override {
    for (auto it = recs.rbegin(); it != recs.rend(); ++it)
      if (it->kid == kid && !it->closed) {
        if (it->b) {
          const hipError_t e = hipEventRecord(it->b, s);
          if (e != hipSuccess) err = e;
        }
        it->closed = true;
        return;
      }
  }
  ~EventTimer() override {
    for (auto& r : recs) {
      if (r.a) (void)hipEventDestroy(r.a);
      if (r.b) (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct psdns_plan {
  psdns_plan_params p;
  Layout L;
  Ops ops;
  void* tw = nullptr;
  SlotDev* slots_dev = nullptr;
  std::vector<SlotDev> slots_host;
  int device = 0;
  EventTimer* timer = nullptr;
  double acc_ms[KID_COUNT] = {0};
  int acc_n[KID_COUNT] = {0};
  std::vector<float> samples[KID_COUNT];  // per-launch milliseconds since the last psdns_get_timing
  // captured graph of one RK4 step (psdns_set_graph)
  bool use_graph = false;
  hipGraphExec_t graph_exec = nullptr;
  const void* graph_state = nullptr;
  const void* graph_ws = nullptr;
  double graph_dt = 0.0;
  bool graph_hold = false;  // captured with the hold forcing's step structure
  bool graph_expl = false;  // captured with the unfused stages of an explicit-integrator slot
  bool general = false;     // runs the general kernels (ops_general)
  int psched[kNumPasses] = {0, 0, 0, 0, 0};  // schedule of each pass (psdns_set_pass_schedules)
};

namespace {

Ctx make_ctx(psdns_plan* plan, void* ws) {
  Ctx c{};
  c.g = plan->L.g;
  for (int p = 0; p < kNumPasses; ++p) c.psched[p] = plan->psched[p];
  c.tw = plan->tw;
  c.slots = plan->slots_dev;
  char* w = static_cast<char*>(ws);
  c.dyn = reinterpret_cast<DynDev*>(w + plan->L.off_dyn);
  c.fband = reinterpret_cast<double*>(w + plan->L.off_fband);
  c.part = reinterpret_cast<double*>(w + plan->L.off_part);
  c.part_len = plan->L.part_len;
  c.stat = reinterpret_cast<double*>(w + plan->L.off_stat);
  c.nbm = plan->L.nbm;
  c.spectra_rec = plan->L.rec;
  c.ystage = w + plan->L.off_ystage;
  c.acc = w + plan->L.off_acc;
  c.abuf = w + plan->L.off_abuf;
  c.bbuf = w + plan->L.off_bbuf;
  c.akeep = plan->L.g.sphere ? w + plan->L.off_akeep : nullptr;
  c.timer = plan->timer;
  return c;
}

// simulated time of every slot into a record block
__global__ void k_record_time(const DynDev* __restrict__ d, double* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = d[i].t;
}

__global__ void k_clear_dyn(DynDev* d, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    DynDev z{};
    d[i] = z;
  }
}

__global__ void k_clear_doubles(double* p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// Step records and stochastic-forcing vectors of slots [first, first + count) start from zero.
// A small kernel, not hipMemsetAsync, so that the clear may be recorded in a captured graph.
psdns_status clear_slots(psdns_plan* plan, void* ws, int first, int count, hipStream_t s) {
  Ctx c = make_ctx(plan, ws);
  k_clear_dyn<<<(count + 63) / 64, 64, 0, s>>>(c.dyn + first, count);
  const long long per = (long long)kStochCand * 12;
  const long long nb = (long long)count * per;
  k_clear_doubles<<<(unsigned)((nb + 255) / 256), 256, 0, s>>>(c.fband + first * per, nb);
  HIP_TRY(hipGetLastError());
  return PSDNS_OK;
}

// device bytes a plan allocates for itself (twiddle and slot tables)
size_t plan_table_bytes(const psdns_plan_params* p) {
  const size_t cs = p->precision == 32 ? 8 : 16;
  return align_up((size_t)root_table_entries(p->n) * cs, 256) + align_up(sizeof(SlotDev) * (size_t)p->batch, 256);
}

psdns_status check_plan(const psdns_plan* plan) {
  if (!plan) return fail(PSDNS_E_INVAL, "plan is NULL");
  return PSDNS_OK;
}

// The stage launcher: each pass in the schedule Ctx::psched names (plans with one
// schedule only: that one).
RhsStageFn stage_fn(const psdns_plan* plan) {
  return plan->ops.rhs_mixed ? plan->ops.rhs_mixed : plan->ops.sched[0].rhs_stage;
}

// Whether an active slot uses the explicit integrator (the fused passes do not run it).
bool any_explicit(const psdns_plan* plan) {
  for (int i = 0; i < plan->p.batch; ++i)
    if (plan->slots_host[i].active && plan->slots_host[i].integrator == PSDNS_INTEGRATOR_EXPLICIT) return true;
  return false;
}

// The steps of psdns_step on workspace ws (graph replay when allowed and enabled).
psdns_status run_steps(psdns_plan* plan, void* state, void* ws, double dt, int nsteps, hipStream_t s,
                       bool allow_graph, Timer* timer) {
  Ctx c = make_ctx(plan, ws);
  c.timer = timer;
  // Every stage's last pass also inverts the next stage input along z (it is in its
  // registers already), so only the first stage of a call runs the standalone z pass.
  // The last stage of a call is fused too, although its inverse goes unused: each
  // y_{n+1} then comes from the same kernel however the steps are split into calls or
  // replayed from a graph, so the results are bitwise the same (the fused and unfused
  // passes compute the same sums, but the compiler may round them differently).
  // With the hold forcing y_{n+1} is rescaled on the band after the last stage, so that
  // stage cannot run the next step's z inverse: every step then starts with its own.
  bool hold = false;
  for (int i = 0; i < plan->p.batch; ++i)
    hold = hold || (plan->slots_host[i].active && plan->slots_host[i].forcing == PSDNS_FORCING_HOLD);
  // The fused passes update integrating-factor slots only; a batch with an explicit-
  // integrator slot runs every stage unfused (its own z inverse, then the update).
  const bool expl = any_explicit(plan);
  auto one_step = [&](const Ctx& cx, bool first) {
    for (int stage = 0; stage < 4; ++stage) {
      const void* sin = stage == 0 ? state : cx.ystage;
      int fl = kStageFuse;
      if ((first || hold) && stage == 0) fl |= kStageZinv;
      if (hold && stage == 3) fl &= ~kStageFuse;
      if (expl) fl = kStageZinv;
      stage_fn(plan)(cx, state, sin, stage, nullptr, stage == 0, dt, fl, s);
    }
    if (hold) plan->ops.band_hold(cx, state, s);
  };
  if (allow_graph && s != nullptr && nsteps > 0) {
    if (!plan->graph_exec || plan->graph_state != state || plan->graph_ws != ws || plan->graph_dt != dt ||
        plan->graph_hold != hold || plan->graph_expl != expl) {
      if (plan->graph_exec) {
        HIP_TRY(hipGraphExecDestroy(plan->graph_exec));
        plan->graph_exec = nullptr;
      }
      Ctx cc = c;
      cc.timer = nullptr;  // no event records inside a captured graph
      HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      one_step(cc, false);
      hipGraph_t graph = nullptr;
      const hipError_t le = hipGetLastError();
      const hipError_t ce = hipStreamEndCapture(s, &graph);
      if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(le, "kernel launch during graph capture");
      }
      if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
      hipError_t ie = hipGraphInstantiate(&plan->graph_exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        plan->graph_exec = nullptr;
        return hip_fail(ie, "hipGraphInstantiate");
      }
      plan->graph_state = state;
      plan->graph_ws = ws;
      plan->graph_hold = hold;
      plan->graph_expl = expl;
      plan->graph_dt = dt;
    }
    // the captured step expects the z inverse of y_n: run it once, then replay
    stage_fn(plan)(c, state, state, 0, nullptr, 0, dt, kStageZinv | kStagePrologue, s);
    HIP_TRY(hipGetLastError());
    for (int n = 0; n < nsteps; ++n) {
      if (timer) timer->begin(KID_STEP, s);
      HIP_TRY(hipGraphLaunch(plan->graph_exec, s));
      if (timer) timer->end(KID_STEP, s);
    }
    return PSDNS_OK;
  }
  for (int n = 0; n < nsteps; ++n) {
    if (timer) timer->begin(KID_STEP, s);
    one_step(c, n == 0);
    if (timer) timer->end(KID_STEP, s);
    HIP_TRY(hipGetLastError());
  }
  return PSDNS_OK;
}


// Streaming copy (psdns_stream_copy): 16-byte accesses, four loads in flight per thread,
// grid-stride over the buffer.
__global__ void __launch_bounds__(256)
k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * 256;
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n; i += stride) dst[i] = src[i];
}

// Step records of every slot into a caller's device buffer (psdns_step_noalloc).
__global__ void k_export_info(const DynDev* __restrict__ d, const SlotDev* __restrict__ slots,
                              psdns_step_info* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    psdns_step_info r;
    r.t = d[i].t;
    r.dt = d[i].dt;
    r.max_u = d[i].max_u;
    r.steps = d[i].steps;
    r.flags = d[i].flags;
    r.active = slots[i].active;
    out[i] = r;
  }
}

}  // namespace

// Workspace of psdns_step_noalloc: a fixed device array, one copy per GPU, held until the
// process ends.  In host code `scratch` names a host-side handle, not device memory; its
// device address is looked up once per device (hipGetSymbolAddress with that device
// current) and only that address is used.
static __device__ __align__(256) unsigned char scratch[PSDNS_NOALLOC_MAX_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

psdns_status scratch_of_device(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(PSDNS_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(PSDNS_E_HIP, "hipGetSymbolAddress(scratch) returned no address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PSDNS_OK;
}

}  // namespace

extern "C" {

size_t psdns_state_bytes(const psdns_plan_params* p) {
  std::string why;
  if (!valid_params(p, &why)) return 0;
  return make_layout(p).st_bytes;
}

size_t psdns_workspace_bytes(const psdns_plan_params* p) {
  std::string why;
  if (!valid_params(p, &why)) return 0;
  return make_layout(p).ws_bytes;
}

size_t psdns_plan_device_bytes(const psdns_plan_params* p) {
  std::string why;
  if (!valid_params(p, &why)) return 0;
  return plan_table_bytes(p);
}

psdns_status psdns_plan_create(const psdns_plan_params* p, psdns_plan** out) {
  if (!out) return fail(PSDNS_E_INVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!valid_params(p, &why)) return fail(PSDNS_E_INVAL, why);
  psdns_plan* plan = new (std::nothrow) psdns_plan();
  if (!plan) return fail(PSDNS_E_NOMEM, "host allocation of the plan failed");
  plan->p = *p;
  plan->ops = ops_for(p);
  plan->general = general_plan(p);
  if (plan->general) plan->ops.sched[0].x_lines = general_x_lines(p->n, p->precision);
  plan->L = make_layout(p);
  hipError_t e = hipGetDevice(&plan->device);
  if (e != hipSuccess) {
    delete plan;
    return hip_fail(e, "hipGetDevice");
  }
  // root table (layout in common.hpp), computed in double precision: twiddles
  // w_N^m = exp(-2 pi i m / N), the roots of the odd radices, the half-cell shift phases
  const int n = p->n;
  const size_t nent = (size_t)root_table_entries(n);
  const size_t twb = nent * plan->L.csize;
  std::vector<double> twd(2 * nent);
  for (int m = 0; m < n; ++m) {
    const double a = 2.0 * M_PI * (double)m / (double)n;
    twd[2 * m] = std::cos(a);
    twd[2 * m + 1] = -std::sin(a);
  }
  for (int R : kOddRadices)
    for (int m = 0; m < R; ++m) {
      const size_t i = (size_t)n + kRootOff(R) + m;
      twd[2 * i] = std::cos(2.0 * M_PI * m / R);
      twd[2 * i + 1] = -std::sin(2.0 * M_PI * m / R);
    }
  for (int k = 0; k <= n / 2; ++k) {
    const size_t i = (size_t)n + kShiftOff + k;
    twd[2 * i] = std::cos(M_PI * k / n);
    twd[2 * i + 1] = std::sin(M_PI * k / n);
  }
  std::vector<char> host(twb);
  if (p->precision == 32) {
    float* f = reinterpret_cast<float*>(host.data());
    for (size_t i = 0; i < 2 * nent; ++i) f[i] = (float)twd[i];
  } else {
    std::memcpy(host.data(), twd.data(), twb);
  }
  e = hipMalloc(&plan->tw, twb);
  if (e != hipSuccess) {
    delete plan;
    return fail(PSDNS_E_NOMEM, std::string("hipMalloc(twiddles): ") + hipGetErrorString(e));
  }
  e = hipMalloc(reinterpret_cast<void**>(&plan->slots_dev), sizeof(SlotDev) * p->batch);
  if (e != hipSuccess) {
    (void)hipFree(plan->tw);
    delete plan;
    return fail(PSDNS_E_NOMEM, std::string("hipMalloc(slot table): ") + hipGetErrorString(e));
  }
  plan->slots_host.resize(p->batch);
  for (auto& s : plan->slots_host) {
    std::memset(&s, 0, sizeof(s));
    s.kf2 = 4.0;
    s.active = 1;
  }
  e = hipMemcpy(plan->tw, host.data(), twb, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(plan->slots_dev, plan->slots_host.data(), sizeof(SlotDev) * p->batch, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(plan->tw);
    (void)hipFree(plan->slots_dev);
    delete plan;
    return hip_fail(e, "hipMemcpy(plan tables)");
  }
  *out = plan;
  return PSDNS_OK;
}

psdns_status psdns_plan_destroy(psdns_plan* plan) {
  if (!plan) return PSDNS_OK;
  if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
  delete plan->timer;
  if (plan->tw) (void)hipFree(plan->tw);
  if (plan->slots_dev) (void)hipFree(plan->slots_dev);
  delete plan;
  return PSDNS_OK;
}

psdns_status psdns_plan_get_info(const psdns_plan* plan, psdns_plan_info* out) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!out) return fail(PSDNS_E_INVAL, "out is NULL");
  const Geom& g = plan->L.g;
  out->n = g.N;
  out->k_max = g.K;
  out->m = g.M;
  out->kx_count = g.KX;
  out->kx_pitch = g.PX;
  out->n_scalars = g.S;
  out->precision = plan->p.precision;
  out->batch = g.batch;
  out->n_shells = g.ns;
  out->spectra_doubles = plan->L.rec;
  out->state_bytes = (int64_t)plan->L.st_bytes;
  out->workspace_bytes = (int64_t)plan->L.ws_bytes;
  out->plan_bytes = (int64_t)plan_table_bytes(&plan->p);
  out->dealias = plan->p.dealias;
  out->general = plan->general ? 1 : 0;
  out->elems_col = plan->ops.sched[plan->psched[kPassYInverse]].ec;
  out->elems_x = plan->ops.sched[plan->psched[kPassX]].ex;
  out->n_schedules = plan->ops.nsched;
  out->schedule = plan->psched[0];
  for (int p = 0; p < kNumPasses; ++p) {
    out->pass_schedules[p] = plan->psched[p];
    if (plan->psched[p] != plan->psched[0]) out->schedule = -1;
  }
  return PSDNS_OK;
}

psdns_status psdns_get_schedule_info(const psdns_plan* plan, int32_t index, psdns_schedule_info* out) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!out) return fail(PSDNS_E_INVAL, "out is NULL");
  if (index < 0 || index >= plan->ops.nsched)
    return fail(PSDNS_E_INVAL, "schedule index out of range [0, " + std::to_string(plan->ops.nsched) + ")");
  const StepSched& d = plan->ops.sched[index];
  out->index = index;
  out->elems_col = d.ec;
  out->col_width = d.col_w;
  out->elems_fused = d.fused_ec;
  out->fused_width = d.fused_w;
  out->elems_x = d.ex;
  out->x_lines = d.x_lines;
  return PSDNS_OK;
}

psdns_status psdns_set_pass_schedules(psdns_plan* plan, const int32_t* sched) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!sched) return fail(PSDNS_E_INVAL, "sched is NULL");
  bool same = true;
  for (int p = 0; p < kNumPasses; ++p) {
    if (sched[p] < 0 || sched[p] >= plan->ops.nsched)
      return fail(PSDNS_E_INVAL, "schedule index out of range [0, " + std::to_string(plan->ops.nsched) + ")");
    same = same && sched[p] == plan->psched[p];
  }
  if (!same && plan->graph_exec) {
    // a captured step holds the kernels of the old schedules
    HIP_TRY(hipGraphExecDestroy(plan->graph_exec));
    plan->graph_exec = nullptr;
  }
  for (int p = 0; p < kNumPasses; ++p) plan->psched[p] = sched[p];
  return PSDNS_OK;
}

psdns_status psdns_use_general_kernels(psdns_plan* plan) {
  if (psdns_status s = check_plan(plan)) return s;
  if (plan->general) return PSDNS_OK;
  if (plan->graph_exec) {
    HIP_TRY(hipGraphExecDestroy(plan->graph_exec));
    plan->graph_exec = nullptr;
  }
  plan->ops = ops_general(plan->p.precision);
  plan->ops.sched[0].x_lines = general_x_lines(plan->p.n, plan->p.precision);
  for (int p = 0; p < kNumPasses; ++p) plan->psched[p] = 0;
  plan->general = true;
  return PSDNS_OK;
}

psdns_status psdns_set_schedule(psdns_plan* plan, int32_t index) {
  if (psdns_status s = check_plan(plan)) return s;
  if (index < 0 || index >= plan->ops.nsched)
    return fail(PSDNS_E_INVAL, "schedule index out of range [0, " + std::to_string(plan->ops.nsched) + ")");
  const int32_t all[kNumPasses] = {index, index, index, index, index};
  return psdns_set_pass_schedules(plan, all);
}

psdns_status psdns_set_slot(psdns_plan* plan, int32_t slot, const psdns_slot_params* prm, int32_t active) {
  if (psdns_status s = check_plan(plan)) return s;
  if (slot < 0 || slot >= plan->p.batch) return fail(PSDNS_E_INVAL, "slot out of range");
  if (!prm) return fail(PSDNS_E_INVAL, "params is NULL");
  if (!(prm->nu >= 0.0) || !std::isfinite(prm->nu)) return fail(PSDNS_E_INVAL, "nu must be finite and >= 0");
  if (!(prm->power >= 0.0) || !std::isfinite(prm->power)) return fail(PSDNS_E_INVAL, "power must be finite and >= 0");
  if (!(prm->k_force > 0.0) || !std::isfinite(prm->k_force)) return fail(PSDNS_E_INVAL, "k_force must be > 0");
  SlotDev s{};
  s.nu = prm->nu;
  s.power = prm->power;
  s.kf2 = prm->k_force * prm->k_force;
  for (int i = 0; i < 3; ++i) s.diff[i] = prm->nu;
  for (int i = 0; i < plan->p.n_scalars; ++i) {
    if (!(prm->schmidt[i] > 0.0) || !std::isfinite(prm->schmidt[i]))
      return fail(PSDNS_E_INVAL, "schmidt numbers must be finite and > 0");
    s.diff[3 + i] = prm->nu / prm->schmidt[i];
    for (int d = 0; d < 3; ++d) {
      if (!std::isfinite(prm->mean_grad[i][d])) return fail(PSDNS_E_INVAL, "mean gradient must be finite");
      s.g[i][d] = prm->mean_grad[i][d];
    }
  }
  if (prm->forcing != PSDNS_FORCING_POWER && prm->forcing != PSDNS_FORCING_HOLD &&
      prm->forcing != PSDNS_FORCING_STOCHASTIC && prm->forcing != PSDNS_FORCING_ALVELIUS)
    return fail(PSDNS_E_INVAL,
                "forcing must be PSDNS_FORCING_POWER, PSDNS_FORCING_HOLD, PSDNS_FORCING_STOCHASTIC or "
                "PSDNS_FORCING_ALVELIUS");
  if (prm->forcing == PSDNS_FORCING_ALVELIUS && !(prm->k_force < PSDNS_STOCHASTIC_KF_MAX + 1.0))
    return fail(PSDNS_E_INVAL, "k_force must be below PSDNS_STOCHASTIC_KF_MAX + 1 with PSDNS_FORCING_ALVELIUS");
  if (prm->forcing == PSDNS_FORCING_STOCHASTIC) {
    if (!(prm->stoch_sigma >= 0.0) || !std::isfinite(prm->stoch_sigma))
      return fail(PSDNS_E_INVAL, "stoch_sigma must be finite and >= 0");
    if (!(prm->stoch_tl > 0.0) || !std::isfinite(prm->stoch_tl))
      return fail(PSDNS_E_INVAL, "stoch_tl must be finite and > 0");
    if (!(prm->k_force < PSDNS_STOCHASTIC_KF_MAX + 1.0))
      return fail(PSDNS_E_INVAL, "k_force must be below PSDNS_STOCHASTIC_KF_MAX + 1 with PSDNS_FORCING_STOCHASTIC");
  }
  if (prm->forcing == PSDNS_FORCING_HOLD && (!(prm->hold_energy > 0.0) || !std::isfinite(prm->hold_energy)))
    return fail(PSDNS_E_INVAL, "hold_energy must be finite and > 0 with PSDNS_FORCING_HOLD");
  if (prm->integrator != PSDNS_INTEGRATOR_IF && prm->integrator != PSDNS_INTEGRATOR_EXPLICIT)
    return fail(PSDNS_E_INVAL, "integrator must be PSDNS_INTEGRATOR_IF or PSDNS_INTEGRATOR_EXPLICIT");
  s.integrator = prm->integrator;
  s.forcing = prm->forcing;
  s.hold = prm->forcing == PSDNS_FORCING_HOLD ? prm->hold_energy : 0.0;
  s.sigma = prm->forcing == PSDNS_FORCING_STOCHASTIC ? prm->stoch_sigma : 0.0;
  s.tl = prm->forcing == PSDNS_FORCING_STOCHASTIC ? prm->stoch_tl : 1.0;
  s.seed = prm->stoch_seed;
  s.active = active ? 1 : 0;
  plan->slots_host[slot] = s;
  HIP_TRY(hipMemcpy(plan->slots_dev + slot, &s, sizeof(SlotDev), hipMemcpyHostToDevice));
  return PSDNS_OK;
}

psdns_status psdns_init_field_spectrum(psdns_plan* plan, void* state, void* ws, int32_t slot, uint64_t seed,
                                       int32_t spectrum, double k_param, double kinetic_energy, void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!state || !ws) return fail(PSDNS_E_INVAL, "state and ws must be device pointers");
  if (slot < 0 || slot >= plan->p.batch) return fail(PSDNS_E_INVAL, "slot out of range");
  if (spectrum != PSDNS_SPECTRUM_CONFIG && spectrum != PSDNS_SPECTRUM_PAPER)
    return fail(PSDNS_E_INVAL, "spectrum must be PSDNS_SPECTRUM_CONFIG or PSDNS_SPECTRUM_PAPER");
  if (!(k_param > 0.0) || !std::isfinite(k_param)) return fail(PSDNS_E_INVAL, "k_peak / k_force must be > 0");
  if (!(kinetic_energy >= 0.0) || !std::isfinite(kinetic_energy))
    return fail(PSDNS_E_INVAL, "kinetic_energy must be >= 0");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // a new realization: its step record and stochastic-forcing vector start from zero
  if (psdns_status st = clear_slots(plan, ws, slot, 1, s)) return st;
  Ctx c = make_ctx(plan, ws);
  plan->ops.init_field(c, state, slot, seed, k_param, spectrum, kinetic_energy, s);
  HIP_TRY(hipGetLastError());
  return PSDNS_OK;
}

psdns_status psdns_init_field(psdns_plan* plan, void* state, void* ws, int32_t slot, uint64_t seed, double k_peak,
                              double kinetic_energy, void* hip_stream) {
  return psdns_init_field_spectrum(plan, state, ws, slot, seed, PSDNS_SPECTRUM_CONFIG, k_peak, kinetic_energy,
                                   hip_stream);
}

psdns_status psdns_zero_scalars(psdns_plan* plan, void* state, int32_t slot, void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!state) return fail(PSDNS_E_INVAL, "state must be a device pointer");
  if (slot < 0 || slot >= plan->p.batch) return fail(PSDNS_E_INVAL, "slot out of range");
  Ctx c{};
  c.g = plan->L.g;
  plan->ops.zero_scalars(c, state, slot, static_cast<hipStream_t>(hip_stream));
  HIP_TRY(hipGetLastError());
  return PSDNS_OK;
}

psdns_status psdns_rhs(psdns_plan* plan, const void* state, void* out, void* ws, void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!state || !out || !ws) return fail(PSDNS_E_INVAL, "state, out and ws must be device pointers");
  if (state == out) return fail(PSDNS_E_INVAL, "out must not alias state");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Ctx c = make_ctx(plan, ws);
  stage_fn(plan)(c, const_cast<void*>(state), state, -1, out, 0, 0.0, kStageZinv, s);
  HIP_TRY(hipGetLastError());
  return PSDNS_OK;
}

psdns_status psdns_tune(psdns_plan* plan, const void* state, void* ws, int32_t reps, double* ms_out,
                        int32_t* best, void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!state || !ws) return fail(PSDNS_E_INVAL, "state and ws must be device pointers");
  if (reps < 1 || reps > 1000) return fail(PSDNS_E_INVAL, "reps must be in [1, 1000]");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Ctx c = make_ctx(plan, ws);
  c.timer = nullptr;  // the trial launches are not part of the kernel timing record
  std::vector<double> ms(plan->ops.nsched, 0.0);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(PSDNS_E_HIP, "hipEventCreate failed");
  }
  hipError_t err = hipSuccess;
  int b = 0;
  for (int i = 0; i < plan->ops.nsched && err == hipSuccess; ++i) {
    RhsStageFn f = plan->ops.sched[i].rhs_stage;
    // one untimed trial, then reps timed ones.  A trial is a steady-state RK stage of a
    // multi-step call (stage 1: forcing amplitude, y inverse, x pass, y forward and the
    // fused z pass); it reads the state and writes only workspace buffers (accumulator,
    // stage input on the band, transform buffers), all of which a step rebuilds.
    void* st = const_cast<void*>(state);
    const int fl = any_explicit(plan) ? kStageZinv : kStageFuse;  // the stage a step would run
    f(c, st, c.ystage, 1, nullptr, 0, 0.0, fl, s);
    err = hipEventRecord(e0, s);
    for (int r = 0; r < reps && err == hipSuccess; ++r) f(c, st, c.ystage, 1, nullptr, 0, 0.0, fl, s);
    if (err == hipSuccess) err = hipEventRecord(e1, s);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    if (err == hipSuccess) err = hipGetLastError();
    ms[i] = (double)t / reps;
    if (ms[i] < ms[b]) b = i;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return hip_fail(err, "schedule trial");
  if (ms_out)
    for (int i = 0; i < plan->ops.nsched; ++i) ms_out[i] = ms[i];
  if (best) *best = b;
  return psdns_set_schedule(plan, b);
}

psdns_status psdns_tune_passes(psdns_plan* plan, const void* state, void* ws, int32_t reps, double* ms_out,
                               int32_t* best, void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!state || !ws) return fail(PSDNS_E_INVAL, "state and ws must be device pointers");
  if (reps < 1 || reps > 1000) return fail(PSDNS_E_INVAL, "reps must be in [1, 1000]");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const int ns = plan->ops.nsched;
  const bool expl = any_explicit(plan);
  // kernel record of each pass in the stage a step runs
  const int kid[kNumPasses] = {KID_ZINV, KID_YINV, KID_XPASS, KID_YFWD, expl ? KID_ZFWD : KID_ZFWDI};
  std::vector<double> ms((size_t)ns * kNumPasses, 0.0);
  for (int i = 0; i < ns; ++i) {
    Ctx c = make_ctx(plan, ws);
    for (int p = 0; p < kNumPasses; ++p) c.psched[p] = i;
    EventTimer t;
    void* st = const_cast<void*>(state);
    const int fl = expl ? kStageZinv : kStageFuse;
    // untimed trial, then reps timed ones of the standalone z inverse (of the state) and
    // of the steady stage (the trial of psdns_tune); workspace buffers only
    c.timer = nullptr;
    stage_fn(plan)(c, st, st, 0, nullptr, 0, 0.0, kStageZinv | kStagePrologue, s);
    stage_fn(plan)(c, st, c.ystage, 1, nullptr, 0, 0.0, fl, s);
    c.timer = &t;
    for (int r = 0; r < reps; ++r) {
      stage_fn(plan)(c, st, st, 0, nullptr, 0, 0.0, kStageZinv | kStagePrologue, s);
      stage_fn(plan)(c, st, c.ystage, 1, nullptr, 0, 0.0, fl, s);
    }
    HIP_TRY(hipGetLastError());
    if (t.err != hipSuccess) return hip_fail(t.err, "hipEventCreate");
    double sum[KID_COUNT] = {0};
    int cnt[KID_COUNT] = {0};
    for (auto& r : t.recs) {
      if (!(r.a && r.b && r.closed)) continue;
      HIP_TRY(hipEventSynchronize(r.b));
      float e = 0.f;
      HIP_TRY(hipEventElapsedTime(&e, r.a, r.b));
      sum[r.kid] += e;
      cnt[r.kid] += 1;
    }
    for (int p = 0; p < kNumPasses; ++p)
      ms[(size_t)i * kNumPasses + p] = cnt[kid[p]] ? sum[kid[p]] / cnt[kid[p]] : 0.0;
  }
  // the lowest-index schedule within 1% of the fastest: schedules whose kernels coincide at
  // this size (or differ within the timing noise) resolve to the same choice on every run
  int32_t pick[kNumPasses];
  for (int p = 0; p < kNumPasses; ++p) {
    double lo = ms[p];
    for (int i = 1; i < ns; ++i) lo = std::min(lo, ms[(size_t)i * kNumPasses + p]);
    pick[p] = 0;
    while (pick[p] < ns - 1 && ms[(size_t)pick[p] * kNumPasses + p] > 1.01 * lo) ++pick[p];
  }
  if (ms_out)
    for (size_t k = 0; k < ms.size(); ++k) ms_out[k] = ms[k];
  if (best)
    for (int p = 0; p < kNumPasses; ++p) best[p] = pick[p];
  return psdns_set_pass_schedules(plan, pick);
}

psdns_status psdns_step(psdns_plan* plan, void* state, void* ws, double dt, int32_t nsteps, void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!state || !ws) return fail(PSDNS_E_INVAL, "state and ws must be device pointers");
  if (nsteps < 0) return fail(PSDNS_E_INVAL, "nsteps must be >= 0");
  if (!(dt != 0.0) || !std::isfinite(dt)) return fail(PSDNS_E_INVAL, "dt must be finite and nonzero");
  return run_steps(plan, state, ws, dt, nsteps, static_cast<hipStream_t>(hip_stream), plan->use_graph, plan->timer);
}

psdns_status psdns_step_noalloc(psdns_plan* plan, void* state, double dt, int32_t nsteps, psdns_step_info* info_out,
                                void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!state) return fail(PSDNS_E_INVAL, "state must be a device pointer");
  if (nsteps < 0) return fail(PSDNS_E_INVAL, "nsteps must be >= 0");
  if (!(dt != 0.0) || !std::isfinite(dt)) return fail(PSDNS_E_INVAL, "dt must be finite and nonzero");
  if (plan->L.ws_bytes > (size_t)PSDNS_NOALLOC_MAX_WORKSPACE_BYTES)
    return fail(PSDNS_E_INVAL, "the plan's workspace (" + std::to_string(plan->L.ws_bytes) +
                                   " bytes) exceeds the static scratch of psdns_step_noalloc (" +
                                   std::to_string((size_t)PSDNS_NOALLOC_MAX_WORKSPACE_BYTES) + " bytes)");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != plan->device) return fail(PSDNS_E_INVAL, "the current device is not the plan's device");
  void* ws = nullptr;
  if (psdns_status st = scratch_of_device(dev, &ws)) return st;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // the array keeps the last call's contents: every call starts its records from zero
  if (psdns_status st = clear_slots(plan, ws, 0, plan->p.batch, s)) return st;
  if (psdns_status st = run_steps(plan, state, ws, dt, nsteps, s, false, nullptr)) return st;
  if (info_out) {
    const int b = plan->p.batch;
    k_export_info<<<(b + 63) / 64, 64, 0, s>>>(make_ctx(plan, ws).dyn, plan->slots_dev, info_out, b);
    HIP_TRY(hipGetLastError());
  }
  return PSDNS_OK;
}

psdns_status psdns_set_graph(psdns_plan* plan, int32_t enable) {
  if (psdns_status s = check_plan(plan)) return s;
  plan->use_graph = enable != 0;
  if (!plan->use_graph && plan->graph_exec) {
    HIP_TRY(hipGraphExecDestroy(plan->graph_exec));
    plan->graph_exec = nullptr;
  }
  return PSDNS_OK;
}

psdns_status psdns_run(psdns_plan* plan, void* state, void* ws, double dt, int32_t nsteps, int32_t every,
                       double* records, int32_t flags, void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!records) return fail(PSDNS_E_INVAL, "records must be a device pointer");
  if (every < 1) return fail(PSDNS_E_INVAL, "every must be >= 1");
  if (nsteps < 0) return fail(PSDNS_E_INVAL, "nsteps must be >= 0");
  if (flags < 1 || flags > 3) return fail(PSDNS_E_INVAL, "flags must be a nonzero combination of PSDNS_SPECTRA_*");
  const int B = plan->p.batch;
  const size_t block = (size_t)B * (1 + plan->L.rec);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int done = 0;
  for (int r = 0; done + every <= nsteps; ++r) {
    if (psdns_status st = psdns_step(plan, state, ws, dt, every, hip_stream)) return st;
    done += every;
    double* blk = records + (size_t)r * block;
    k_record_time<<<(B + 255) / 256, 256, 0, s>>>(reinterpret_cast<const DynDev*>(static_cast<char*>(ws) + plan->L.off_dyn),
                                                  blk, B);
    HIP_TRY(hipGetLastError());
    if (psdns_status st = psdns_spectra(plan, state, ws, blk + B, flags, hip_stream)) return st;
  }
  if (done < nsteps) return psdns_step(plan, state, ws, dt, nsteps - done, hip_stream);
  return PSDNS_OK;
}

psdns_status psdns_pressure(psdns_plan* plan, const void* state, void* ws, void* canonical_out, void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!state || !ws || !canonical_out) return fail(PSDNS_E_INVAL, "state, ws and canonical_out must be device pointers");
  if (state == canonical_out) return fail(PSDNS_E_INVAL, "canonical_out must not alias state");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (!plan->ops.pressure)
    return fail(PSDNS_E_UNSUPPORTED,
                "psdns_pressure is not available for plans with the general kernels or the phase-shift dealiasing");
  Ctx c = make_ctx(plan, ws);
  std::vector<int> active(plan->p.batch);
  for (int i = 0; i < plan->p.batch; ++i) active[i] = plan->slots_host[i].active;
  plan->ops.pressure(c, state, canonical_out, active.data(), s);
  HIP_TRY(hipGetLastError());
  return PSDNS_OK;
}

psdns_status psdns_spectra(psdns_plan* plan, const void* state, void* ws, double* out, int32_t flags,
                           void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!state || !ws || !out) return fail(PSDNS_E_INVAL, "state, ws and out must be device pointers");
  if (flags & ~3) return fail(PSDNS_E_INVAL, "flags must be a combination of PSDNS_SPECTRA_SHELLS and PSDNS_SPECTRA_MOMENTS");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Ctx c = make_ctx(plan, ws);
  plan->ops.spectra(c, state, out, flags, s);
  HIP_TRY(hipGetLastError());
  return PSDNS_OK;
}

psdns_status psdns_read_step_info(psdns_plan* plan, const void* ws, psdns_step_info* out, void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!ws || !out) return fail(PSDNS_E_INVAL, "ws and out must be non-NULL");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::vector<DynDev> d(plan->p.batch);
  Ctx c = make_ctx(plan, const_cast<void*>(ws));
  HIP_TRY(hipMemcpyAsync(d.data(), c.dyn, sizeof(DynDev) * d.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < plan->p.batch; ++i) {
    out[i].t = d[i].t;
    out[i].dt = d[i].dt;
    out[i].max_u = d[i].max_u;
    out[i].steps = d[i].steps;
    out[i].flags = d[i].flags;
    out[i].active = plan->slots_host[i].active;
  }
  return PSDNS_OK;
}

psdns_status psdns_clear_step_info(psdns_plan* plan, void* ws, void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!ws) return fail(PSDNS_E_INVAL, "ws is NULL");
  return clear_slots(plan, ws, 0, plan->p.batch, static_cast<hipStream_t>(hip_stream));
}

psdns_status psdns_clear_slot_info(psdns_plan* plan, void* ws, int32_t slot, void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!ws) return fail(PSDNS_E_INVAL, "ws is NULL");
  if (slot < 0 || slot >= plan->p.batch) return fail(PSDNS_E_INVAL, "slot out of range");
  return clear_slots(plan, ws, slot, 1, static_cast<hipStream_t>(hip_stream));
}

psdns_status psdns_get_state(psdns_plan* plan, const void* state, int32_t slot, void* canonical_out,
                             void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!state || !canonical_out) return fail(PSDNS_E_INVAL, "state and canonical_out must be device pointers");
  if (slot < 0 || slot >= plan->p.batch) return fail(PSDNS_E_INVAL, "slot out of range");
  Ctx c = make_ctx(plan, nullptr);
  c.timer = plan->timer;
  plan->ops.get_state(c, state, slot, canonical_out, static_cast<hipStream_t>(hip_stream));
  HIP_TRY(hipGetLastError());
  return PSDNS_OK;
}

psdns_status psdns_set_state(psdns_plan* plan, void* state, int32_t slot, const void* canonical_in,
                             void* hip_stream) {
  if (psdns_status s = check_plan(plan)) return s;
  if (!state || !canonical_in) return fail(PSDNS_E_INVAL, "state and canonical_in must be device pointers");
  if (slot < 0 || slot >= plan->p.batch) return fail(PSDNS_E_INVAL, "slot out of range");
  Ctx c = make_ctx(plan, nullptr);
  plan->ops.set_state(c, state, slot, canonical_in, static_cast<hipStream_t>(hip_stream));
  HIP_TRY(hipGetLastError());
  return PSDNS_OK;
}

psdns_status psdns_set_timing(psdns_plan* plan, int32_t enable) {
  if (psdns_status s = check_plan(plan)) return s;
  if (enable && !plan->timer) plan->timer = new (std::nothrow) EventTimer();
  if (!enable && plan->timer) {
    delete plan->timer;
    plan->timer = nullptr;
  }
  return PSDNS_OK;
}

psdns_status psdns_get_timing(psdns_plan* plan, psdns_kernel_timing* out, int32_t max, int32_t* count) {
  if (psdns_status s = check_plan(plan)) return s;
  EventTimer* t = plan->timer;
  if (t) {
    if (t->err != hipSuccess) return hip_fail(t->err, "hipEventCreate");
    for (auto& r : t->recs) {
      if (r.a && r.b && r.closed) {
        HIP_TRY(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        plan->acc_ms[r.kid] += ms;
        plan->acc_n[r.kid] += 1;
        plan->samples[r.kid].push_back(ms);
      }
      if (r.a) t->pool.push_back(r.a);
      if (r.b) t->pool.push_back(r.b);
    }
    t->recs.clear();
  }
  int k = 0;
  for (int i = 0; i < KID_COUNT && k < max; ++i) {
    if (!out) break;
    std::snprintf(out[k].name, sizeof(out[k].name), "%s", kKernelNames[i]);
    out[k].launches = plan->acc_n[i];
    out[k].total_ms = plan->acc_ms[i];
    std::vector<float>& v = plan->samples[i];
    out[k].median_ms = 0.0;
    out[k].min_ms = 0.0;
    if (!v.empty()) {
      std::sort(v.begin(), v.end());
      const size_t n = v.size();
      out[k].median_ms = n % 2 ? v[n / 2] : 0.5 * ((double)v[n / 2 - 1] + v[n / 2]);
      out[k].min_ms = v[0];
    }
    ++k;
  }
  if (count) *count = k;
  for (int i = 0; i < KID_COUNT; ++i) {
    plan->acc_ms[i] = 0;
    plan->acc_n[i] = 0;
    plan->samples[i].clear();
  }
  return PSDNS_OK;
}

psdns_status psdns_stream_copy(void* dst, const void* src, size_t bytes, int32_t blocks, void* hip_stream) {
  if (!dst || !src) return fail(PSDNS_E_INVAL, "dst and src must be device pointers");
  if (bytes % 16 || (reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) % 16)
    return fail(PSDNS_E_INVAL, "bytes and both pointers must be multiples of 16");
  if (blocks < 1 || blocks > (1 << 20)) return fail(PSDNS_E_INVAL, "blocks must be in [1, 2^20]");
  const char* d = static_cast<const char*>(dst);
  const char* q = static_cast<const char*>(src);
  if (d < q + bytes && q < d + bytes) return fail(PSDNS_E_INVAL, "dst and src overlap");
  if (bytes == 0) return PSDNS_OK;
  k_stream_copy<<<blocks, 256, 0, static_cast<hipStream_t>(hip_stream)>>>(static_cast<const uint4*>(src),
                                                                          static_cast<uint4*>(dst), bytes / 16);
  HIP_TRY(hipGetLastError());
  return PSDNS_OK;
}

const char* psdns_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// C ABI of libnse_sphere.so (declared in include/nse_sphere.h): context
// lifetime, argument validation, grouping of members by grid, the NDF_p step
// schedule and the launch sequences of the hot path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "ndf_control.h"
#include "nse_internal.h"

using namespace nse;

// Scratch of nse_nonlinear_adjoint_noalloc (the adjoint's Fourier intermediates
// for callers that cannot allocate): one copy per device, held until the process
// ends. Host code never passes this name to a kernel; it uses the device address
// that hipGetSymbolAddress returns for the current device (bind_noalloc_scratch).
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) double2 scratch[kNoAllocScratchBytes / sizeof(double2)];

namespace {

struct Group {
  int N = 0, nlat = 0, nh = 0, M = 0;
  int precision = NSE_PREC_FP64;
  int mb_synth = 0, mb_anal = 0;     // member blocks of the batched kernels
  std::vector<int> members;          // global member indices
  std::vector<int64_t> offsets;      // complex-slot offsets of those members
  std::vector<double> nu;
  std::vector<double> mu, w;         // all nlat nodes (host)
  FftPlan plan{};
  double *d_mu = nullptr, *d_w = nullptr, *d_T1 = nullptr, *d_T2 = nullptr;
  float *d_T1f = nullptr, *d_T2f = nullptr;
  int64_t* d_t2off = nullptr;
  double2 *d_rec_a = nullptr, *d_rec_g = nullptr, *d_rec_p = nullptr;  // recurrence coefficients (rec_slot)
  uint64_t* d_lps = nullptr;      // split-bf16 synthesis panels (BF16X3 groups)
  int64_t* d_lpsoff = nullptr;
  int64_t lps_stride = 0;         // per member, 8-byte units
  std::vector<int64_t> t2off;  // [N+2] start of order m in T2
  double2 *d_F = nullptr, *d_W = nullptr, *d_tw = nullptr;
  double2 *d_Fa = nullptr, *d_Fbar = nullptr, *d_Pbar = nullptr;  // adjoint, allocated on demand
  int64_t* d_off = nullptr;
  double* d_nu = nullptr;

  GroupView view() const {
    GroupView g{};
    g.precision = precision;
    g.mb_synth = mb_synth;
    g.mb_anal = mb_anal;
    g.N = N;
    g.nlat = nlat;
    g.nh = nh;
    g.M = M;
    g.nb = (int)members.size();
    g.mu = d_mu;
    g.w = d_w;
    g.T1 = d_T1;
    g.T2 = d_T2;
    g.T1f = d_T1f;
    g.T2f = d_T2f;
    g.t2off = d_t2off;
    g.rec_a = d_rec_a;
    g.rec_g = d_rec_g;
    g.rec_p = d_rec_p;
    g.F = d_F;
    g.Fa = d_Fa;
    g.Fbar = d_Fbar;
    g.Pbar = d_Pbar;
    g.W = d_W;
    g.lps = d_lps;
    g.lpsoff = d_lpsoff;
    g.tw = d_tw;
    g.off = d_off;
    g.nu = d_nu;
    return g;
  }
  // View restricted to the i-th member of the group.
  GroupView member_view(int i) const {
    GroupView g = view();
    g.nb = 1;
    g.mb_synth = g.mb_anal = 0;
    if (d_lps) g.lps = d_lps + (int64_t)i * lps_stride;
    g.F = d_F + (int64_t)i * 4 * nlat * (N + 1);
    g.W = d_W + (int64_t)i * nlat * (N + 1);
    if (d_Fa) {
      g.Fa = d_Fa + (int64_t)i * 5 * nlat * (N + 1);
      g.Fbar = d_Fbar + (int64_t)i * 4 * nlat * (N + 1);
      g.Pbar = d_Pbar + (int64_t)i * (N + 1) * (N + 2) * 4;
    }
    g.off = d_off + i;
    g.nu = d_nu + i;
    return g;
  }
};

// A captured chunk of fixed-coefficient steps for one (history, forcing) pair.
struct GraphEntry {
  const void* hist = nullptr;
  const void* forcing = nullptr;
  // trajectory sequences (kind 1 forward, 2 adjoint): the cotangent buffer,
  // the buffer length and the range of steps captured
  int kind = 0;
  const void* aux = nullptr;
  int64_t n = 0, i0 = 0, i1 = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t used = 0;  // last use, for least-recently-used eviction
};

}  // namespace

struct nse_ctx {
  std::vector<nse_member> members;
  std::vector<int64_t> member_offset;
  std::vector<int> member_group, member_index;  // group and index within it
  nse_params params{};
  hipStream_t stream = nullptr;
  std::vector<Group> groups;
  // streams of groups 1.. (forked from `stream` for each evaluation chain) and
  // the fork / join events
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> ev_join;
  hipEvent_t ev_fork = nullptr;
  int64_t state_count = 0;
  double2* d_iter = nullptr;
  int* d_flag = nullptr;
  std::string err;
  // captured step chunks, at most kGraphCache (history, forcing) pairs
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
  // per-kernel timing: every launch is issued `profile_repeat` times between
  // one pair of events (0 = timing off)
  bool profiling = false;
  int profile_repeat = 0;
  double2* d_hist_save = nullptr;  // history copy for repeated in-place step updates
  struct Pending {
    int kind;
    int repeat;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  int64_t prof_count[NSE_KERNEL_KINDS] = {0, 0, 0};
  double prof_ms[NSE_KERNEL_KINDS] = {0, 0, 0};
  // adaptive NDF integrator: controller state (ndf_control.h) mirrored between
  // host and device, differences and sweep buffers on the device
  struct Adaptive {
    bool active = false, started = false;
    nse_adaptive_params p{};
    const double2* forcing = nullptr;
    nse_forcing_fn fn = nullptr;
    void* user = nullptr;
    nse_forcing_schedule sched{};  // device-evaluated forcing scale (no callback)
    double fnorm = 0.0;
    NdfCtl c{};  // authoritative between nse_adaptive_* calls
    int64_t waits = 0;
    double wait_seconds = 0.0;
    std::vector<nse_adaptive_record> log;
  } ad;
  NdfCtl* d_ctl = nullptr;               // device copy during device-controlled runs
  NdfCtl* h_ctl = nullptr;               // pinned staging of its copies
  nse_adaptive_record* d_log = nullptr;  // [kNdfLogCap] ring of attempt records
  unsigned long long* d_spread = nullptr;  // [2][kNdfSpreadRow] sweep norm copies (slot parity)
  hipGraph_t ad_graph = nullptr;         // captured sweep-slot sequence
  hipGraphExec_t ad_exec = nullptr;
  struct {                               // what its kernel arguments name
    const double2* forcing;
    nse_forcing_schedule sched;
    int K;
  } ad_key{};
  hipStream_t cap_stream = nullptr;      // private stream it is captured on (the
                                         // context stream may be the null stream)
  double2* d_diag = nullptr;  // inertial manifold: band-limited input, its nonlinear term
  double2* d_ndf = nullptr;  // D [depth][S], then y0, psi, y, dA, dB, n (each S)
  int ndf_depth = 0;
  unsigned long long* d_norms = nullptr;   // [4 x max sweeps] then block counters
  unsigned long long* h_pub = nullptr;     // host-mapped: norms of every sweep + sequence word
  unsigned long long* d_pub = nullptr;     // its device address
  unsigned long long pub_seq = 0;
  // device address of this device's static scratch (nse_nonlinear_adjoint_noalloc)
  double2* noalloc_scratch = nullptr;
};

namespace {

constexpr int kGraphChunk = 10;
// captured step graphs kept per context (each new history or forcing address
// captures its own; the least recently used is dropped beyond this)
constexpr size_t kGraphCache = 8;
constexpr double kPi = 3.14159265358979323846;

nse_status fail(nse_ctx* c, nse_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

thread_local std::string g_init_error;

nse_status hip_fail(nse_ctx* c, hipError_t e, const char* what) {
  return fail(c, NSE_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define NSE_HIP(ctx, call)                         \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

// Coefficients of sum_{m=1}^{q} (1/m) nabla^m y_{n+1} - kappa_q gamma_q nabla^{q+1} y_{n+1}
// (eq. (ode_disc)) as c_0..c_{len-1} of sum_j c_j y_{n+1-j}, and the
// predictor sum_{j=0}^{d} nabla^j y_n = sum_i pi_i y_{n-i} for step index k:
// start-up order q = min(p, k+1), kappa only once q+1 past states exist,
// predictor degree d = min(q, k).
void step_scheme(int p, int64_t k, std::vector<double>& c, std::vector<double>& pi) {
  const int q = (int)std::min<int64_t>(p, k + 1);
  const bool kap = (k >= q) && ndf_kappa(q) != 0.0;
  const int len = kap ? q + 2 : q + 1;
  c.assign(len, 0.0);
  for (int m = 1; m <= q; ++m)
    for (int j = 0; j <= m; ++j) c[j] += ((j & 1) ? -1.0 : 1.0) * ndf_binom(m, j) / m;
  if (kap) {
    double gamma = 0.0;
    for (int j = 1; j <= q; ++j) gamma += 1.0 / j;
    for (int j = 0; j <= q + 1; ++j)
      c[j] -= ndf_kappa(q) * gamma * ((j & 1) ? -1.0 : 1.0) * ndf_binom(q + 1, j);
  }
  const int d = (int)std::min<int64_t>(q, k);
  pi.assign(d + 1, 0.0);
  for (int j = 0; j <= d; ++j)
    for (int i = 0; i <= j; ++i) pi[i] += ((i & 1) ? -1.0 : 1.0) * ndf_binom(j, i);
}

int min_nlat(int N) { return (3 * N + 2 + 1) / 2; }


void free_group(Group& g) {
  (void)hipFree(g.d_mu);
  (void)hipFree(g.d_w);
  (void)hipFree(g.d_T1);
  (void)hipFree(g.d_T2);
  (void)hipFree(g.d_T1f);
  (void)hipFree(g.d_T2f);
  (void)hipFree(g.d_t2off);
  (void)hipFree(g.d_rec_a);
  (void)hipFree(g.d_rec_g);
  (void)hipFree(g.d_rec_p);
  (void)hipFree(g.d_lps);
  (void)hipFree(g.d_lpsoff);
  (void)hipFree(g.d_F);
  (void)hipFree(g.d_W);
  (void)hipFree(g.d_Fa);
  (void)hipFree(g.d_Fbar);
  (void)hipFree(g.d_Pbar);
  (void)hipFree(g.d_tw);
  (void)hipFree(g.d_off);
  (void)hipFree(g.d_nu);
}

void destroy_graph(GraphEntry& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
}

void drop_graphs(nse_ctx* c) {
  // a graph launched earlier may still run on the stream
  if (!c->graphs.empty() && c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& g : c->graphs) destroy_graph(g);
  c->graphs.clear();
}

template <typename T>
hipError_t dalloc(T** p, size_t count) {
  return hipMalloc((void**)p, sizeof(T) * (count ? count : 1));
}

nse_status build_group(nse_ctx* c, Group& g) {
  g.nh = (g.nlat + 1) / 2;
  g.M = 2 * g.nlat;
  gauss_legendre(g.nlat, g.mu, g.w);
  const int nb = (int)g.members.size();
  NSE_HIP(c, dalloc(&g.d_mu, g.nh));
  NSE_HIP(c, dalloc(&g.d_w, g.nh));
  NSE_HIP(c, hipMemcpy(g.d_mu, g.mu.data(), sizeof(double) * g.nh, hipMemcpyHostToDevice));
  NSE_HIP(c, hipMemcpy(g.d_w, g.w.data(), sizeof(double) * g.nh, hipMemcpyHostToDevice));
  const int64_t ts1 = t1_size(g.N, g.nh);
  g.t2off.assign(g.N + 2, 0);
  for (int m = 0; m <= g.N; ++m) {
    const int L = g.N + 2 - m;
    g.t2off[m + 1] = g.t2off[m] + (int64_t)((L + kTile - 1) / kTile) * g.nh * kTile;
  }
  const int64_t ts2 = g.t2off[g.N + 1];
  NSE_HIP(c, dalloc(&g.d_t2off, g.N + 2));
  NSE_HIP(c, hipMemcpy(g.d_t2off, g.t2off.data(), sizeof(int64_t) * (g.N + 2),
                       hipMemcpyHostToDevice));
  NSE_HIP(c, dalloc(&g.d_T1, ts1));
  NSE_HIP(c, dalloc(&g.d_T2, ts2));
  {
    // recurrence coefficients, in long double and rounded once
    const int64_t nrec = (int64_t)(g.N + 2) * (g.N + 3) / 2;
    std::vector<double2> ra(nrec), rg(nrec), rp(nrec);
    for (int m = 0; m <= g.N; ++m) {
      const long double lm = m;
      auto a_of = [&](int l) -> long double {
        const long double ll = l;
        return std::sqrt((4.0L * ll * ll - 1.0L) / (ll * ll - lm * lm));
      };
      for (int l = m; l <= g.N + 1; ++l) {
        const int64_t sl = rec_slot(g.N, l, m);
        const long double al = (l > m) ? a_of(l) : 0.0L;
        const long double ratio = (l > m + 1) ? al / a_of(l - 1) : 0.0L;
        const long double gl = (l > m) ? (2.0L * l + 1.0L) / al : 0.0L;
        const long double rs = (l > 0) ? 1.0L / std::sqrt((long double)l * (l + 1)) : 0.0L;
        ra[sl] = make_double2((double)al, (double)ratio);
        rg[sl] = make_double2((double)gl, (double)rs);
        const long double en = (l + 1 <= g.N + 1) ? 1.0L / a_of(l + 1) : 0.0L;  // e(l+1)
        const long double el = (l > m) ? 1.0L / al : 0.0L;                      // e(l)
        rp[sl] = make_double2((double)((long double)l * en), (double)((l + 1.0L) * el));
      }
    }
    NSE_HIP(c, dalloc(&g.d_rec_a, nrec));
    NSE_HIP(c, dalloc(&g.d_rec_g, nrec));
    NSE_HIP(c, dalloc(&g.d_rec_p, nrec));
    NSE_HIP(c, hipMemcpy(g.d_rec_a, ra.data(), sizeof(double2) * nrec, hipMemcpyHostToDevice));
    NSE_HIP(c, hipMemcpy(g.d_rec_g, rg.data(), sizeof(double2) * nrec, hipMemcpyHostToDevice));
    NSE_HIP(c, hipMemcpy(g.d_rec_p, rp.data(), sizeof(double2) * nrec, hipMemcpyHostToDevice));
  }
  if (c->params.precision == NSE_PREC_BF16X3) {
    // FP32 copies of the tables, split into bf16 pieces in registers (the FP64
    // and FP32 modes continue the recurrences from FP64 seed rows instead)
    NSE_HIP(c, dalloc(&g.d_T1f, ts1));
    NSE_HIP(c, dalloc(&g.d_T2f, ts2));
    // per order: ceil(L / 32) blocks x 3 pieces x 64 lanes of 4 bf16
    std::vector<int64_t> off(g.N + 2, 0);
    for (int m = 0; m <= g.N; ++m) off[m + 1] = off[m] + (int64_t)((g.N + 2 - m + 31) / 32) * 3 * 64;
    NSE_HIP(c, dalloc(&g.d_lpsoff, g.N + 2));
    NSE_HIP(c, hipMemcpy(g.d_lpsoff, off.data(), sizeof(int64_t) * (g.N + 2), hipMemcpyHostToDevice));
    g.lps_stride = off[g.N + 1];
    NSE_HIP(c, dalloc(&g.d_lps, (size_t)nb * off[g.N + 1]));
  }
  NSE_HIP(c, dalloc(&g.d_F, (size_t)nb * 4 * g.nlat * (g.N + 1)));
  NSE_HIP(c, dalloc(&g.d_W, (size_t)nb * g.nlat * (g.N + 1)));
  std::vector<double2> tw(g.M);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int k = 0; k < g.M; ++k) {
    const long double a = two_pi * k / g.M;
    tw[k] = make_double2((double)std::cos(a), (double)-std::sin(a));
  }
  NSE_HIP(c, dalloc(&g.d_tw, g.M));
  NSE_HIP(c, hipMemcpy(g.d_tw, tw.data(), sizeof(double2) * g.M, hipMemcpyHostToDevice));
  NSE_HIP(c, dalloc(&g.d_off, nb));
  NSE_HIP(c, dalloc(&g.d_nu, nb));
  NSE_HIP(c, hipMemcpy(g.d_off, g.offsets.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice));
  NSE_HIP(c, hipMemcpy(g.d_nu, g.nu.data(), sizeof(double) * nb, hipMemcpyHostToDevice));
  NSE_HIP(c, launch_legendre_table(g.view(), g.d_T1, g.d_T2, g.d_T1f, g.d_T2f, c->stream));
  return NSE_OK;
}

bool is_finite(double x) { return std::isfinite(x); }

hipError_t take_event(nse_ctx* c, hipEvent_t* e) {
  if (!c->event_pool.empty()) {
    *e = c->event_pool.back();
    c->event_pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Resolves recorded event pairs into the per-kind totals.
nse_status collect_profile(nse_ctx* c) {
  NSE_HIP(c, hipStreamSynchronize(c->stream));
  for (auto& p : c->pending) {
    float ms = 0.f;
    NSE_HIP(c, hipEventElapsedTime(&ms, p.a, p.b));
    c->prof_count[p.kind] += 1;
    c->prof_ms[p.kind] += ms / p.repeat;
    c->event_pool.push_back(p.a);
    c->event_pool.push_back(p.b);
  }
  c->pending.clear();
  return NSE_OK;
}

// Runs one launcher. When profiling, the launch is issued profile_repeat
// times back to back between two events, so that the event overhead is
// spread over the repeats (the launchers passed here are pure functions of
// their inputs, or are made so by the caller).
template <typename F>
nse_status timed_launch(nse_ctx* c, int kind, F&& launch) {
  if (!c->profiling) {
    NSE_HIP(c, launch());
    return NSE_OK;
  }
  nse_ctx::Pending p{kind, c->profile_repeat, nullptr, nullptr};
  NSE_HIP(c, take_event(c, &p.a));
  NSE_HIP(c, take_event(c, &p.b));
  NSE_HIP(c, hipEventRecord(p.a, c->stream));
  for (int r = 0; r < p.repeat; ++r) NSE_HIP(c, launch());
  NSE_HIP(c, hipEventRecord(p.b, c->stream));
  c->pending.push_back(p);
  if (c->pending.size() > 4096) return collect_profile(c);
  return NSE_OK;
}

// FP64 and FP32 contractions run on the vector units (HBM-bound table streams);
// the split-bf16 form runs on MFMA.
// Groups of several FP64 members use the member-batched MFMA products.
hipError_t launch_synth_any(const GroupView& v, const SynthInput& in, int mode, hipStream_t s) {
  if (v.precision == NSE_PREC_BF16X3) return launch_synthesis_lp(v, in, mode, v.precision, s);
  if (v.precision == NSE_PREC_FP64 && mode == SYNTH_NONLINEAR && v.mb_synth >= 2)
    return launch_synthesis_mb(v, in, v.mb_synth, s);
  return launch_synthesis(v, in, mode, s);
}

hipError_t launch_anal_any(const GroupView& v, const AnalOutput& out, hipStream_t s) {
  if (v.precision == NSE_PREC_BF16X3) return launch_analysis_lp(v, out, v.precision, s);
  if (v.precision == NSE_PREC_FP64 && v.mb_anal >= 2) return launch_analysis_mb(v, out, v.mb_anal, s);
  return launch_analysis(v, out, s);
}

bool valid_synth_block(int B) { return B == 0 || B == 2 || B == 4 || B == 8; }
bool valid_anal_block(int B) { return B == 0 || B == 2 || B == 4 || B == 8; }

// Largest power of two <= min(nb, cap) for groups of >= 2 members, else 0.
int default_block(int nb, int cap) {
  if (nb < 2) return 0;
  int B = 2;
  while (B * 2 <= nb && B * 2 <= cap) B *= 2;
  return B;
}

// Times `reps` launches of `launch` on the context stream (after one warm-up).
template <typename F>
nse_status time_launches(nse_ctx* c, int reps, F&& launch, float* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  NSE_HIP(c, hipEventCreate(&a));
  hipError_t e = hipEventCreate(&b);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(a, c->stream);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
  (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (e != hipSuccess) return hip_fail(c, e, "autotune timing");
  return NSE_OK;
}

// Picks the fastest member blocks of every FP64 group with >= 2 members by
// timing its synthesis and analysis (nonlinear mode) on a zero state.
nse_status autotune_blocks(nse_ctx* c) {
  double2* zero_state = nullptr;
  NSE_HIP(c, dalloc(&zero_state, (size_t)c->state_count));
  NSE_HIP(c, hipMemsetAsync(zero_state, 0, sizeof(double2) * c->state_count, c->stream));
  nse_status st = NSE_OK;
  for (auto& g : c->groups) {
    if (g.precision != NSE_PREC_FP64 || g.members.size() < 2 || st != NSE_OK) continue;
    SynthInput in{};
    in.nsrc = 1;
    in.src[0] = zero_state;
    in.coef[0] = 1.0;
    AnalOutput out{};
    out.mode = ANAL_NONLINEAR;
    out.n_out = c->d_iter;
    out.state_count = c->state_count;
    float best = 1e30f;
    for (int B : {0, 2, 4, 8}) {
      if (B > 2 * (int)g.members.size()) continue;
      GroupView v = g.view();
      v.mb_synth = B;
      float ms = 0.f;
      st = time_launches(c, 5, [&] { return launch_synth_any(v, in, SYNTH_NONLINEAR, c->stream); },
                         &ms);
      if (st != NSE_OK) break;
      if (ms < best) {
        best = ms;
        g.mb_synth = B;
      }
    }
    best = 1e30f;
    for (int B : {0, 2, 4, 8}) {
      if (st != NSE_OK || B > 2 * (int)g.members.size()) continue;
      GroupView v = g.view();
      v.mb_anal = B;
      float ms = 0.f;
      st = time_launches(c, 5, [&] { return launch_anal_any(v, out, c->stream); }, &ms);
      if (st != NSE_OK) break;
      if (ms < best) {
        best = ms;
        g.mb_anal = B;
      }
    }
  }
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(zero_state);
  return st;
}

// Streams and events for running the chains of several groups side by side.
nse_status ensure_aux_streams(nse_ctx* c) {
  const size_t need = c->groups.size() - 1;
  if (!c->ev_fork) NSE_HIP(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  while (c->aux.size() < need) {
    hipStream_t st = nullptr;
    NSE_HIP(c, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    c->aux.push_back(st);
    hipEvent_t e = nullptr;
    NSE_HIP(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->ev_join.push_back(e);
  }
  return NSE_OK;
}

// Enqueues one full evaluation chain (synthesis, ring, analysis) for every
// group. The groups are independent: unless kernels are being timed, group 0
// runs on the context stream and every other group on its own stream forked
// from it and joined back, so that the chains of different truncations overlap
// on the GPU (inside a captured graph the fork and the join become edges).
nse_status enqueue_chain(nse_ctx* c, const SynthInput& in, const AnalOutput& out,
                         const int* gate = nullptr, const NdfArgs* step_a = nullptr,
                         const NdfStepArgs* step = nullptr) {
  const bool fork = !c->profiling && c->groups.size() > 1;
  if (fork) {
    nse_status s = ensure_aux_streams(c);
    if (s != NSE_OK) return s;
    NSE_HIP(c, hipEventRecord(c->ev_fork, c->stream));
    for (size_t i = 0; i + 1 < c->groups.size(); ++i)
      NSE_HIP(c, hipStreamWaitEvent(c->aux[i], c->ev_fork, 0));
  }
  for (size_t gi = 0; gi < c->groups.size(); ++gi) {
    auto& g = c->groups[gi];
    GroupView v = g.view();
    v.gate = gate;
    if (fork) {
      hipStream_t st = gi ? c->aux[gi - 1] : c->stream;
      NSE_HIP(c, launch_synth_any(v, in, SYNTH_NONLINEAR, st));
      NSE_HIP(c, launch_ring(v, g.plan, SYNTH_NONLINEAR, nullptr, st));
      NSE_HIP(c, launch_anal_any(v, out, st));
      continue;
    }
    nse_status s;
    // with `step` the synthesis also runs the sweep slot's controller step and
    // decides for itself whether the slot runs (it writes the gate flag)
    GroupView vs = v;
    if (step) vs.gate = nullptr;
    s = timed_launch(c, NSE_KERNEL_SYNTHESIS, [&] {
      return step ? launch_synthesis_step(vs, in, *step_a, *step, c->stream)
                  : launch_synth_any(v, in, SYNTH_NONLINEAR, c->stream);
    });
    if (s != NSE_OK) return s;
    s = timed_launch(c, NSE_KERNEL_RING,
                     [&] { return launch_ring(v, g.plan, SYNTH_NONLINEAR, nullptr, c->stream); });
    if (s != NSE_OK) return s;
    // the final sweep of a step rotates the history in place: repeated timing
    // launches run from a saved copy, which is restored for one last launch
    const bool rotates = out.mode == ANAL_STEP_FINAL && c->profiling && c->profile_repeat > 1;
    const size_t hbytes = sizeof(double2) * (size_t)out.depth * c->state_count;
    if (rotates) {
      if (!c->d_hist_save)
        NSE_HIP(c, dalloc(&c->d_hist_save, (size_t)(c->params.order + 1) * c->state_count));
      NSE_HIP(c, hipMemcpyAsync(c->d_hist_save, out.hist, hbytes, hipMemcpyDeviceToDevice,
                                c->stream));
    }
    s = timed_launch(c, NSE_KERNEL_ANALYSIS, [&] { return launch_anal_any(v, out, c->stream); });
    if (s != NSE_OK) return s;
    if (rotates) {
      NSE_HIP(c, hipMemcpyAsync(out.hist, c->d_hist_save, hbytes, hipMemcpyDeviceToDevice,
                                c->stream));
      NSE_HIP(c, launch_anal_any(v, out, c->stream));
    }
  }
  if (fork) {
    for (size_t i = 0; i + 1 < c->groups.size(); ++i) {
      NSE_HIP(c, hipEventRecord(c->ev_join[i], c->aux[i]));
      NSE_HIP(c, hipStreamWaitEvent(c->stream, c->ev_join[i], 0));
    }
  }
  return NSE_OK;
}

// Enqueues step k (all fixed-point sweeps) on the context stream.
nse_status enqueue_step(nse_ctx* c, double2* hist, const double2* forcing, int64_t k,
                        bool shift = false) {
  std::vector<double> cc, pi;
  step_scheme(c->params.order, k, cc, pi);
  const int K = c->params.newton_iters;
  for (int it = 0; it < K; ++it) {
    SynthInput in{};
    in.coriolis = 2.0 * c->params.omega * std::sqrt(4.0 * kPi / 3.0);
    if (it == 0) {
      in.nsrc = (int)pi.size();
      for (int i = 0; i < in.nsrc; ++i) {
        in.src[i] = hist + (int64_t)i * c->state_count;
        in.coef[i] = pi[i];
      }
    } else {
      in.nsrc = 1;
      in.src[0] = c->d_iter;
      in.coef[0] = 1.0;
    }
    AnalOutput out{};
    out.mode = (it == K - 1) ? ANAL_STEP_FINAL : ANAL_STEP_ITER;
    out.hist = hist;
    out.state_count = c->state_count;
    out.depth = c->params.order + 1;
    out.ncoef = (int)cc.size();
    for (int j = 0; j < out.ncoef; ++j) out.c[j] = cc[j];
    out.h = c->params.dt;
    out.forcing = forcing;
    out.iter = c->d_iter;
    out.nonfinite = (c->params.flags & NSE_FLAG_CHECK_FINITE) ? c->d_flag : nullptr;
    out.shift = shift ? 1 : 0;
    nse_status s = enqueue_chain(c, in, out);
    if (s != NSE_OK) return s;
  }
  return NSE_OK;
}

// Buffers of the adjoint (four forward fields plus the analysis cotangent,
// the field-spectrum cotangents and the panel cotangents), allocated on the
// first adjoint call.
nse_status ensure_adjoint_buffers(nse_ctx* c) {
  for (auto& g : c->groups) {
    if (g.d_Fa) continue;
    const size_t nb = g.members.size();
    const size_t fs = (size_t)g.nlat * (g.N + 1);
    NSE_HIP(c, dalloc(&g.d_Fa, nb * 5 * fs));
    NSE_HIP(c, dalloc(&g.d_Fbar, nb * 4 * fs));
    NSE_HIP(c, dalloc(&g.d_Pbar, nb * (size_t)(g.N + 1) * (g.N + 2) * 4));
  }
  return NSE_OK;
}

// alpha_bar = J^T n_bar at the synthesis input `in` (always FP64 tables):
// recompute the forward spectra with the analysis cotangent as a fifth field,
// then the transposed ring, synthesis and prologue.
// `scratch_base` (optional): device memory of noalloc_bytes(c) bytes that holds
// the groups' Fa, Fbar and Pbar instead of the context's own buffers.
nse_status enqueue_nonlinear_adjoint(nse_ctx* c, SynthInput in, const double2* n_bar,
                                     double2* alpha_bar, double2* scratch_base = nullptr) {
  in.adj = n_bar;
  char* sp = (char*)scratch_base;
  auto carve = [&](size_t bytes) {
    double2* p = (double2*)sp;
    sp += (bytes + 255) & ~size_t(255);
    return p;
  };
  for (auto& g : c->groups) {
    GroupView v = g.view();
    if (scratch_base) {
      const size_t nb = g.members.size();
      const size_t fs = (size_t)g.nlat * (g.N + 1);
      v.Fa = carve(sizeof(double2) * nb * 5 * fs);
      v.Fbar = carve(sizeof(double2) * nb * 4 * fs);
      v.Pbar = carve(sizeof(double2) * nb * (size_t)(g.N + 1) * (g.N + 2) * 4);
    }
    NSE_HIP(c, launch_synthesis(v, in, SYNTH_ADJ, c->stream));
    NSE_HIP(c, launch_ring_adjoint(v, g.plan, c->stream));
    NSE_HIP(c, launch_synthesis_adjoint(v, c->stream));
    NSE_HIP(c, launch_prep_adjoint(v, alpha_bar, c->stream));
  }
  return NSE_OK;
}

// ---------------------------------------------------------------------------
// Adaptive NDF integrator. The controller (ndf_control.h) runs on the host when
// a forcing callback has to be called per time level, else on the device.

constexpr int kSlotsPerGraph = 16;       // sweep slots in one captured sequence (even)
constexpr int kMaxGraphsPerBatch = 32;   // sequences enqueued between two waits
static_assert(kSlotsPerGraph % 2 == 0, "slots alternate between two state buffers");

void drop_attempt_graph(nse_ctx* c);

nse_status ensure_ndf_buffers(nse_ctx* c, int depth) {
  if (c->d_ndf && c->ndf_depth == depth) return NSE_OK;
  drop_attempt_graph(c);  // names the old buffers
  (void)hipFree(c->d_ndf);
  c->d_ndf = nullptr;
  c->ndf_depth = 0;
  NSE_HIP(c, dalloc(&c->d_ndf, (size_t)(depth + 6) * c->state_count));
  c->ndf_depth = depth;
  if (!c->d_norms) {
    // norms, then kMaxNewton 32-bit workgroup counters (half as many 64-bit slots)
    NSE_HIP(c, dalloc(&c->d_norms, 4 * kMaxNewton + kMaxNewton / 2));
    NSE_HIP(c, hipHostMalloc((void**)&c->h_pub, sizeof(unsigned long long) * (4 * kMaxNewton + 1),
                             hipHostMallocMapped | hipHostMallocCoherent));
    std::memset(c->h_pub, 0, sizeof(unsigned long long) * (4 * kMaxNewton + 1));
    NSE_HIP(c, hipHostGetDevicePointer((void**)&c->d_pub, c->h_pub, 0));
  }
  if (!c->d_ctl) {
    NSE_HIP(c, hipMalloc((void**)&c->d_ctl, 2 * sizeof(NdfCtl)));  // read / written by alternate slots
    NSE_HIP(c, hipHostMalloc((void**)&c->h_ctl, sizeof(NdfCtl), hipHostMallocDefault));
    NSE_HIP(c, hipMalloc((void**)&c->d_log, sizeof(nse_adaptive_record) * kNdfLogCap));
    NSE_HIP(c, hipMalloc((void**)&c->d_spread, sizeof(unsigned long long) * 2 * kNdfSpreadRow));
  }
  return NSE_OK;
}

void drop_attempt_graph(nse_ctx* c) {
  if (c->ad_exec) (void)hipGraphExecDestroy(c->ad_exec);
  if (c->ad_graph) (void)hipGraphDestroy(c->ad_graph);
  c->ad_exec = nullptr;
  c->ad_graph = nullptr;
}

double2* ndf_buf(nse_ctx* c, int i) {  // 0 y0, 1 psi, 2 y, 3 dA, 4 dB, 5 n
  return c->d_ndf + (int64_t)(c->ndf_depth + i) * c->state_count;
}

// Norms of sweeps 0..rows-1 (square roots of the published squares), after the
// last corrector launch has published sequence number c->pub_seq: the host
// polls the sequence word in mapped memory instead of waiting for the stream;
// after two seconds of polling it waits for the stream and checks once more.
nse_status read_norms(nse_ctx* c, int rows, double out[][4]) {
  const auto t0 = std::chrono::steady_clock::now();
  volatile unsigned long long* seq = c->h_pub + 4 * kMaxNewton;
  for (uint64_t spin = 1; *seq != c->pub_seq; ++spin) {
    if ((spin & 4095) == 0 &&
        std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
      NSE_HIP(c, hipStreamSynchronize(c->stream));
      if (*seq != c->pub_seq)
        return fail(c, NSE_ERR_HIP, "corrector norms were not published (sequence %llu)",
                    (unsigned long long)c->pub_seq);
      break;
    }
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  c->ad.waits++;
  c->ad.wait_seconds +=
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  volatile unsigned long long* pub = c->h_pub;
  for (int r = 0; r < rows; ++r)
    for (int q = 0; q < 4; ++q) {
      const unsigned long long bits = pub[4 * r + q];
      double v;
      std::memcpy(&v, &bits, sizeof(double));
      out[r][q] = std::sqrt(v);
    }
  return NSE_OK;
}

NdfArgs ndf_args(nse_ctx* c) {
  NdfArgs a{};
  a.D = c->d_ndf;
  a.S = c->state_count;
  a.depth = c->ndf_depth;
  a.kmax = c->ad.p.max_order;
  const double r = c->ad.p.atol / c->ad.p.rtol;
  a.thr2 = r * r;
  a.norms = c->d_norms;
  a.nnorms = 4 * kMaxNewton;
  a.done = reinterpret_cast<unsigned int*>(c->d_norms + 4 * kMaxNewton);
  for (int j = 0; j <= kNdfMaxOrder; ++j) a.gam[j] = ndf_gamma(j);
  a.y0 = ndf_buf(c, 0);
  a.psi = ndf_buf(c, 1);
  return a;
}

// k_ndf_prepare from the prepare snapshot of the host's controller state
// (clears the sweep norms).
nse_status ndf_prepare_host(nse_ctx* c) {
  const NdfCtl& k = c->ad.c;
  NdfArgs a = ndf_args(c);
  a.accept = k.prep_accept;
  a.k_acc = k.prep_k_acc;
  a.dacc = ndf_buf(c, 3 + k.prep_dsel);
  a.transform = k.prep_transform;
  a.k = k.prep_k;
  std::memcpy(a.R, k.prepR, sizeof(a.R));
  a.predict = k.prep_predict;
  NSE_HIP(c, launch_ndf_prepare(a, c->stream));
  return NSE_OK;
}

// One nonlinear evaluation n(src) into the n buffer. `gate`: the device flag
// of a device-controlled run (null: unconditional).
nse_status ndf_eval(nse_ctx* c, const double2* src, const int* gate = nullptr) {
  SynthInput in{};
  in.nsrc = 1;
  in.src[0] = src;
  in.coef[0] = 1.0;
  in.coriolis = 2.0 * c->params.omega * std::sqrt(4.0 * kPi / 3.0);
  AnalOutput out{};
  out.mode = ANAL_NONLINEAR;
  out.n_out = ndf_buf(c, 5);
  out.state_count = c->state_count;
  return enqueue_chain(c, in, out, gate);
}

// Corrector sweep `sweep` (0-based) or the NDF_RHS evaluation. Host-controlled:
// h, k and the forcing scale from the host state, the last launch publishing the
// norms; device-controlled (ctl): those from the control block, gated by the
// sweep slot (k_ndf_decide then runs the controller).
nse_status ndf_correct(nse_ctx* c, int mode, int sweep, const double2* dprev, double2* dout,
                       const NdfCtl* ctl = nullptr) {
  const NdfCtl& k = c->ad.c;
  NdfArgs a = ndf_args(c);
  a.mode = mode;
  a.k = k.k;
  a.n = ndf_buf(c, 5);
  a.f = c->ad.forcing;
  a.fscale = k.fscale;
  a.dprev = dprev;
  a.dout = dout;
  a.yout = ndf_buf(c, 2);
  a.h = mode == NDF_RHS ? 0.0 : k.h;
  a.ak = ndf_alpha(k.k);
  // device-controlled: `sweep` is the slot parity, which selects the norm row
  a.nrow = ctl ? c->d_spread + (int64_t)sweep * kNdfSpreadRow : c->d_norms + 4 * sweep;
  a.sweep = sweep;
  a.pub = c->d_pub;
  a.ctl = ctl;
  a.dsel[0] = ndf_buf(c, 3);
  a.dsel[1] = ndf_buf(c, 4);
  if (!ctl) a.seq = ++c->pub_seq;
  for (size_t gi = 0; gi < c->groups.size(); ++gi) {
    // stream order: the last launch ends the sweep
    a.publish = !ctl && gi + 1 == c->groups.size();
    NSE_HIP(c, launch_ndf_correct(c->groups[gi].view(), a, c->stream));
  }
  return NSE_OK;
}

// The corrector can ride in the analysis epilogue (ANAL_NDF) when the context is
// one group whose analysis is k_analysis_otf.
bool ndf_fusable(const nse_ctx* c) {
  if (c->groups.size() != 1) return false;
  const Group& g = c->groups[0];
  return g.precision != NSE_PREC_BF16X3 && !(g.precision == NSE_PREC_FP64 && g.mb_anal >= 2);
}

// The chain of device-controlled sweep slot parity `sel` with the corrector in
// the analysis epilogue: the iterate y in, the correction to buffer sel (the
// previous one in 1 - sel), the norms to spread row sel, the control block
// written by the slot's k_ndf_step.
nse_status ndf_sweep_fused(nse_ctx* c, int sel, const NdfArgs* step_a = nullptr,
                           const NdfStepArgs* step = nullptr) {
  const NdfCtl* ctl = c->d_ctl + (1 - sel);
  SynthInput in{};
  in.nsrc = 1;
  in.src[0] = ndf_buf(c, 2);
  in.coef[0] = 1.0;
  in.coriolis = 2.0 * c->params.omega * std::sqrt(4.0 * kPi / 3.0);
  AnalOutput out{};
  out.mode = ANAL_NDF;
  out.state_count = c->state_count;
  out.forcing = c->ad.forcing;
  out.ctl = ctl;
  out.D = c->d_ndf;
  out.y0 = ndf_buf(c, 0);
  out.psi = ndf_buf(c, 1);
  out.dprev = ndf_buf(c, 3 + (1 - sel));
  out.dout = ndf_buf(c, 3 + sel);
  out.yout = ndf_buf(c, 2);
  out.nrow = c->d_spread + (int64_t)sel * kNdfSpreadRow;
  out.kmax = c->ad.p.max_order;
  const double r = c->ad.p.atol / c->ad.p.rtol;
  out.thr2 = r * r;
  out.Dw = c->d_ndf;
  out.dacc[0] = ndf_buf(c, 3);
  out.dacc[1] = ndf_buf(c, 4);
  out.ddepth = c->ndf_depth;
  return enqueue_chain(c, in, out, &ctl->running, step_a, step);
}

nse_status ndf_failure(nse_ctx* c, int code) {
  c->ad.active = false;
  switch (code) {
    case NDF_FAIL_CORRECTOR: return fail(c, NSE_ERR_NONFINITE, "non-finite corrector");
    case NDF_FAIL_ESTIMATE: return fail(c, NSE_ERR_NONFINITE, "non-finite error estimate");
    default: return fail(c, NSE_ERR_STATE, "step size underflow at t = %.17g", c->ad.c.t);
  }
}

// One attempt with the controller on the host (a forcing callback per time
// level): a wait for the norms after every sweep from the second on.
nse_status ndf_attempt_host(nse_ctx* c) {
  auto& ad = c->ad;
  NdfCtl& k = ad.c;
  k.fscale = ad.fn ? ad.fn(ad.user, k.t + k.h) : 1.0;
  ndf_take_prepare(k, 1);
  nse_status s = ndf_prepare_host(c);
  if (s != NSE_OK) return s;
  const int K = k.K;
  double nrm[kMaxNewton][4];
  for (int i = 1; i <= K; ++i) {
    s = ndf_eval(c, i == 1 ? ndf_buf(c, 0) : ndf_buf(c, 2));
    if (s != NSE_OK) return s;
    s = ndf_correct(c, NDF_SWEEP, i - 1, i == 1 ? nullptr : ndf_buf(c, 3 + ((i - 2) & 1)),
                    ndf_buf(c, 3 + ((i - 1) & 1)));
    if (s != NSE_OK) return s;
    if (K > 1 && i == 1) continue;  // sweep 1's norms are read with sweep 2's
    s = read_norms(c, i, nrm);
    if (s != NSE_OK) return s;
    if (K > 1 && i == 2) {
      const int r0 = ndf_after_sweep(k, nrm[0]);
      if (r0 < 0) return ndf_failure(c, -r0);
    }
    const int r = ndf_after_sweep(k, nrm[i - 1]);
    if (r < 0) return ndf_failure(c, -r);
    if (r == NDF_ENDED) {
      ad.log.push_back(k.rec);
      return NSE_OK;
    }
  }
  return fail(c, NSE_ERR_STATE, "attempt did not end after %d sweeps", K);
}

// Captures kSlotsPerGraph sweep slots of the device-controlled run. Slot j
// (parity sel = j % 2): k_ndf_step (controller state from buffer sel to 1 - sel,
// norms of the previous slot from spread row 1 - sel, this slot's row cleared,
// the prepare of a newly opened attempt), then the chain with the corrector,
// run while an attempt is open. Every slot is a sweep while the run lasts.
nse_status capture_attempt_graph(nse_ctx* c) {
  if (!c->cap_stream) NSE_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  const hipStream_t user_stream = c->stream;
  c->stream = c->cap_stream;
  struct Restore {
    nse_ctx* c;
    hipStream_t s;
    ~Restore() { c->stream = s; }
  } restore{c, user_stream};
  NSE_HIP(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  nse_status s = NSE_OK;
  const bool fused = ndf_fusable(c);
  // the synthesis takes over the step kernel (one launch fewer per sweep) when
  // it is the single-latitude FP64 kernel and its launch is resident at once
  const bool in_synth = fused && synthesis_takes_step(c->groups[0].view());
  for (int j = 0; j < kSlotsPerGraph && s == NSE_OK; ++j) {
    const int sel = j & 1;
    NdfArgs a = ndf_args(c);
    a.yout = ndf_buf(c, 2);
    a.dsel[0] = ndf_buf(c, 3);
    a.dsel[1] = ndf_buf(c, 4);
    a.spread_words = kNdfSpreadRow;
    NdfStepArgs st{};
    st.ctl_in = c->d_ctl + sel;
    st.ctl_out = c->d_ctl + (1 - sel);
    st.spread_in = c->d_spread + (int64_t)(1 - sel) * kNdfSpreadRow;
    st.spread_clear = c->d_spread + (int64_t)sel * kNdfSpreadRow;
    st.sel = sel;
    st.log = c->d_log;
    st.sched = c->ad.sched;
    if (in_synth) {
      s = ndf_sweep_fused(c, sel, &a, &st);
      continue;
    }
    const hipError_t e = launch_ndf_step(a, st, c->stream);
    if (e != hipSuccess) {
      s = hip_fail(c, e, "launch_ndf_step");
      break;
    }
    if (fused) {
      s = ndf_sweep_fused(c, sel);
    } else {
      const NdfCtl* ctl = c->d_ctl + (1 - sel);
      s = ndf_eval(c, ndf_buf(c, 2), &ctl->running);
      if (s == NSE_OK)
        s = ndf_correct(c, NDF_SWEEP, sel, ndf_buf(c, 3 + (1 - sel)), ndf_buf(c, 3 + sel), ctl);
    }
  }
  hipGraph_t gr = nullptr;
  const hipError_t e = hipStreamEndCapture(c->stream, &gr);
  if (s != NSE_OK) {
    if (gr) (void)hipGraphDestroy(gr);
    return s;
  }
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(gr);
    return hip_fail(c, ei, "hipGraphInstantiate");
  }
  c->ad_graph = gr;
  c->ad_exec = ex;
  c->ad_key.forcing = c->ad.forcing;
  c->ad_key.sched = c->ad.sched;
  c->ad_key.K = c->ad.c.K;
  return NSE_OK;
}

// Advances with the controller on the device: the host state goes to the
// device, batches of captured attempt sequences run (the attempts after the
// end do nothing), and the state and the new attempt records come back after
// each batch.
nse_status advance_device(nse_ctx* c) {
  auto& ad = c->ad;
  NdfCtl& k = ad.c;
  if (!c->ad_exec) {
    nse_status s = capture_attempt_graph(c);
    if (s != NSE_OK) return s;
  }
  ndf_open_attempt(k, ad.sched);  // the first attempt; the device opens the others
  if (k.status) return ndf_failure(c, k.status);
  if (k.done) return NSE_OK;
  k.fresh = 1;  // the first slot's step kernel prepares it
  *c->h_ctl = k;
  NSE_HIP(c, hipMemcpyAsync(c->d_ctl, c->h_ctl, sizeof(NdfCtl), hipMemcpyHostToDevice, c->stream));
  long long read = k.nlog;
  std::vector<nse_adaptive_record> recs;
  for (;;) {
    // enough sweeps for the remaining interval at the current step and the mean
    // sweeps per attempt so far, plus a margin for rejections; the slots after
    // the end find no open attempt
    const double attempts = std::max<double>(1.0, (double)(k.nlog > 0 ? k.nlog : 1));
    const double per = k.nlog > 0 ? (double)(k.evaluations - 1) / attempts : (double)k.K;
    const double need = ((k.t_end - k.t) / k.h * 1.1 + 1.0) * std::max(1.0, per);
    int graphs = (int)std::min<double>(kMaxGraphsPerBatch, std::ceil(need / kSlotsPerGraph));
    graphs = std::max(graphs, 1);
    for (int i = 0; i < graphs; ++i) NSE_HIP(c, hipGraphLaunch(c->ad_exec, c->stream));
    NSE_HIP(c, hipMemcpyAsync(c->h_ctl, c->d_ctl, sizeof(NdfCtl), hipMemcpyDeviceToHost,
                              c->stream));
    const auto t0 = std::chrono::steady_clock::now();
    NSE_HIP(c, hipStreamSynchronize(c->stream));
    ad.waits++;
    ad.wait_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    k = *c->h_ctl;
    const long long fresh = k.nlog - read;
    if (fresh > kNdfLogCap) return fail(c, NSE_ERR_STATE, "attempt log overflow");
    if (fresh > 0) {
      recs.resize((size_t)fresh);
      const long long first = read % kNdfLogCap;
      const long long n1 = std::min<long long>(fresh, kNdfLogCap - first);
      NSE_HIP(c, hipMemcpy(recs.data(), c->d_log + first, sizeof(nse_adaptive_record) * n1,
                           hipMemcpyDeviceToHost));
      if (fresh > n1)
        NSE_HIP(c, hipMemcpy(recs.data() + n1, c->d_log,
                             sizeof(nse_adaptive_record) * (fresh - n1), hipMemcpyDeviceToHost));
      ad.log.insert(ad.log.end(), recs.begin(), recs.end());
      read = k.nlog;
    }
    if (k.status) return ndf_failure(c, k.status);
    if (k.done) return NSE_OK;
  }
}

}  // namespace

extern "C" {

const char* nse_status_string(nse_status s) {
  switch (s) {
    case NSE_OK: return "NSE_OK";
    case NSE_ERR_ARG: return "NSE_ERR_ARG: invalid argument";
    case NSE_ERR_ALLOC: return "NSE_ERR_ALLOC: allocation failed";
    case NSE_ERR_HIP: return "NSE_ERR_HIP: HIP runtime error";
    case NSE_ERR_UNSUPPORTED: return "NSE_ERR_UNSUPPORTED: not supported by this build";
    case NSE_ERR_NONFINITE: return "NSE_ERR_NONFINITE: NaN or Inf in the state";
    case NSE_ERR_STATE: return "NSE_ERR_STATE: invalid context state";
  }
  return "unknown nse_status";
}

const char* nse_last_error(const nse_ctx* ctx) {
  if (!ctx) return g_init_error.c_str();
  return ctx->err.c_str();
}

int64_t nse_coeff_count(int32_t N) {
  if (N < 0) return -1;
  return (int64_t)(N + 1) * (N + 2) / 2;
}

int64_t nse_state_count(const nse_ctx* ctx) { return ctx ? ctx->state_count : -1; }

namespace {

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double2* g_scratch_ptr[kMaxDevices] = {};

// Device address of the static scratch on the current device, looked up once
// per device (with that device current) and kept for the process.
static nse_status bind_noalloc_scratch(nse_ctx* c) {
  int dev = -1;
  NSE_HIP(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(c, NSE_ERR_UNSUPPORTED, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    NSE_HIP(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(c, NSE_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch");
    g_scratch_ptr[dev] = (double2*)p;
  }
  c->noalloc_scratch = g_scratch_ptr[dev];
  return NSE_OK;
}

// Bytes of adjoint intermediates (Fa, Fbar, Pbar of every group) carved from the
// static scratch, each piece 256-byte aligned.
static size_t noalloc_bytes(const nse_ctx* c) {
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  size_t total = 0;
  for (const auto& g : c->groups) {
    const size_t nb = g.members.size();
    const size_t fs = (size_t)g.nlat * (g.N + 1);
    total += up(sizeof(double2) * nb * 5 * fs) + up(sizeof(double2) * nb * 4 * fs) +
             up(sizeof(double2) * nb * (size_t)(g.N + 1) * (g.N + 2) * 4);
  }
  return total;
}

}  // namespace

nse_status nse_sphere_init(const nse_member* members, int32_t n_members, const nse_params* params,
                           void* hip_stream, nse_ctx** out) {
  g_init_error.clear();
  auto init_fail = [&](nse_status s, const std::string& msg) {
    g_init_error = msg;
    return s;
  };
  if (!out) return init_fail(NSE_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!members || n_members < 1) return init_fail(NSE_ERR_ARG, "need at least one member");
  if (!params) return init_fail(NSE_ERR_ARG, "params is NULL");
  const nse_params& P = *params;
  if (P.order < 1 || P.order > 5) return init_fail(NSE_ERR_ARG, "order must be 1..5");
  if (P.newton_iters < 1 || P.newton_iters > 1000)
    return init_fail(NSE_ERR_ARG, "newton_iters must be 1..1000");
  if (P.precision != NSE_PREC_FP64 && P.precision != NSE_PREC_FP32 &&
      P.precision != NSE_PREC_BF16X3)
    return init_fail(NSE_ERR_ARG, "unknown precision");
  if (P.flags & ~(uint32_t)(NSE_FLAG_GRAPH | NSE_FLAG_AUTOTUNE | NSE_FLAG_CHECK_FINITE))
    return init_fail(NSE_ERR_ARG, "unknown flag bits");
  if (!is_finite(P.omega)) return init_fail(NSE_ERR_ARG, "omega must be finite");
  if (!is_finite(P.dt) || !(P.dt > 0.0)) return init_fail(NSE_ERR_ARG, "dt must be finite and > 0");

  std::vector<nse_member> mem(members, members + n_members);
  for (int i = 0; i < n_members; ++i) {
    nse_member& m = mem[i];
    char buf[256];
    if (m.N < 1) {
      snprintf(buf, sizeof buf, "member %d: N must be >= 1", i);
      return init_fail(NSE_ERR_ARG, buf);
    }
    if (!is_finite(m.nu) || m.nu < 0.0) {
      snprintf(buf, sizeof buf, "member %d: nu must be finite and >= 0", i);
      return init_fail(NSE_ERR_ARG, buf);
    }
    if (m.nlat < 0) {
      snprintf(buf, sizeof buf, "member %d: nlat must be >= 0", i);
      return init_fail(NSE_ERR_ARG, buf);
    }
    FftPlan plan{};
    if (m.nlat == 0) {
      int nl = min_nlat(m.N);
      while (2 * nl <= kMaxM && !fft_factor(2 * nl, plan)) ++nl;
      m.nlat = nl;
    } else if (2 * (int64_t)m.nlat < 3 * (int64_t)m.N + 2) {
      snprintf(buf, sizeof buf,
               "member %d: M = 2*nlat = %d < 3N+2 = %d aliases the nonlinear term", i,
               2 * m.nlat, 3 * m.N + 2);
      return init_fail(NSE_ERR_ARG, buf);
    }
    if (2 * (int64_t)m.nlat > kMaxM || !fft_factor(2 * m.nlat, plan)) {
      snprintf(buf, sizeof buf,
               "member %d: M = %d must be <= %d and factor into 2, 3 and 5", i, 2 * m.nlat, kMaxM);
      return init_fail(NSE_ERR_UNSUPPORTED, buf);
    }
    if (synthesis_lds_bytes(m.N, 5) > 65536 || synthesis_lds_bytes(m.N, 4) > 65536 || ring_lds_bytes(2 * m.nlat) > 65536 ||
        synthesis_adjoint_lds_bytes((m.nlat + 1) / 2) > 65536 ||
        analysis_otf_lds_bytes((m.nlat + 1) / 2) > 65536 || synthesis_lp_lds_bytes(m.N) > 65536 ||
        split_panel_lp_lds_bytes(m.N) > 65536 ||
        analysis_lp_lds_bytes((m.nlat + 1) / 2) > 65536) {
      snprintf(buf, sizeof buf, "member %d: N = %d exceeds the largest supported truncation", i,
               m.N);
      return init_fail(NSE_ERR_UNSUPPORTED, buf);
    }
  }

  std::unique_ptr<nse_ctx> c(new (std::nothrow) nse_ctx);
  if (!c) return init_fail(NSE_ERR_ALLOC, "host allocation failed");
  c->members = mem;
  c->params = P;
  c->stream = (hipStream_t)hip_stream;
  c->member_offset.resize(n_members);
  c->member_group.resize(n_members);
  c->member_index.resize(n_members);
  int64_t off = 0;
  for (int i = 0; i < n_members; ++i) {
    c->member_offset[i] = off;
    off += nse_coeff_count(mem[i].N);
    int gi = -1;
    for (size_t j = 0; j < c->groups.size(); ++j)
      if (c->groups[j].N == mem[i].N && c->groups[j].nlat == mem[i].nlat) gi = (int)j;
    if (gi < 0) {
      Group g;
      g.precision = P.precision;
      g.N = mem[i].N;
      g.nlat = mem[i].nlat;
      fft_factor(2 * g.nlat, g.plan);
      c->groups.push_back(g);
      gi = (int)c->groups.size() - 1;
    }
    c->member_group[i] = gi;
    c->member_index[i] = (int)c->groups[gi].members.size();
    c->groups[gi].members.push_back(i);
    c->groups[gi].offsets.push_back(c->member_offset[i]);
    c->groups[gi].nu.push_back(mem[i].nu);
  }
  c->state_count = off;
  for (auto& g : c->groups) {
    if (g.precision != NSE_PREC_FP64) continue;
    g.mb_synth = default_block((int)g.members.size(), 4);
    g.mb_anal = default_block((int)g.members.size(), 8);
  }

  auto cleanup = [&](nse_status s) {
    for (auto& g : c->groups) free_group(g);
    (void)hipFree(c->d_iter);
    (void)hipFree(c->d_flag);
    g_init_error = c->err;
    return s;
  };
  for (auto& g : c->groups) {
    nse_status s = build_group(c.get(), g);
    if (s != NSE_OK) return cleanup(s);
  }
  hipError_t e = dalloc(&c->d_iter, (size_t)c->state_count);
  if (e == hipSuccess) e = dalloc(&c->d_flag, 1);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return cleanup(hip_fail(c.get(), e, "init"));
  {
    nse_status s = bind_noalloc_scratch(c.get());
    if (s != NSE_OK) return cleanup(s);
  }
  if (P.flags & NSE_FLAG_AUTOTUNE) {
    nse_status s = autotune_blocks(c.get());
    if (s != NSE_OK) return cleanup(s);
  }
  *out = c.release();
  return NSE_OK;
}

nse_status nse_sphere_destroy(nse_ctx* ctx) {
  if (!ctx) return NSE_OK;
  (void)hipStreamSynchronize(ctx->stream);
  drop_graphs(ctx);
  for (auto& p : ctx->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  for (auto st : ctx->aux) (void)hipStreamDestroy(st);
  for (auto e : ctx->ev_join) (void)hipEventDestroy(e);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  for (auto& g : ctx->groups) free_group(g);
  (void)hipFree(ctx->d_iter);
  (void)hipFree(ctx->d_flag);
  (void)hipFree(ctx->d_hist_save);
  (void)hipFree(ctx->d_ndf);
  (void)hipFree(ctx->d_diag);
  (void)hipFree(ctx->d_norms);
  if (ctx->h_pub) (void)hipHostFree(ctx->h_pub);
  drop_attempt_graph(ctx);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  (void)hipFree(ctx->d_ctl);
  (void)hipFree(ctx->d_log);
  (void)hipFree(ctx->d_spread);
  if (ctx->h_ctl) (void)hipHostFree(ctx->h_ctl);
  delete ctx;
  return NSE_OK;
}

nse_status nse_get_member_blocks(const nse_ctx* ctx, int32_t member, int32_t* synth_block,
                                 int32_t* anal_block) {
  if (!ctx) return NSE_ERR_ARG;
  nse_ctx* c = const_cast<nse_ctx*>(ctx);
  if (member < 0 || member >= (int)ctx->members.size())
    return fail(c, NSE_ERR_ARG, "member %d out of range", member);
  const Group& g = ctx->groups[ctx->member_group[member]];
  if (synth_block) *synth_block = g.mb_synth;
  if (anal_block) *anal_block = g.mb_anal;
  return NSE_OK;
}

nse_status nse_set_member_blocks(nse_ctx* ctx, int32_t member, int32_t synth_block,
                                 int32_t anal_block) {
  if (!ctx) return NSE_ERR_ARG;
  if (member < 0 || member >= (int)ctx->members.size())
    return fail(ctx, NSE_ERR_ARG, "member %d out of range", member);
  if (!valid_synth_block(synth_block) || !valid_anal_block(anal_block))
    return fail(ctx, NSE_ERR_ARG, "member blocks (%d, %d): both take 0, 2, 4 or 8", synth_block,
                anal_block);
  Group& g = ctx->groups[ctx->member_group[member]];
  if ((synth_block || anal_block) && (g.members.size() < 2 || g.precision != NSE_PREC_FP64))
    return fail(ctx, NSE_ERR_ARG, "member blocks need an FP64 group of at least two members");
  g.mb_synth = synth_block;
  g.mb_anal = anal_block;
  drop_graphs(ctx);
  return NSE_OK;
}

nse_status nse_set_stream(nse_ctx* ctx, void* hip_stream) {
  if (!ctx) return NSE_ERR_ARG;
  drop_graphs(ctx);
  ctx->stream = (hipStream_t)hip_stream;
  return NSE_OK;
}

nse_status nse_member_grid(const nse_ctx* ctx, int32_t member, int32_t* nlat, double* mu_host,
                           double* w_host) {
  if (!ctx) return NSE_ERR_ARG;
  nse_ctx* c = const_cast<nse_ctx*>(ctx);
  if (member < 0 || member >= (int)ctx->members.size())
    return fail(c, NSE_ERR_ARG, "member %d out of range", member);
  const Group& g = ctx->groups[ctx->member_group[member]];
  if (nlat) *nlat = g.nlat;
  if (mu_host) std::memcpy(mu_host, g.mu.data(), sizeof(double) * g.nlat);
  if (w_host) std::memcpy(w_host, g.w.data(), sizeof(double) * g.nlat);
  return NSE_OK;
}

nse_status nse_nonlinear(nse_ctx* ctx, const double* alpha, double* n_out) {
  if (!ctx) return NSE_ERR_ARG;
  if (!alpha || !n_out) return fail(ctx, NSE_ERR_ARG, "alpha and n_out must be non-NULL");
  if (alpha == n_out) return fail(ctx, NSE_ERR_ARG, "alpha and n_out may not alias");
  SynthInput in{};
  in.nsrc = 1;
  in.src[0] = (const double2*)alpha;
  in.coef[0] = 1.0;
  in.coriolis = 2.0 * ctx->params.omega * std::sqrt(4.0 * kPi / 3.0);
  AnalOutput out{};
  out.mode = ANAL_NONLINEAR;
  out.n_out = (double2*)n_out;
  out.state_count = ctx->state_count;
  return enqueue_chain(ctx, in, out);
}

namespace {

// The executable graph of kGraphChunk fixed-coefficient steps (global index
// k > order) on (h, f), captured on first use; the least recently used entry is
// dropped once kGraphCache pairs are held.
static nse_status step_graph(nse_ctx* ctx, double2* h, const double2* f, int64_t k,
                             hipGraphExec_t* out) {
  for (auto& g : ctx->graphs) {
    if (g.kind == 0 && g.hist == (const void*)h && g.forcing == (const void*)f) {
      g.used = ++ctx->graph_clock;
      *out = g.exec;
      return NSE_OK;
    }
  }
  if (ctx->graphs.size() >= kGraphCache) {
    auto lru = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                [](const GraphEntry& a, const GraphEntry& b) { return a.used < b.used; });
    // its last launch may still run on the stream
    NSE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    destroy_graph(*lru);
    ctx->graphs.erase(lru);
  }
  GraphEntry ge;
  ge.hist = h;
  ge.forcing = f;
  NSE_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  nse_status s = NSE_OK;
  for (int i = 0; i < kGraphChunk && s == NSE_OK; ++i) s = enqueue_step(ctx, h, f, k + i);
  hipGraph_t gr = nullptr;
  hipError_t e = hipStreamEndCapture(ctx->stream, &gr);
  if (s != NSE_OK) {
    if (gr) (void)hipGraphDestroy(gr);
    return s;
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
  ge.graph = gr;
  e = hipGraphInstantiate(&ge.exec, gr, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(gr);
    return hip_fail(ctx, e, "hipGraphInstantiate");
  }
  ge.used = ++ctx->graph_clock;
  ctx->graphs.push_back(ge);
  *out = ge.exec;
  return NSE_OK;
}

}  // namespace

nse_status nse_step(nse_ctx* ctx, double* hist, const double* forcing, int64_t step0,
                    int32_t nsteps) {
  if (!ctx) return NSE_ERR_ARG;
  if (!hist) return fail(ctx, NSE_ERR_ARG, "hist must be non-NULL");
  if (step0 < 0) return fail(ctx, NSE_ERR_ARG, "step0 must be >= 0");
  if (nsteps < 0) return fail(ctx, NSE_ERR_ARG, "nsteps must be >= 0");
  double2* h = (double2*)hist;
  const double2* f = (const double2*)forcing;
  const int p = ctx->params.order;
  int64_t k = step0;
  const int64_t end = step0 + nsteps;
  // start-up steps use their own coefficients; from k = p+1 on the step is fixed
  for (; k < end && k <= p; ++k) {
    nse_status s = enqueue_step(ctx, h, f, k);
    if (s != NSE_OK) return s;
  }
  const bool graph =
      (ctx->params.flags & NSE_FLAG_GRAPH) && ctx->stream != nullptr && !ctx->profiling;
  if (graph && k < end) {
    // the first call that reaches the fixed-coefficient steps captures the chunk
    // graph even when fewer than a chunk of steps remain, so that the capture
    // cost falls on that call and not on the later calls that replay it
    hipGraphExec_t exec = nullptr;
    nse_status s = step_graph(ctx, h, f, k, &exec);
    if (s != NSE_OK) return s;
    for (; end - k >= kGraphChunk; k += kGraphChunk)
      NSE_HIP(ctx, hipGraphLaunch(exec, ctx->stream));
  }
  for (; k < end; ++k) {
    nse_status s = enqueue_step(ctx, h, f, k);
    if (s != NSE_OK) return s;
  }
  return NSE_OK;
}

nse_status nse_nonlinear_adjoint(nse_ctx* ctx, const double* alpha, const double* n_bar,
                                 double* alpha_bar) {
  if (!ctx) return NSE_ERR_ARG;
  if (!alpha || !n_bar || !alpha_bar) return fail(ctx, NSE_ERR_ARG, "NULL array");
  if (alpha_bar == alpha || alpha_bar == n_bar)
    return fail(ctx, NSE_ERR_ARG, "alpha_bar may not alias alpha or n_bar");
  nse_status s = ensure_adjoint_buffers(ctx);
  if (s != NSE_OK) return s;
  SynthInput in{};
  in.nsrc = 1;
  in.src[0] = (const double2*)alpha;
  in.coef[0] = 1.0;
  in.coriolis = 2.0 * ctx->params.omega * std::sqrt(4.0 * kPi / 3.0);
  return enqueue_nonlinear_adjoint(ctx, in, (const double2*)n_bar, (double2*)alpha_bar);
}

nse_status nse_nonlinear_adjoint_noalloc(nse_ctx* ctx, const double* alpha, const double* n_bar,
                                         double* alpha_bar) {
  if (!ctx) return NSE_ERR_ARG;
  if (!alpha || !n_bar || !alpha_bar) return fail(ctx, NSE_ERR_ARG, "NULL array");
  if (alpha_bar == alpha || alpha_bar == n_bar)
    return fail(ctx, NSE_ERR_ARG, "alpha_bar may not alias alpha or n_bar");
  const size_t need = noalloc_bytes(ctx);
  if (need > kNoAllocScratchBytes)
    return fail(ctx, NSE_ERR_ARG,
                "the context needs %zu bytes of adjoint scratch; the static scratch holds %zu "
                "(use nse_nonlinear_adjoint)",
                need, kNoAllocScratchBytes);
  if (!ctx->noalloc_scratch) return fail(ctx, NSE_ERR_STATE, "static scratch not bound");
  SynthInput in{};
  in.nsrc = 1;
  in.src[0] = (const double2*)alpha;
  in.coef[0] = 1.0;
  in.coriolis = 2.0 * ctx->params.omega * std::sqrt(4.0 * kPi / 3.0);
  return enqueue_nonlinear_adjoint(ctx, in, (const double2*)n_bar, (double2*)alpha_bar,
                                   ctx->noalloc_scratch);
}

extern "C++" {
namespace {

// The adjoints (one fixed-point sweep each) of steps i_hi - 1 down to i_lo of
// a trajectory buffer, step i at history tr + (n - i) S and absolute index
// step0 + i, accumulating into hb.
nse_status enqueue_adjoint_sweep(nse_ctx* ctx, const double2* tr, int64_t n, int64_t step0,
                                 int64_t i_hi, int64_t i_lo, double2* hb) {
  const int64_t S = ctx->state_count;
  for (int64_t i = i_hi - 1; i >= i_lo; --i) {
    std::vector<double> cc, pi;
    step_scheme(ctx->params.order, step0 + i, cc, pi);
    const double2* hist = tr + (n - i) * S;
    SynthInput in{};
    in.nsrc = (int)pi.size();
    for (int j = 0; j < in.nsrc; ++j) {
      in.src[j] = hist + (int64_t)j * S;
      in.coef[j] = pi[j];
    }
    in.coriolis = 2.0 * ctx->params.omega * std::sqrt(4.0 * kPi / 3.0);
    in.adj = hb;      // hbar_out[0]; n_bar is formed inside the five-field synthesis
    in.adj_step = 1;
    in.adj_c0 = cc[0];
    in.adj_h = ctx->params.dt;
    StepAdjointArgs a{};
    a.hin = hb;
    a.hout = hb;
    a.state_count = S;
    a.depth = ctx->params.order + 1;
    a.ncoef = (int)cc.size();
    for (int j = 0; j < a.ncoef; ++j) a.c[j] = cc[j];
    a.npi = (int)pi.size();
    for (int j = 0; j < a.npi; ++j) a.pi[j] = pi[j];
    a.h = ctx->params.dt;
    for (auto& g : ctx->groups) {
      const GroupView v = g.view();
      NSE_HIP(ctx, launch_synthesis(v, in, SYNTH_ADJ, ctx->stream));
      NSE_HIP(ctx, launch_ring_adjoint(v, g.plan, ctx->stream));
      NSE_HIP(ctx, launch_synthesis_adjoint(v, ctx->stream));
      NSE_HIP(ctx, launch_prep_step_adjoint(v, a, ctx->stream));
    }
  }
  return NSE_OK;
}

// Runs `enqueue` (the steps i0 .. i1 - 1 of a trajectory sequence) from a
// captured graph kept under (kind, traj, aux, forcing, n, i0, i1); captured on
// the context's private stream (the context stream may be the null stream).
template <typename F>
nse_status run_sequence_graph(nse_ctx* ctx, int kind, const void* traj, const void* aux,
                                     const void* forcing, int64_t n, int64_t i0, int64_t i1,
                                     F&& enqueue) {
  for (auto& g : ctx->graphs) {
    if (g.kind == kind && g.hist == traj && g.aux == aux && g.forcing == forcing && g.n == n &&
        g.i0 == i0 && g.i1 == i1) {
      g.used = ++ctx->graph_clock;
      NSE_HIP(ctx, hipGraphLaunch(g.exec, ctx->stream));
      return NSE_OK;
    }
  }
  if (ctx->graphs.size() >= kGraphCache) {
    auto lru = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                [](const GraphEntry& a, const GraphEntry& b) { return a.used < b.used; });
    NSE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    destroy_graph(*lru);
    ctx->graphs.erase(lru);
  }
  if (!ctx->cap_stream)
    NSE_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  GraphEntry ge;
  ge.kind = kind;
  ge.hist = traj;
  ge.aux = aux;
  ge.forcing = forcing;
  ge.n = n;
  ge.i0 = i0;
  ge.i1 = i1;
  const hipStream_t user_stream = ctx->stream;
  ctx->stream = ctx->cap_stream;
  nse_status s = NSE_OK;
  hipGraph_t gr = nullptr;
  hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    s = enqueue();
    e = hipStreamEndCapture(ctx->stream, &gr);
  }
  ctx->stream = user_stream;
  if (s != NSE_OK) {
    if (gr) (void)hipGraphDestroy(gr);
    return s;
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "graph capture of a trajectory sequence");
  ge.graph = gr;
  e = hipGraphInstantiate(&ge.exec, gr, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(gr);
    return hip_fail(ctx, e, "hipGraphInstantiate");
  }
  ge.used = ++ctx->graph_clock;
  ctx->graphs.push_back(ge);
  NSE_HIP(ctx, hipGraphLaunch(ge.exec, ctx->stream));
  return NSE_OK;
}

}  // namespace
}  // extern "C++"

nse_status nse_step_adjoint(nse_ctx* ctx, const double* hist, const double* forcing, int64_t step,
                            double* hist_bar) {
  if (!ctx) return NSE_ERR_ARG;
  (void)forcing;  // the forcing enters affinely and is not differentiated
  if (!hist || !hist_bar) return fail(ctx, NSE_ERR_ARG, "NULL array");
  if (hist == hist_bar) return fail(ctx, NSE_ERR_ARG, "hist and hist_bar may not alias");
  if (step < 0) return fail(ctx, NSE_ERR_ARG, "step must be >= 0");
  if (ctx->params.newton_iters != 1)
    return fail(ctx, NSE_ERR_UNSUPPORTED, "the step adjoint needs newton_iters == 1");
  nse_status s = ensure_adjoint_buffers(ctx);
  if (s != NSE_OK) return s;
  // a sweep of one step (i = 0) over a buffer whose history slot n - i = 0 is hist
  return enqueue_adjoint_sweep(ctx, (const double2*)hist, 0, step, 1, 0, (double2*)hist_bar);
}

nse_status nse_step_trajectory(nse_ctx* ctx, double* traj, const double* forcing, int64_t step0,
                               int32_t nsteps) {
  if (!ctx) return NSE_ERR_ARG;
  if (!traj) return fail(ctx, NSE_ERR_ARG, "traj must be non-NULL");
  if (step0 < 0) return fail(ctx, NSE_ERR_ARG, "step0 must be >= 0");
  if (nsteps < 0) return fail(ctx, NSE_ERR_ARG, "nsteps must be >= 0");
  const int64_t S = ctx->state_count, n = nsteps;
  double2* tr = (double2*)traj;
  const double2* f = (const double2*)forcing;
  const int p = ctx->params.order;
  // step i reads the history at traj[n - i] and writes traj[n - i - 1]
  int64_t i = 0;
  for (; i < n && step0 + i <= p; ++i) {
    nse_status s = enqueue_step(ctx, tr + (n - i) * S, f, step0 + i, true);
    if (s != NSE_OK) return s;
  }
  if (i == n) return NSE_OK;
  const bool graph =
      (ctx->params.flags & NSE_FLAG_GRAPH) && !ctx->profiling && n - i >= 2;
  const int64_t i0 = i;
  const auto body = [&]() -> nse_status {
    for (int64_t j = i0; j < n; ++j) {
      nse_status s = enqueue_step(ctx, tr + (n - j) * S, f, step0 + j, true);
      if (s != NSE_OK) return s;
    }
    return NSE_OK;
  };
  if (!graph) return body();
  return run_sequence_graph(ctx, 1, traj, nullptr, forcing, n, i0, n, body);
}

nse_status nse_step_adjoint_trajectory(nse_ctx* ctx, const double* traj, const double* forcing,
                                       int64_t step0, int32_t nsteps, double* hist_bar) {
  if (!ctx) return NSE_ERR_ARG;
  (void)forcing;  // the forcing enters affinely and is not differentiated
  if (!traj || !hist_bar) return fail(ctx, NSE_ERR_ARG, "NULL array");
  if (step0 < 0) return fail(ctx, NSE_ERR_ARG, "step0 must be >= 0");
  if (nsteps < 0) return fail(ctx, NSE_ERR_ARG, "nsteps must be >= 0");
  if (ctx->params.newton_iters != 1)
    return fail(ctx, NSE_ERR_UNSUPPORTED, "the step adjoint needs newton_iters == 1");
  const int64_t S = ctx->state_count, n = nsteps;
  const double2* tr = (const double2*)traj;
  double2* hb = (double2*)hist_bar;
  if (hb + (ctx->params.order + 1) * S > tr && tr + (n + ctx->params.order + 1) * S > hb)
    return fail(ctx, NSE_ERR_ARG, "hist_bar may not overlap traj");
  nse_status s = ensure_adjoint_buffers(ctx);
  if (s != NSE_OK) return s;
  const int p = ctx->params.order;
  // steps n - 1 .. 0; those with fixed coefficients (step0 + i > p) first
  const int64_t ifix = std::max<int64_t>(0, std::min<int64_t>(n, p + 1 - step0));
  const auto body = [&]() -> nse_status {
    return enqueue_adjoint_sweep(ctx, tr, n, step0, n, ifix, hb);
  };
  const bool graph =
      (ctx->params.flags & NSE_FLAG_GRAPH) && !ctx->profiling && n - ifix >= 2;
  s = graph ? run_sequence_graph(ctx, 2, traj, hist_bar, forcing, n, ifix, n, body) : body();
  if (s != NSE_OK) return s;
  return enqueue_adjoint_sweep(ctx, tr, n, step0, ifix, 0, hb);
}

nse_status nse_synthesize(nse_ctx* ctx, const double* alpha, double* grid_out) {
  if (!ctx) return NSE_ERR_ARG;
  if (!alpha || !grid_out) return fail(ctx, NSE_ERR_ARG, "NULL array");
  SynthInput in{};
  in.nsrc = 1;
  in.src[0] = (const double2*)alpha;
  in.coef[0] = 1.0;
  int64_t goff = 0;
  for (size_t i = 0; i < ctx->members.size(); ++i) {
    const Group& g = ctx->groups[ctx->member_group[i]];
    const GroupView v = g.member_view(ctx->member_index[i]);
    NSE_HIP(ctx, launch_synth_any(v, in, SYNTH_GRID, ctx->stream));
    NSE_HIP(ctx, launch_ring(v, g.plan, SYNTH_GRID, grid_out + goff, ctx->stream));
    goff += (int64_t)3 * g.nlat * g.M;
  }
  return NSE_OK;
}

nse_status nse_analyze_velocity(nse_ctx* ctx, const double* u_grid, double* alpha_out) {
  if (!ctx) return NSE_ERR_ARG;
  if (!u_grid || !alpha_out) return fail(ctx, NSE_ERR_ARG, "NULL array");
  nse_status s = ensure_adjoint_buffers(ctx);
  if (s != NSE_OK) return s;
  int64_t goff = 0;
  for (size_t i = 0; i < ctx->members.size(); ++i) {
    const Group& g = ctx->groups[ctx->member_group[i]];
    const GroupView v = g.member_view(ctx->member_index[i]);
    NSE_HIP(ctx, launch_ring_project(v, g.plan, u_grid + goff, ctx->stream));
    NSE_HIP(ctx, launch_synthesis_adjoint(v, ctx->stream));
    NSE_HIP(ctx, launch_prep_adjoint(v, (double2*)alpha_out, ctx->stream));
    goff += (int64_t)2 * g.nlat * g.M;
  }
  return NSE_OK;
}

nse_status nse_legendre_values(nse_ctx* ctx, int32_t member, int32_t m, double* out) {
  if (!ctx) return NSE_ERR_ARG;
  if (!out) return fail(ctx, NSE_ERR_ARG, "out is NULL");
  if (member < 0 || member >= (int)ctx->members.size())
    return fail(ctx, NSE_ERR_ARG, "member %d out of range", member);
  const Group& g = ctx->groups[ctx->member_group[member]];
  if (m < 0 || m > g.N) return fail(ctx, NSE_ERR_ARG, "order m = %d outside 0..%d", m, g.N);
  const size_t count = (size_t)(g.N + 2 - m) * g.nh;
  NSE_HIP(ctx, hipMemcpyAsync(out, g.d_T1 + t1_order_offset(g.N, m, g.nh), sizeof(double) * count,
                              hipMemcpyDeviceToDevice, ctx->stream));
  return NSE_OK;
}

nse_status nse_profile_enable(nse_ctx* ctx, int32_t enable) {
  if (!ctx) return NSE_ERR_ARG;
  nse_status s = collect_profile(ctx);
  if (s != NSE_OK) return s;
  for (int k = 0; k < NSE_KERNEL_KINDS; ++k) {
    ctx->prof_count[k] = 0;
    ctx->prof_ms[k] = 0.0;
  }
  if (enable < 0 || enable > 1000)
    return fail(ctx, NSE_ERR_ARG, "profile repeat count %d outside 0..1000", enable);
  ctx->profiling = enable != 0;
  ctx->profile_repeat = enable;
  return NSE_OK;
}

nse_status nse_profile_read(nse_ctx* ctx, int32_t kind, int64_t* launches, double* total_ms) {
  if (!ctx) return NSE_ERR_ARG;
  if (kind < 0 || kind >= NSE_KERNEL_KINDS)
    return fail(ctx, NSE_ERR_ARG, "kernel kind %d out of range", kind);
  nse_status s = collect_profile(ctx);
  if (s != NSE_OK) return s;
  if (launches) *launches = ctx->prof_count[kind];
  if (total_ms) *total_ms = ctx->prof_ms[kind];
  ctx->prof_count[kind] = 0;
  ctx->prof_ms[kind] = 0.0;
  return NSE_OK;
}

nse_status nse_energy_spectrum(nse_ctx* ctx, const double* alpha, double* E_out) {
  if (!ctx) return NSE_ERR_ARG;
  if (!alpha || !E_out) return fail(ctx, NSE_ERR_ARG, "alpha and E_out must be non-NULL");
  int64_t eoff = 0;
  for (size_t i = 0; i < ctx->members.size(); ++i) {
    const Group& g = ctx->groups[ctx->member_group[i]];
    const GroupView v = g.member_view(ctx->member_index[i]);
    NSE_HIP(ctx, launch_energy_spectrum(v, (const double2*)alpha, E_out + eoff, ctx->stream));
    eoff += g.N + 1;
  }
  return NSE_OK;
}

nse_status nse_synthesize_psi(nse_ctx* ctx, const double* alpha, double* grid_out) {
  if (!ctx) return NSE_ERR_ARG;
  if (!alpha || !grid_out) return fail(ctx, NSE_ERR_ARG, "NULL array");
  SynthInput in{};
  in.nsrc = 1;
  in.src[0] = (const double2*)alpha;
  in.coef[0] = 1.0;
  in.stream = 1;
  int64_t goff = 0;
  for (size_t i = 0; i < ctx->members.size(); ++i) {
    const Group& g = ctx->groups[ctx->member_group[i]];
    const GroupView v = g.member_view(ctx->member_index[i]);
    NSE_HIP(ctx, launch_synth_any(v, in, SYNTH_GRID, ctx->stream));
    NSE_HIP(ctx, launch_ring(v, g.plan, SYNTH_GRID, grid_out + goff, ctx->stream));
    goff += (int64_t)3 * g.nlat * g.M;
  }
  return NSE_OK;
}

nse_status nse_inertial_manifold(nse_ctx* ctx, const double* alpha_src, int32_t n_src,
                                 int32_t N1, const double* forcing, double* phi_out) {
  if (!ctx) return NSE_ERR_ARG;
  if (!alpha_src || !phi_out) return fail(ctx, NSE_ERR_ARG, "alpha_src and phi_out must be non-NULL");
  if (n_src < 1) return fail(ctx, NSE_ERR_ARG, "n_src must be >= 1");
  if (N1 < 1 || N1 > n_src) return fail(ctx, NSE_ERR_ARG, "N1 must be in 1..n_src");
  for (size_t i = 0; i < ctx->members.size(); ++i) {
    if (N1 > ctx->members[i].N)
      return fail(ctx, NSE_ERR_ARG, "N1 exceeds the truncation of member %zu", i);
    if (!(ctx->members[i].nu > 0.0))
      return fail(ctx, NSE_ERR_ARG, "nu of member %zu must be > 0 ((nu A + C) is inverted)", i);
  }
  if ((const void*)phi_out == (const void*)alpha_src || (const void*)phi_out == (const void*)forcing)
    return fail(ctx, NSE_ERR_ARG, "phi_out may not alias the inputs");
  if (!ctx->d_diag) NSE_HIP(ctx, dalloc(&ctx->d_diag, 2 * (size_t)ctx->state_count));
  double2* band = ctx->d_diag;
  double2* nl = ctx->d_diag + ctx->state_count;
  const int64_t src_stride = nse_coeff_count(n_src);
  for (size_t i = 0; i < ctx->members.size(); ++i) {
    const Group& g = ctx->groups[ctx->member_group[i]];
    const GroupView v = g.member_view(ctx->member_index[i]);
    NSE_HIP(ctx, launch_band_input(v, (const double2*)alpha_src + (int64_t)i * src_stride, n_src,
                                   N1, band, ctx->stream));
  }
  // B(u1, u1) alone: the Coriolis part belongs to the inverted operator
  SynthInput in{};
  in.nsrc = 1;
  in.src[0] = band;
  in.coef[0] = 1.0;
  in.coriolis = 0.0;
  AnalOutput out{};
  out.mode = ANAL_NONLINEAR;
  out.n_out = nl;
  out.state_count = ctx->state_count;
  nse_status s = enqueue_chain(ctx, in, out);
  if (s != NSE_OK) return s;
  for (size_t i = 0; i < ctx->members.size(); ++i) {
    const Group& g = ctx->groups[ctx->member_group[i]];
    const GroupView v = g.member_view(ctx->member_index[i]);
    NSE_HIP(ctx, launch_inertial_manifold(v, nl, (const double2*)forcing, N1, ctx->params.omega,
                                          (double2*)phi_out, ctx->stream));
  }
  return NSE_OK;
}

static nse_status adaptive_begin(nse_ctx* ctx, const double* alpha0, double t0,
                                 const nse_adaptive_params* params, const double* forcing,
                                 nse_forcing_fn fn, void* user,
                                 const nse_forcing_schedule* sched) {
  if (!ctx) return NSE_ERR_ARG;
  if (!alpha0 || !params) return fail(ctx, NSE_ERR_ARG, "alpha0 and params must be non-NULL");
  const nse_adaptive_params& p = *params;
  if (!(p.rtol > 0.0) || !(p.atol > 0.0) || !std::isfinite(p.rtol) || !std::isfinite(p.atol))
    return fail(ctx, NSE_ERR_ARG, "rtol and atol must be finite and > 0");
  if (!(p.h0 >= 0.0) || !(p.hmax >= 0.0))
    return fail(ctx, NSE_ERR_ARG, "h0 and hmax must be >= 0");
  if (p.max_order < 1 || p.max_order > kNdfMaxOrder)
    return fail(ctx, NSE_ERR_ARG, "max_order must be 1..5");
  if (p.max_newton < 1 || p.max_newton > kMaxNewton)
    return fail(ctx, NSE_ERR_ARG, "max_newton must be 1..8");
  if (!std::isfinite(t0)) return fail(ctx, NSE_ERR_ARG, "t0 must be finite");
  if (sched) {
    const nse_forcing_schedule& f = *sched;
    if (!std::isfinite(f.t_on) || !std::isfinite(f.before) || !std::isfinite(f.amp) ||
        !std::isfinite(f.omega) || !std::isfinite(f.phase) || !std::isfinite(f.decay))
      return fail(ctx, NSE_ERR_ARG, "forcing schedule entries must be finite");
  }
  auto& ad = ctx->ad;
  ad = nse_ctx::Adaptive{};
  ad.p = p;
  ad.forcing = (const double2*)forcing;
  ad.fn = fn;
  ad.user = user;
  if (sched) {
    ad.sched = *sched;
  } else {
    ad.sched.t_on = INFINITY;  // s = 1
    ad.sched.before = 1.0;
  }
  NdfCtl& k = ad.c;
  k.rtol = p.rtol;
  k.hmax = p.hmax > 0.0 ? p.hmax : INFINITY;
  k.kmax = p.max_order;
  k.K = p.max_newton;
  k.t = t0;
  k.k = 1;
  // the captured slot sequence names the forcing, the schedule and max_newton
  if (ctx->ad_exec && (ctx->ad_key.forcing != ad.forcing || ctx->ad_key.K != k.K ||
                       std::memcmp(&ctx->ad_key.sched, &ad.sched, sizeof(ad.sched)) != 0)) {
    NSE_HIP(ctx, hipStreamSynchronize(ctx->stream));
    drop_attempt_graph(ctx);
  }
  nse_status s = ensure_ndf_buffers(ctx, p.max_order + 3);
  if (s != NSE_OK) return s;
  const size_t bytes = sizeof(double2) * (size_t)ctx->state_count;
  NSE_HIP(ctx, hipMemcpyAsync(ctx->d_ndf, alpha0, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  NSE_HIP(ctx, hipMemsetAsync(ctx->d_ndf + ctx->state_count, 0, bytes * (ctx->ndf_depth - 1),
                              ctx->stream));
  k.fscale = fn ? fn(user, t0) : schedule_scale(ad.sched, t0);
  ndf_take_prepare(k, 0);  // nothing pending: clears the norms
  s = ndf_prepare_host(ctx);
  if (s != NSE_OK) return s;
  s = ndf_eval(ctx, ctx->d_ndf);
  if (s != NSE_OK) return s;
  s = ndf_correct(ctx, NDF_RHS, 0, nullptr, ctx->d_ndf + ctx->state_count);
  if (s != NSE_OK) return s;
  k.evaluations = 1;
  double nrm[kMaxNewton][4];
  s = read_norms(ctx, 1, nrm);
  if (s != NSE_OK) return s;
  if (!std::isfinite(nrm[0][0])) return fail(ctx, NSE_ERR_NONFINITE, "non-finite F(t0, alpha0)");
  ad.fnorm = nrm[0][0];
  ad.active = true;
  return NSE_OK;
}

nse_status nse_adaptive_begin(nse_ctx* ctx, const double* alpha0, double t0,
                              const nse_adaptive_params* params, const double* forcing,
                              nse_forcing_fn fn, void* user) {
  return adaptive_begin(ctx, alpha0, t0, params, forcing, fn, user, nullptr);
}

nse_status nse_adaptive_begin_scheduled(nse_ctx* ctx, const double* alpha0, double t0,
                                        const nse_adaptive_params* params,
                                        const double* forcing,
                                        const nse_forcing_schedule* schedule) {
  return adaptive_begin(ctx, alpha0, t0, params, forcing, nullptr, nullptr, schedule);
}

nse_status nse_adaptive_advance(nse_ctx* ctx, double t_end, double* alpha_out,
                                nse_adaptive_stats* stats) {
  if (!ctx) return NSE_ERR_ARG;
  auto& ad = ctx->ad;
  NdfCtl& k = ad.c;
  if (!ad.active) return fail(ctx, NSE_ERR_STATE, "nse_adaptive_begin has not been called");
  if (!(t_end >= k.t) || !std::isfinite(t_end))
    return fail(ctx, NSE_ERR_ARG, "t_end must be finite and >= the current time");
  const double rtol = ad.p.rtol;
  if (t_end > k.t && !ad.started) {
    double h = std::min(k.hmax, t_end - k.t);
    if (ad.p.h0 > 0.0)
      h = std::min(h, ad.p.h0);
    else if (ad.fnorm > 0.0 && h * ad.fnorm / (0.8 * std::sqrt(rtol)) > 1.0)
      h = 0.8 * std::sqrt(rtol) / ad.fnorm;
    // D[1] holds F(t0, alpha0): scale it to h F
    k.pend_transform = 1;
    k.pend_tk = 1;
    for (int j = 0; j <= kNdfMaxOrder; ++j)
      for (int i = 0; i <= kNdfMaxOrder; ++i) k.R[j][i] = 0.0;
    k.R[0][0] = 1.0;
    k.R[1][1] = h;
    k.h = h;
    k.k = 1;
    ad.started = true;
  }
  k.t_end = t_end;
  k.done = 0;
  nse_status s = NSE_OK;
  if (!(k.t < t_end)) {
    // nothing to integrate
  } else if (!ad.fn && !ctx->profiling) {
    s = advance_device(ctx);
    if (s != NSE_OK) {
      ad.active = false;
      return s;
    }
  } else {
    for (;;) {
      const int r = ndf_begin_attempt(k);
      if (r == NDF_STOP) break;
      if (r < 0) return ndf_failure(ctx, -r);
      s = ndf_attempt_host(ctx);
      if (s != NSE_OK) {
        ad.active = false;
        return s;
      }
    }
  }
  if (k.pend_accept || k.pend_transform) {
    ndf_take_prepare(k, 0);
    s = ndf_prepare_host(ctx);
    if (s != NSE_OK) return s;
  }
  if (alpha_out)
    NSE_HIP(ctx, hipMemcpyAsync(alpha_out, ctx->d_ndf, sizeof(double2) * ctx->state_count,
                                hipMemcpyDeviceToDevice, ctx->stream));
  if (stats) {
    nse_adaptive_stats st{};
    st.t = k.t;
    st.h = k.h;
    st.order = k.k;
    st.accepted = k.accepted;
    st.error_failures = k.error_failures;
    st.newton_failures = k.newton_failures;
    st.evaluations = k.evaluations;
    st.waits = ad.waits;
    st.wait_seconds = ad.wait_seconds;
    *stats = st;
  }
  return NSE_OK;
}

nse_status nse_adaptive_log(const nse_ctx* ctx, nse_adaptive_record* out, int64_t capacity,
                            int64_t* count) {
  if (!ctx) return NSE_ERR_ARG;
  nse_ctx* c = const_cast<nse_ctx*>(ctx);
  if (capacity < 0 || (capacity > 0 && !out))
    return fail(c, NSE_ERR_ARG, "out must be non-NULL for capacity > 0");
  const int64_t n = (int64_t)ctx->ad.log.size();
  for (int64_t i = 0; i < std::min(n, capacity); ++i) out[i] = ctx->ad.log[i];
  if (count) *count = n;
  return NSE_OK;
}

nse_status nse_sync(nse_ctx* ctx) {
  if (!ctx) return NSE_ERR_ARG;
  NSE_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (ctx->params.flags & NSE_FLAG_CHECK_FINITE) {
    int flag = 0;
    NSE_HIP(ctx, hipMemcpy(&flag, ctx->d_flag, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) {
      NSE_HIP(ctx, hipMemset(ctx->d_flag, 0, sizeof(int)));
      return fail(ctx, NSE_ERR_NONFINITE, "a step produced NaN or Inf");
    }
  }
  return NSE_OK;
}

}  // extern "C"

// Host-side AddressSanitizer harness for the C ABI (the library's host code
// built with -fsanitize=address, device code unchanged). Without a GPU it runs
// the synchronous argument checks; with one it also drives the paths whose host
// bookkeeping is most involved: a mixed-truncation ensemble context (three
// truncation groups on forked streams, autotuned member blocks, step graphs
// captured and replayed, the graph cache filled past its bound and evicted),
// many single-member contexts sharing one stream, the nonlinear adjoint on
// allocated and on static scratch, a trajectory and its step adjoints (eager and
// from captured graphs), one step adjoint, the grid synthesis and the
// projection, an adaptive integration, and destruction of everything. Any host memory error aborts with an ASan report; the last line
// printed on success is "asan driver: ok".
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "nse_sphere.h"

#define EXPECT(cond)                                                  \
  do {                                                                \
    if (!(cond)) {                                                    \
      std::fprintf(stderr, "asan driver: check failed: %s (line %d)\n", #cond, __LINE__); \
      std::exit(2);                                                   \
    }                                                                 \
  } while (0)

static nse_params params(uint32_t flags) {
  nse_params p{};
  p.omega = 2.0 * M_PI;
  p.dt = 1e-3;
  p.order = 2;
  p.newton_iters = 1;
  p.precision = NSE_PREC_FP64;
  p.flags = flags;
  return p;
}

static void argument_checks() {
  nse_ctx* c = nullptr;
  nse_params p = params(0);
  nse_member bad[] = {{0, 0, 1e-3}};
  EXPECT(nse_sphere_init(bad, 1, &p, nullptr, &c) == NSE_ERR_ARG && c == nullptr);
  nse_member alias[] = {{31, 40, 1e-3}};
  EXPECT(nse_sphere_init(alias, 1, &p, nullptr, &c) == NSE_ERR_ARG);
  nse_member prime[] = {{31, 49, 1e-3}};
  EXPECT(nse_sphere_init(prime, 1, &p, nullptr, &c) == NSE_ERR_UNSUPPORTED);
  p.order = 6;
  nse_member ok[] = {{31, 0, 1e-3}};
  EXPECT(nse_sphere_init(ok, 1, &p, nullptr, &c) == NSE_ERR_ARG);
  EXPECT(nse_sphere_init(ok, 1, nullptr, nullptr, &c) == NSE_ERR_ARG);
  EXPECT(nse_last_error(nullptr)[0] != '\0');
  EXPECT(nse_nonlinear(nullptr, nullptr, nullptr) == NSE_ERR_ARG);
  EXPECT(nse_step(nullptr, nullptr, nullptr, 0, 1) == NSE_ERR_ARG);
  EXPECT(nse_sphere_destroy(nullptr) == NSE_OK);
  EXPECT(nse_coeff_count(511) == 131328);
  for (int s = 0; s < 7; ++s) EXPECT(nse_status_string((nse_status)s)[0] == 'N');
  std::printf("asan driver: argument checks ok\n");
}

static double* device_state(int64_t n, double scale) {
  std::vector<double> h(2 * n);
  unsigned long long x = 88172645463325252ull;
  for (auto& v : h) {
    x ^= x << 13; x ^= x >> 7; x ^= x << 17;
    v = scale * ((double)(x >> 11) / 9007199254740992.0 - 0.5);
  }
  double* d = nullptr;
  EXPECT(hipMalloc((void**)&d, sizeof(double) * 2 * n) == hipSuccess);
  EXPECT(hipMemcpy(d, h.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice) == hipSuccess);
  return d;
}

static void gpu_paths() {
  hipStream_t st = nullptr;
  EXPECT(hipStreamCreate(&st) == hipSuccess);
  // mixed ensemble: 24 x N=63, 24 x N=127, 16 x N=255
  std::vector<nse_member> ms;
  for (int i = 0; i < 64; ++i) ms.push_back({i < 24 ? 63 : (i < 48 ? 127 : 255), 0, 1e-4});
  nse_params p = params(NSE_FLAG_GRAPH | NSE_FLAG_AUTOTUNE | NSE_FLAG_CHECK_FINITE);
  nse_ctx* c = nullptr;
  EXPECT(nse_sphere_init(ms.data(), (int)ms.size(), &p, st, &c) == NSE_OK);
  const int64_t S = nse_state_count(c);
  std::vector<double*> hist;
  double* f = device_state(S, 1e-6);
  for (int k = 0; k < 6; ++k) {  // more history arrays than the graph cache holds
    double* h = nullptr;
    EXPECT(hipMalloc((void**)&h, sizeof(double) * 2 * 3 * S) == hipSuccess);
    EXPECT(hipMemset(h, 0, sizeof(double) * 2 * 3 * S) == hipSuccess);
    hist.push_back(h);
  }
  for (int round = 0; round < 2; ++round)
    for (double* h : hist) EXPECT(nse_step(c, h, f, 0, 33) == NSE_OK);
  EXPECT(nse_sync(c) == NSE_OK);
  EXPECT(nse_set_member_blocks(c, 48, 2, 4) == NSE_OK);  // drops the graphs
  EXPECT(nse_step(c, hist[0], f, 33, 20) == NSE_OK);
  EXPECT(nse_sync(c) == NSE_OK);
  EXPECT(nse_sphere_destroy(c) == NSE_OK);
  std::printf("asan driver: ensemble context ok\n");

  // one context per member on a shared stream
  std::vector<nse_ctx*> singles;
  std::vector<double*> sh;
  for (int i = 0; i < 64; ++i) {
    nse_ctx* s1 = nullptr;
    nse_params q = params(NSE_FLAG_GRAPH);
    EXPECT(nse_sphere_init(&ms[i], 1, &q, st, &s1) == NSE_OK);
    double* h = nullptr;
    const int64_t n = nse_state_count(s1);
    EXPECT(hipMalloc((void**)&h, sizeof(double) * 2 * 3 * n) == hipSuccess);
    EXPECT(hipMemset(h, 0, sizeof(double) * 2 * 3 * n) == hipSuccess);
    EXPECT(nse_step(s1, h, nullptr, 0, 23) == NSE_OK);
    singles.push_back(s1);
    sh.push_back(h);
  }
  for (size_t i = 0; i < singles.size(); ++i) EXPECT(nse_sphere_destroy(singles[i]) == NSE_OK);
  std::printf("asan driver: single-member contexts ok\n");

  // adjoint on allocated and on static scratch; adaptive integration
  nse_member m1[] = {{127, 0, 1e-4}};
  nse_params q = params(0);
  nse_ctx* a = nullptr;
  EXPECT(nse_sphere_init(m1, 1, &q, st, &a) == NSE_OK);
  const int64_t n1 = nse_state_count(a);
  double* al = device_state(n1, 1e-2);
  double* nb = device_state(n1, 1.0);
  double* out = device_state(n1, 0.0);
  EXPECT(nse_nonlinear_adjoint(a, al, nb, out) == NSE_OK);
  EXPECT(nse_nonlinear_adjoint_noalloc(a, al, nb, out) == NSE_OK);

  // trajectory buffers and step adjoints, eager here and from captured graphs
  // in a second context (each call twice: capture, then replay)
  const int32_t nsteps = 25, depth = q.order + 1;
  double* traj = device_state((int64_t)(nsteps + depth) * n1, 1e-3);
  double* hbar = device_state((int64_t)depth * n1, 1.0);
  EXPECT(nse_step_trajectory(a, traj, nullptr, 0, nsteps) == NSE_OK);
  EXPECT(nse_step_adjoint_trajectory(a, traj, nullptr, 0, nsteps, hbar) == NSE_OK);
  EXPECT(nse_step_adjoint(a, traj + 2 * n1 * 3, nullptr, 7, hbar) == NSE_OK);
  EXPECT(nse_step_adjoint_trajectory(a, traj, nullptr, 0, nsteps, traj) == NSE_ERR_ARG);
  nse_params qg = params(NSE_FLAG_GRAPH);
  nse_ctx* ag = nullptr;
  EXPECT(nse_sphere_init(m1, 1, &qg, st, &ag) == NSE_OK);
  for (int rep = 0; rep < 2; ++rep) {
    EXPECT(nse_step_trajectory(ag, traj, nullptr, 3, nsteps) == NSE_OK);
    EXPECT(nse_step_adjoint_trajectory(ag, traj, nullptr, 3, nsteps, hbar) == NSE_OK);
  }
  EXPECT(nse_sync(ag) == NSE_OK);
  EXPECT(nse_sphere_destroy(ag) == NSE_OK);
  // grid synthesis and the projection back onto the basis
  int32_t nlat = 0;
  EXPECT(nse_member_grid(a, 0, &nlat, nullptr, nullptr) == NSE_OK);
  double* grid = nullptr;
  EXPECT(hipMalloc((void**)&grid, sizeof(double) * 3 * nlat * 2 * nlat) == hipSuccess);
  EXPECT(nse_synthesize(a, al, grid) == NSE_OK);
  EXPECT(nse_analyze_velocity(a, grid, out) == NSE_OK);
  EXPECT(nse_sync(a) == NSE_OK);
  std::printf("asan driver: trajectory, step adjoints and projection ok\n");
  nse_adaptive_params ap{};
  ap.rtol = 1e-3;
  ap.atol = 1e-6;
  ap.max_order = 5;
  ap.max_newton = 4;
  EXPECT(nse_adaptive_begin(a, al, 0.0, &ap, nullptr, nullptr, nullptr) == NSE_OK);
  nse_adaptive_stats stats{};
  EXPECT(nse_adaptive_advance(a, 0.02, out, &stats) == NSE_OK);
  std::vector<nse_adaptive_record> log(64);
  int64_t count = 0;
  EXPECT(nse_adaptive_log(a, log.data(), (int64_t)log.size(), &count) == NSE_OK);
  EXPECT(nse_sync(a) == NSE_OK);
  EXPECT(nse_sphere_destroy(a) == NSE_OK);
  std::printf("asan driver: adjoint and adaptive ok (%lld attempts)\n", (long long)count);

  for (double* h : hist) (void)hipFree(h);
  for (double* h : sh) (void)hipFree(h);
  (void)hipFree(f);
  (void)hipFree(al);
  (void)hipFree(nb);
  (void)hipFree(out);
  (void)hipFree(traj);
  (void)hipFree(hbar);
  (void)hipFree(grid);
  (void)hipStreamDestroy(st);
}

int main() {
  argument_checks();
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) gpu_paths();
  else std::printf("asan driver: no GPU, device paths skipped\n");
  std::printf("asan driver: ok\n");
  return 0;
}

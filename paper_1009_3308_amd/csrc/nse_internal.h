// Internal declarations shared by the HIP sources of libnse_sphere.so.
// Nothing here is part of the C ABI (include/nse_sphere.h).
#pragma once

#include <hip/hip_runtime.h>

#include "nse_sphere.h"

#include <cstdint>
#include <string>
#include <vector>

namespace nse {

constexpr int kMaxSources = 6;   // predictor terms of NDF_5 (q + 1 <= 6)
constexpr int kMaxStepCoef = 7;  // c_0 .. c_{q+1} of NDF_5
constexpr int kMaxRadices = 16;
constexpr int kMaxM = 1536;      // largest supported longitude count (ring LDS <= 64 KiB)

// Linear work item of block `bid` such that the blocks the dispatcher places on one
// XCD (bid % 8, round-robin) take consecutive chunks of `chunk` items, and chunks
// alternate between XCDs. Neighbouring items then share that XCD's L2.
__host__ __device__ inline int xcd_item(int bid, int chunk) {
  const int x = bid & 7, k = bid >> 3;
  return ((x + 8 * (k / chunk)) * chunk) + (k % chunk);
}
// As xcd_item, with the XCD order reversed on every other round of chunks, so
// that when the cost of a chunk falls with its index (orders m of decreasing
// degree count) every XCD gets a similar share.
__host__ __device__ inline int xcd_item_snake(int bid, int chunk) {
  const int x = bid & 7, k = bid >> 3;
  const int round = k / chunk;
  const int xs = (round & 1) ? 7 - x : x;
  return ((xs + 8 * round) * chunk) + (k % chunk);
}
// Grid size covering `items` work items for xcd_item (a multiple of 8 * chunk).
__host__ __device__ inline int xcd_grid(int items, int chunk) {
  const int per = 8 * chunk;
  return ((items + per - 1) / per) * per;
}

// Slot of (l, m) inside one member: m-major, l fastest.
__host__ __device__ inline int64_t coeff_offset(int N, int m) {
  return (int64_t)m * (2 * N + 3 - m) / 2;
}
// Per-degree coefficients of the normalised Legendre recurrence of eq. (sph_har),
// computed once per group on the host, for l = m .. N+1 at rec_slot(N, l, m):
//   rec_a = (a(l,m), a(l,m) / a(l-1,m)),  a(l,m) = sqrt((4 l^2 - 1) / (l^2 - m^2)),
//   rec_g = ((2l+1) e(l), lambda_l^(-1/2)),  e(l) = 1 / a(l,m),
//   rec_p = (l e(l+1), (l+1) e(l))  (the coefficients of the transposed panel
//           recurrences of the adjoint; l e(l+1) = 0 at l = N+1),
// with a(m,m) = e(m) = 0, the ratio 0 for l <= m+1 (it multiplies Pbar[m-1,m] = 0)
// and lambda^(-1/2) = 0 at l = 0.
__host__ __device__ inline int64_t rec_slot(int N, int l, int m) {
  return coeff_offset(N + 1, m) + (l - m);
}
// Legendre tables, l = m .. N+1 (L = N + 2 - m degrees for order m, k = l - m):
//   T1[m][k][p]                        (synthesis; latitude fastest, row stride nh)
//   T2[m][deg tile][p][64 degrees]     (analysis; ceil(L/64) tiles of 64 degrees,
//                                       each a contiguous block streamed by one
//                                       workgroup; orders start at t2off[m])
constexpr int kTile = 64;
__host__ __device__ inline int64_t t1_order_offset(int N, int m, int nh) {
  return (int64_t)nh * ((int64_t)m * (2 * N + 5 - m) / 2);
}
__host__ __device__ inline int64_t t1_size(int N, int nh) {
  return (int64_t)nh * ((int64_t)(N + 1) * (N + 4) / 2);
}

// Device view of one truncation group (members sharing N and nlat).
struct GroupView {
  int N, nlat, nh, M, nb;   // nh = northern latitudes incl. the equator if nlat is odd
  int precision;            // NSE_PREC_* of the Legendre contractions
  int mb_synth, mb_anal;    // member blocks of the batched FP64 MFMA kernels (0 = per member)
  const double* mu;         // [nh] Gauss-Legendre nodes, descending
  const double* w;          // [nh]
  const double* T1;         // FP64 synthesis table (layouts above)
  const double* T2;         // FP64 analysis table
  const float* T1f;         // FP32 copies (split-bf16x3 mode only), else null
  const float* T2f;
  const int64_t* t2off;     // [N+2] start of order m in T2 (element units)
  const double2* rec_a;     // [(N+2)(N+3)/2] (a(l,m), a(l,m) / a(l-1,m)), slot rec_slot(N, l, m)
  const double2* rec_g;     // same slots: ((2l+1) e(l), lambda_l^(-1/2)), see rec_slot
  const double2* rec_p;     // same slots: (l e(l+1), (l+1) e(l)), see rec_slot
  double2* F;               // [nb][4][N+1][nlat] Fourier coefficients of grid fields
  double2* Fa;              // adjoint: [nb][5][N+1][nlat] (4 forward fields + adjoint input)
  double2* Fbar;            // adjoint: [nb][4][N+1][nlat] cotangents of the field spectra
  double2* Pbar;            // adjoint: [nb][N+1][N+2][4] cotangents of the panels
  double2* W;               // [nb][N+1][nlat] weighted ring spectra (analysis input),
                            // latitude fastest so the analysis reads them coalesced
  uint64_t* lps;            // split-bf16 synthesis panels, 8-byte groups (precision BF16X3)
  const int64_t* lpsoff;    // [N+2] start of order m in one member's lps (member stride lpsoff[N+1])
  const double2* tw;        // [M] exp(-2 pi i k / M)
  const int64_t* off;       // [nb] complex-slot offset of each member in a state
  const double* nu;         // [nb]
  const int* gate;          // null, or a device flag: the chain kernels do nothing while it is 0
};

// True when the launch belongs to a gated sequence whose flag is closed (read
// once per workgroup; uniform, so the whole workgroup returns).
__device__ inline bool gate_closed(const GroupView& g) {
  return g.gate && __hip_atomic_load(g.gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
}

struct FftPlan {
  int nstages;
  int radix[kMaxRadices];
  int ns_log2[kMaxRadices];  // log2 of the stride Ns before each stage, -1 if not a power of 2
};

// The history update that ends the adjoint of one NDF step (eq. (ode_disc)
// transposed), from the panel cotangents Pbar of its nonlinear adjoint:
//   r = hin[0] / (c_0 + h nu lambda)   (zero at l = 0, real at m = 0),
//   hout[j] = hin[j+1] - c_{j+1} r + pi_j alpha_bar,   j = 0 .. depth-1,
// with alpha_bar the predictor cotangent (the transposed panel recurrences) and
// pi_j the predictor's weights.
struct StepAdjointArgs {
  const double2* hin;  // [depth][state]
  double2* hout;       // [depth][state]; may equal hin
  int64_t state_count;
  int depth;           // order + 1
  int ncoef;           // c_0 .. c_{ncoef-1}
  int npi;             // pi_0 .. pi_{npi-1}
  double c[kMaxStepCoef];
  double pi[kMaxSources];
  double h;
};

// Input of the synthesis: sum_i coef[i] * src[i] (predictor or plain state).
struct SynthInput {
  const double2* src[kMaxSources];
  double coef[kMaxSources];
  int nsrc;
  double coriolis;  // 2 Omega sqrt(4 pi / 3): absolute-vorticity fold of zeta[1,0]
  const double2* adj;  // SYNTH_ADJ: cotangent n_bar of the nonlinear term (state array)
  // SYNTH_ADJ inside the step adjoint: adj is hbar_out[0] and
  // n_bar = -h hbar_out[0] / (c_0 + h nu lambda) (zero at l = 0, real at m = 0)
  int adj_step;
  double adj_c0, adj_h;
  int stream;  // SYNTH_GRID: third field Psi_N = -sum lambda^(-1/2) alpha Y instead of zeta
};

// SYNTH_ADJ: the four forward fields plus a fifth, lambda^(-1/2) n_bar (the
// adjoint of the analysis), written to GroupView::Fa.
enum SynthMode { SYNTH_NONLINEAR = 0, SYNTH_GRID = 1, SYNTH_ADJ = 2 };
enum AnalMode { ANAL_NONLINEAR = 0, ANAL_STEP_ITER = 1, ANAL_STEP_FINAL = 2, ANAL_NDF = 3 };

struct NdfCtl;  // ndf_control.h

struct AnalOutput {
  int mode;
  double2* n_out;            // ANAL_NONLINEAR: state array
  double2* hist;             // step modes: [depth][state]
  int64_t state_count;
  int depth;                 // order + 1
  int ncoef;                 // c_0 .. c_{ncoef-1}
  double c[kMaxStepCoef];
  double h;
  const double2* forcing;    // may be null
  double2* iter;             // ANAL_STEP_ITER output
  int* nonfinite;            // may be null
  int shift;                 // ANAL_STEP_FINAL on a trajectory buffer: the new state goes
                             // to hist[-1] (the slot before the history), nothing rotates
  // ANAL_NDF (k_analysis_otf): the corrector sweep of a device-controlled
  // adaptive run in the epilogue, with h, the order and the forcing scale from
  // the control block: d = (h (s f - n) - h nu lambda y0 - psi) / (alpha_k + h nu lambda),
  // y = y0 + d, and the sweep's four weighted max norms (as k_ndf_correct)
  const NdfCtl* ctl;
  const double2* D;          // [kmax + 3][state_count] backward differences
  const double2 *y0, *psi, *dprev;  // dprev: read only when the attempt has had a sweep
  double2 *dout, *yout;
  unsigned long long* nrow;  // the sweep's spread norm row (squares, IEEE bits, atomic max)
  int kmax;
  double thr2;               // (atol / rtol)^2
  // when ctl->prep_in_analysis: the epilogue applies the slot's update of the
  // differences D[0..ddepth) (accepted correction from dacc[ctl->prep_dsel])
  double2* Dw;
  const double2* dacc[2];
  int ddepth;
};

// Adaptive NDF integrator (Section 4.2, eq. (ode_disc) in backward differences
// at a quasi-constant step). D[j] = nabla^j y_n at the current spacing h,
// j = 0..k+2; one attempt predicts y0 = sum_{j<=k} D[j] and
// psi = sum_{1<=j<=k} gamma_j D[j] and sweeps
//   d_i = (h (f - n(y_{i-1})) - h nu lambda y0 - psi) / ((1 - kappa_k) gamma_k + h nu lambda),
//   y_i = y0 + d_i.
constexpr int kNdfMaxOrder = 5;
constexpr int kNdfDepth = kNdfMaxOrder + 3;
enum NdfMode { NDF_SWEEP = 0, NDF_RHS = 1 };
struct NdfArgs {
  double2* D;                  // [depth][S]
  int64_t S;                   // state count (stride of D)
  int depth;                   // max_order + 3
  // k_ndf_prepare: accept, then rescale, then predict
  int accept, k_acc;           // D update with the correction dacc of an order-k_acc step
  const double2* dacc;
  int transform, k;            // D[j] <- sum_{i=j..k} R[j][i] D[i], D[k+1..] <- 0
  double R[kNdfMaxOrder + 1][kNdfMaxOrder + 1];
  int predict;                 // write y0 and psi for order k
  double gam[kNdfMaxOrder + 1];  // gamma_j = sum_{i<=j} 1/i
  double2 *y0, *psi;
  unsigned long long* norms;   // zeroed by k_ndf_prepare (nnorms entries)
  int nnorms;
  // k_ndf_correct
  int mode;                    // NDF_SWEEP, or NDF_RHS: dout = f - nu lambda D[0] - n
  int kmax;
  const double2* n;            // nonlinear term of the previous iterate
  const double2* f;            // forcing buffer (null = 0), scaled by fscale
  double fscale;
  const double2* dprev;        // previous correction (null = 0)
  double2* dout;               // this correction
  double2* yout;               // this iterate
  double h, ak, thr2;          // step, (1 - kappa_k) gamma_k, (atol / rtol)^2
  unsigned long long* nrow;    // squared weighted max norms of this sweep (IEEE bits):
                               // [0] d - dprev, [1] d, [2] D[k] + d (k > 1), [3] d - D[k+1] (k < kmax)
  // publication of the sweep's norms to host memory by the launch's last workgroup
  int publish, sweep;
  unsigned int* done;          // [max sweeps] workgroup counters, zeroed by k_ndf_prepare
  unsigned long long* pub;     // host-mapped: [4 x max sweeps] norms, then the sequence word
  unsigned long long seq;
  // device-controlled integration (k_ndf_step, and k_ndf_correct with h, the
  // order and the forcing scale from the control block ctl, run while an
  // attempt is open)
  const NdfCtl* ctl;
  double2* dsel[2];            // the two correction buffers (accepted one chosen by the control block)
  int64_t spread_words;        // k_ndf_step: words of a spread norm row
};

// Launchers (each enqueues on `s` and returns the launch status).
hipError_t launch_legendre_table(const GroupView& g, double* T1, double* T2, float* T1f,
                                 float* T2f, hipStream_t s);
hipError_t launch_synthesis(const GroupView& g, const SynthInput& in, int mode, hipStream_t s);
hipError_t launch_ring(const GroupView& g, const FftPlan& plan, int mode, double* grid_out,
                       hipStream_t s);
hipError_t launch_analysis(const GroupView& g, const AnalOutput& out, hipStream_t s);
hipError_t launch_ring_adjoint(const GroupView& g, const FftPlan& plan, hipStream_t s);
hipError_t launch_ring_project(const GroupView& g, const FftPlan& plan, const double* u_grid,
                               hipStream_t s);
hipError_t launch_synthesis_adjoint(const GroupView& g, hipStream_t s);
hipError_t launch_prep_adjoint(const GroupView& g, double2* alpha_bar, hipStream_t s);
hipError_t launch_prep_step_adjoint(const GroupView& g, const StepAdjointArgs& a, hipStream_t s);
hipError_t launch_synthesis_mb(const GroupView& g, const SynthInput& in, int B, hipStream_t s);
hipError_t launch_analysis_mb(const GroupView& g, const AnalOutput& out, int B, hipStream_t s);
hipError_t launch_synthesis_lp(const GroupView& g, const SynthInput& in, int mode, int prec,
                               hipStream_t s);
hipError_t launch_analysis_lp(const GroupView& g, const AnalOutput& out, int prec, hipStream_t s);
hipError_t launch_ndf_prepare(const NdfArgs& a, hipStream_t s);
// Diagnostics (Section 5.3): energy spectrum E[b][L], band-limited copy of a
// state stored at truncation n_src, approximate inertial manifold.
hipError_t launch_energy_spectrum(const GroupView& g, const double2* alpha, double* E,
                                  hipStream_t s);
hipError_t launch_band_input(const GroupView& g, const double2* src, int n_src, int lmax,
                             double2* dst, hipStream_t s);
hipError_t launch_inertial_manifold(const GroupView& g, const double2* n, const double2* f,
                                    int N1, double omega, double2* phi, hipStream_t s);
hipError_t launch_ndf_correct(const GroupView& g, const NdfArgs& a, hipStream_t s);

// Dynamic LDS of the launches (validated against 64 KiB at init).
size_t synthesis_lds_bytes(int N, int NF);
size_t ring_lds_bytes(int M);
size_t analysis_otf_lds_bytes(int nh);
size_t synthesis_adjoint_lds_bytes(int nh);
size_t synthesis_lp_lds_bytes(int N);
size_t split_panel_lp_lds_bytes(int N);
size_t analysis_lp_lds_bytes(int nh);

// Host numerics.
void gauss_legendre(int n, std::vector<double>& mu, std::vector<double>& w);
bool fft_factor(int M, FftPlan& plan);

}  // namespace nse

// Host runtime of the SPG solver: validation, workspace carving, launch sequence and the
// extern "C" entry points declared in include/spg.h.  All device state lives in the
// caller's workspace; this file allocates host memory only (and HIP events while
// profiling is on).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/spg.h"
#include "spg_internal.h"

using namespace spg;

namespace {

constexpr size_t kAlign = 256;
constexpr int kStatBlocks = 1024;           // grid of the input-check / reweight kernels
constexpr int kPartials = 262144;           // fp64 partials in the workspace
constexpr int kPartA = 0;                   // z-pass objective partials (<= 8192 blocks)
constexpr int kPartB = 8192;                // kx = 0 / nx/2 plane partials (<= 257 blocks)
constexpr int kPartC = 16384;               // stencil partials: check 6 x <= 8192, monitor 3 x <= 65536
constexpr int kHistCap = 4096;              // monitored objectives kept (a ring)
constexpr uint64_t kStateMagic = 0x5350475354415431ull;  // "SPGSTAT1"

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

// Supported axis lengths: powers of two in [4, 512], and the mixed-radix 160 = 5 * 32 and
// 192 = 3 * 64 (their x-axis half lengths 80 and 96 are also supported transforms).
bool axis_ok(int n) { return pow2_in(n, 4, 512) || n == 160 || n == 192; }

struct Layout {
  size_t xhi[3], xlo[3], u, v, S, rbuf, xprev, ws, w0p, wnyq, cs, c0p, cnyq, tw_m, tw_n, tw_y, tw_z, part, res, hist,
      total;
};

Layout make_layout(const spg_params& p) {
  Layout L{};
  const size_t nvox = (size_t)p.nx * p.ny * p.nz;
  const size_t P = (size_t)p.nx / 2;
  const bool comp = (p.flags & SPG_FLAG_COMPENSATED) != 0;
  const size_t rbytes = (p.flags & SPG_FLAG_BF16_STORAGE) ? 2 : 4;  // weights and map buffer
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  for (int s = 0; s < 3; ++s) L.xhi[s] = take(nvox * 4);
  for (int s = 0; s < 3; ++s) L.xlo[s] = comp ? take(nvox * 2) : 0;
  L.u = take(nvox * rbytes);
  L.v = take(nvox * rbytes);
  L.S = take((size_t)p.nz * p.ny * P * 8);
  L.rbuf = take(nvox * rbytes);
  L.xprev = take(nvox * 4);
  L.ws = take((size_t)p.nz * p.ny * P * 4);
  L.w0p = take((size_t)p.nz * p.ny * 4);
  L.wnyq = take((size_t)p.nz * p.ny * 4);
  L.cs = take((size_t)p.nz * p.ny * P * 8);
  L.c0p = take((size_t)p.nz * p.ny * 8);
  L.cnyq = take((size_t)p.nz * p.ny * 8);
  L.tw_m = take(P * 8);
  L.tw_n = take((size_t)p.nx * 8);
  L.tw_y = take((size_t)p.ny * 8);
  L.tw_z = take((size_t)p.nz * 8);
  L.part = take((size_t)kPartials * 8);
  L.res = take(64 * 8);
  L.hist = take((size_t)kHistCap * 8);
  L.total = off;
  return L;
}

const char* check_params(const spg_params* p, spg_status* st) {
  *st = SPG_E_INVAL;
  if (!p) return "params is NULL";
  if (!axis_ok(p->nx) || !axis_ok(p->ny) || !axis_ok(p->nz))
    return "nx, ny, nz must be powers of two in [4, 512], or 160 or 192";
  if (!std::isfinite(p->lambda) || p->lambda < 0) return "lambda must be finite and >= 0";
  if (!std::isfinite(p->mu) || p->mu < 0) return "mu must be finite and >= 0";
  if (!std::isfinite(p->eps) || p->eps <= 0) return "eps must be finite and > 0";
  if (!std::isfinite(p->gamma) || p->gamma < 0) return "gamma must be finite and >= 0";
  if (p->accel != 0 && p->accel != 1) return "accel must be 0 or 1";
  if (p->flags & ~(SPG_FLAG_COMPENSATED | SPG_FLAG_BF16_STORAGE | SPG_FLAG_MONITOR)) return "unknown flag bits";
  if (p->obj_every < 0 || ((p->flags & SPG_FLAG_MONITOR) && p->obj_every < 1))
    return "obj_every must be >= 0, and >= 1 with SPG_FLAG_MONITOR";
  if ((p->flags & SPG_FLAG_COMPENSATED) && (p->flags & SPG_FLAG_BF16_STORAGE))
    return "SPG_FLAG_COMPENSATED and SPG_FLAG_BF16_STORAGE are exclusive";
  *st = SPG_OK;
  return nullptr;
}

// Round to the nearest bf16 (ties to even), as the device conversion does.
double bf16_round(double v) {
  float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  u &= 0xFFFF0000u;
  std::memcpy(&f, &u, 4);
  return f;
}

double dnorm2_of(int nx, int ny, int nz) {
  // largest eigenvalue of D^T D for periodic backward differences: 4 per even axis
  double s = 0;
  const int ns[3] = {nx, ny, nz};
  for (int a = 0; a < 3; ++a) {
    double m = 0;
    for (int k = 0; k < ns[a]; ++k) {
      const double v = 4.0 * std::pow(std::sin(M_PI * k / ns[a]), 2);
      m = v > m ? v : m;
    }
    s += m;
  }
  return s;
}

}  // namespace

struct spg_problem {
  spg_params prm{};
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  Layout lay{};
  Dims d{};
  bool comp = false;
  int store = ST_PLAIN;
  bool prior_set = false;
  bool data_set = false;
  bool primed = false;
  bool sticky = false;
  bool dev_ready = false;   // twiddle tables uploaded and x_0 = 0 written
  int32_t fail_after = -1;  // failure injection: checked HIP calls to let pass, -1 = off
  bool unif_u = true, unif_v = true;
  double maxwt = 0, vmax = 1, C0 = 0, L = 0, lr = 0, dn2 = 12;
  double rms_unreg = 0, mean_w = 0;  // parameter scales of the current data
  int cur = 0, old = 1;
  int64_t iters_done = 0;
  int32_t round = 1;
  int32_t j = 1;         // index of the next iteration within the round (1-based)
  // objective monitor: F_eps(y_j) of every iteration with j % mon_every == 0, into the
  // device ring hist (slot = entry % kHistCap) with the iteration numbers on the host
  int32_t mon_every = 0;
  int64_t hist_n = 0;
  std::vector<int64_t> hist_iter;
  double t = 1.0;        // FISTA t_j
  double m_cur = 0.0;    // momentum m_j of y_j
  char err[512] = {0};
  // launch shapes (chosen by spg_autotune): columns per tile of the y and z passes, z-slab
  // depth of the stencil kernel
  int nt_y = 16, nt_z = 16, zc = PT_ZC;
  bool fused = false;  // fused x-axis transforms in the stencil/prox kernel
  bool shared_gpu = false;  // being captured into a batch graph with other problems
  // unrolled solve recorded by spg_run_checkpointed for spg_vjp
  bool vjp_valid = false;
  int32_t vjp_K = 0, vjp_C = 0;
  double vjp_lr = 0;
  std::vector<double> vjp_m;
  // profiling: events [class][launch][begin/end]
  bool prof_on = false;
  int prof_class = -1, prof_cap = 0;
  int prof_n[SPG_KERNEL_COUNT] = {0};
  std::vector<hipEvent_t> ev;

  template <typename T>
  T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
  float* xhi(int s) { return at<float>(lay.xhi[s]); }
  uint16_t* xlo(int s) { return comp ? at<uint16_t>(lay.xlo[s]) : nullptr; }
  float2* S() { return at<float2>(lay.S); }
  float* rbuf() { return at<float>(lay.rbuf); }
  double* part() { return at<double>(lay.part); }
  double* res() { return at<double>(lay.res); }
  bool bf() const { return store == ST_BF16; }
  const void* uptr() { return unif_u ? nullptr : at<void>(lay.u); }
  const void* vptr() { return unif_v ? nullptr : at<void>(lay.v); }
  size_t wbytes() const { return (size_t)d.nvox * (store == ST_BF16 ? 2 : 4); }
};

namespace {

spg_status set_err(spg_problem* P, spg_status s, const char* fmt, const char* a = "") {
  if (P) std::snprintf(P->err, sizeof(P->err), fmt, a);
  return s;
}

spg_status fail_device(spg_problem* P, hipError_t e, const char* what) {
  P->sticky = true;
  std::snprintf(P->err, sizeof(P->err), "HIP error in %s: %s", what, hipGetErrorString(e));
  return SPG_E_DEVICE;
}

// An injected failure (spg_debug_fail_after) reports the call as failed after issuing it,
// as a device error found late would.
hipError_t injected(spg_problem* P, hipError_t e) {
  if (P->fail_after >= 0 && e == hipSuccess && P->fail_after-- == 0) return hipErrorLaunchFailure;
  return e;
}

#define SPG_CK(P, expr)                                         \
  do {                                                          \
    hipError_t e_ = injected((P), (expr));                      \
    if (e_ != hipSuccess) return fail_device((P), e_, #expr);   \
  } while (0)

void restart(spg_problem* P);

// Device state of a new problem, on its first call that enqueues work: the twiddle tables
// exp(-2 pi i m / n), computed in fp64 and rounded once, and x_0 = 0.
spg_status device_init(spg_problem* P) {
  const spg_params* p = &P->prm;
  const int lens[4] = {p->nx / 2, p->nx, p->ny, p->nz};
  const size_t offs[4] = {P->lay.tw_m, P->lay.tw_n, P->lay.tw_y, P->lay.tw_z};
  std::vector<float2> tab;
  for (int t = 0; t < 4; ++t) {
    const int n = lens[t];
    tab.resize(n);
    for (int m = 0; m < n; ++m) {
      const double ang = -2.0 * M_PI * (double)m / (double)n;
      tab[m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    SPG_CK(P, hipMemcpyAsync(P->ws + offs[t], tab.data(), n * sizeof(float2), hipMemcpyHostToDevice, P->stream));
    SPG_CK(P, hipStreamSynchronize(P->stream));
  }
  SPG_CK(P, launch_set_map(P->d, nullptr, P->xhi(P->cur), P->xlo(P->cur), P->stream));
  restart(P);
  P->dev_ready = true;
  return SPG_OK;
}

spg_status usable(spg_problem* P) {
  if (!P) return SPG_E_INVAL;
  if (P->sticky) return SPG_E_DEVICE;
  if (!P->dev_ready) return device_init(P);
  return SPG_OK;
}

void recompute_L(spg_problem* P) {
  P->L = P->maxwt + P->prm.mu * P->vmax * P->dn2 / P->prm.eps + 2.0 * P->prm.gamma;
  P->lr = P->L > 0 ? 1.0 / P->L : 0.0;
}

void restart(spg_problem* P) {
  P->vjp_valid = false;  // a recorded unrolled solve no longer matches
  P->j = 1;
  P->t = 1.0;
  P->m_cur = 0.0;
  P->primed = false;
}

// Profiling hooks around one launch of kernel class cls.
bool prof_wants(spg_problem* P, int cls) {
  return P->prof_on && (P->prof_class == SPG_KERNEL_ALL || P->prof_class == cls) && P->prof_n[cls] < P->prof_cap;
}
size_t prof_slot(spg_problem* P, int cls) { return 2 * ((size_t)cls * P->prof_cap + P->prof_n[cls]); }
void prof_begin(spg_problem* P, int cls) {
  if (prof_wants(P, cls)) (void)hipEventRecord(P->ev[prof_slot(P, cls)], P->stream);
}
void prof_end(spg_problem* P, int cls) {
  if (prof_wants(P, cls)) {
    (void)hipEventRecord(P->ev[prof_slot(P, cls) + 1], P->stream);
    ++P->prof_n[cls];
  }
}

spg_status read_results_to(spg_problem* P, const double* dev, double* host, int n) {
  SPG_CK(P, hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  SPG_CK(P, hipStreamSynchronize(P->stream));
  return SPG_OK;
}

spg_status read_results(spg_problem* P, double* host, int n) {
  SPG_CK(P, hipMemcpyAsync(host, P->res(), n * sizeof(double), hipMemcpyDeviceToHost, P->stream));
  SPG_CK(P, hipStreamSynchronize(P->stream));
  return SPG_OK;
}

// The y, z passes with the weight step on the x-spectrum rows in S (the forward x
// transform of y already done), the y inverse and, unless x_inverse is false, the x
// inverse into gout.  obj: also collect the data-term partials.
spg_status gradient_pipeline(spg_problem* P, bool obj, int* nA, int* nB, void* gout, bool gout_bf16,
                             bool x_inverse = true) {
  const Dims& d = P->d;
  hipStream_t st = P->stream;
  const float2* twy = P->at<float2>(P->lay.tw_y);
  const float2* twz = P->at<float2>(P->lay.tw_z);
  const float* wsp = P->at<float>(P->lay.ws);
  const float2* csp = P->at<float2>(P->lay.cs);
  if (!obj && yz_plane_supported(d)) {
    // small maps: the y, z (with the weight step and the packed plane) and y inverse passes
    // in one launch, timed as the z pass
    prof_begin(P, SPG_KERNEL_FFT_Z_WEIGHT);
    SPG_CK(P, launch_yz_plane(d, P->S(), twy, twz, wsp, csp, P->at<float>(P->lay.w0p), P->at<float>(P->lay.wnyq),
                              P->at<float2>(P->lay.c0p), P->at<float2>(P->lay.cnyq), st));
    prof_end(P, SPG_KERNEL_FFT_Z_WEIGHT);
  } else {
    // Where the spectrum outgrows the 256 MiB last-level cache, the y, z, y passes run on four
    // column ranges (kx quarters) in turn, so that each pass reads what the previous one just
    // wrote while it is still cached (measured at 512^3: 1.3% more iterations/s, most of it in
    // the stencil kernel that follows).  The objective variant of the z pass takes whole rows.
    const int nch = (!obj && (double)d.nvox * 4.0 >= 256.0 * 1024 * 1024 && d.P % 64 == 0) ? 4 : 1;
    const int cw = d.P / nch;
    for (int c = 0; c < nch; ++c) {
      const int kx0 = c * cw, nkx = nch > 1 ? cw : 0;
      prof_begin(P, SPG_KERNEL_FFT_Y_FWD);
      SPG_CK(P, launch_fft_cols(d, P->S(), 1, 0, twy, nullptr, nullptr, nullptr, st, nullptr, P->nt_y, true, kx0, nkx));
      prof_end(P, SPG_KERNEL_FFT_Y_FWD);
      prof_begin(P, SPG_KERNEL_FFT_Z_WEIGHT);
      // the objective variant writes one partial per block: 16-column tiles keep <= 8192 blocks
      SPG_CK(P, launch_fft_cols(d, P->S(), 2, obj ? 3 : 2, twz, wsp, csp, obj ? P->part() + kPartA : nullptr, st, nA,
                                obj ? 16 : P->nt_z, !P->shared_gpu, kx0, nkx));
      prof_end(P, SPG_KERNEL_FFT_Z_WEIGHT);
      if (c == 0) {  // the packed kx = 0 / nx/2 plane
        prof_begin(P, SPG_KERNEL_DC_NYQUIST);
        SPG_CK(P, launch_dc_nyquist(d, P->S(), twz, P->at<float>(P->lay.w0p), P->at<float>(P->lay.wnyq),
                                    P->at<float2>(P->lay.c0p), P->at<float2>(P->lay.cnyq),
                                    obj ? P->part() + kPartB : nullptr, st, nB));
        prof_end(P, SPG_KERNEL_DC_NYQUIST);
      }
      prof_begin(P, SPG_KERNEL_FFT_Y_INV);
      SPG_CK(P, launch_fft_cols(d, P->S(), 1, 1, twy, nullptr, nullptr, nullptr, st, nullptr, P->nt_y, true, kx0, nkx));
      prof_end(P, SPG_KERNEL_FFT_Y_INV);
    }
  }
  if (!x_inverse) return SPG_OK;
  prof_begin(P, SPG_KERNEL_C2R_X);
  SPG_CK(P, launch_c2r_x(d, P->S(), gout, gout_bf16, P->at<float2>(P->lay.tw_m), P->at<float2>(P->lay.tw_n), st));
  prof_end(P, SPG_KERNEL_C2R_X);
  return SPG_OK;
}

spg_status r2c(spg_problem* P, const void* rin, bool rin_bf16) {
  prof_begin(P, SPG_KERNEL_R2C_X);
  SPG_CK(P, launch_r2c_x(P->d, rin, rin_bf16, P->S(), P->at<float2>(P->lay.tw_m), P->at<float2>(P->lay.tw_n),
                         P->stream));
  prof_end(P, SPG_KERNEL_R2C_X);
  return SPG_OK;
}

ProxArgs prox_args(spg_problem* P, int nxt, double m, double m_next) {
  ProxArgs a{};
  a.rbuf = P->rbuf();
  a.xk_hi = P->xhi(P->cur);
  a.xk_lo = P->xlo(P->cur);
  a.xo_hi = P->xhi(P->old);
  a.xo_lo = P->xlo(P->old);
  a.xn_hi = P->xhi(nxt);
  a.xn_lo = P->xlo(nxt);
  a.u = P->uptr();
  a.v = P->vptr();
  a.gin = nullptr;
  a.xprev = (P->prm.gamma != 0 && P->prior_set) ? P->at<float>(P->lay.xprev) : nullptr;
  a.gamma = P->prm.gamma;
  a.partials = nullptr;
  a.nx = P->d.nx;
  a.ny = P->d.ny;
  a.nz = P->d.nz;
  a.read_old = m != 0.0 ? 1 : 0;
  a.m = m;
  a.m_next = m_next;
  a.lr = P->lr;
  a.lam = P->prm.lambda;
  a.mu = P->prm.mu;
  a.eps = (float)P->prm.eps;
  a.eps2_normal = a.eps * a.eps >= FLT_MIN ? 1 : 0;
  a.zc = P->zc;
  return a;
}

}  // namespace

extern "C" {

const char* spg_status_string(spg_status s) {
  switch (s) {
    case SPG_OK: return "ok";
    case SPG_E_INVAL: return "invalid argument";
    case SPG_E_NOMEM: return "workspace too small";
    case SPG_E_DEVICE: return "device (HIP) error";
    case SPG_E_STATE: return "call out of order";
    case SPG_E_NONFINITE: return "non-finite input";
    case SPG_E_DIVERGED: return "objective is not finite";
    case SPG_E_UNSUPPORTED: return "unsupported by this build";
  }
  return "unknown status";
}

const char* spg_last_error(const spg_problem* P) { return P ? P->err : "problem is NULL"; }

spg_status spg_workspace_size(const spg_params* p, size_t* bytes) {
  spg_status st;
  if (check_params(p, &st)) return st;
  if (!bytes) return SPG_E_INVAL;
  *bytes = make_layout(*p).total;
  return SPG_OK;
}

spg_status spg_create(const spg_params* p, void* d_workspace, size_t bytes, void* hip_stream, spg_problem** out) {
  spg_status st;
  if (!out) return SPG_E_INVAL;
  *out = nullptr;
  if (check_params(p, &st)) return st;
  if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0) return SPG_E_INVAL;
  const Layout lay = make_layout(*p);
  if (bytes < lay.total) return SPG_E_NOMEM;
  spg_problem* P = new (std::nothrow) spg_problem();
  if (!P) return SPG_E_NOMEM;
  P->prm = *p;
  P->stream = reinterpret_cast<hipStream_t>(hip_stream);
  P->ws = reinterpret_cast<char*>(d_workspace);
  P->ws_bytes = bytes;
  P->lay = lay;
  P->d.nx = p->nx;
  P->d.ny = p->ny;
  P->d.nz = p->nz;
  P->d.P = p->nx / 2;
  P->d.nvox = (long long)p->nx * p->ny * p->nz;
  P->comp = (p->flags & SPG_FLAG_COMPENSATED) != 0;
  P->store = P->comp ? ST_COMP : ((p->flags & SPG_FLAG_BF16_STORAGE) ? ST_BF16 : ST_PLAIN);
  P->dn2 = dnorm2_of(p->nx, p->ny, p->nz);
  P->fused = prox_fft_supported(P->d);
  // z-slab depth of the stencil kernel: 32 planes, or fewer on small maps, whose blocks
  // (ny / 4 tiles per slab) would otherwise be too few to keep more than a few CUs busy and
  // each march through many planes in turn
  while (P->zc > 4 && (long long)(p->ny / 4) * ((p->nz + P->zc - 1) / P->zc) < 512) P->zc /= 2;
  P->mon_every = (p->flags & SPG_FLAG_MONITOR) ? p->obj_every : 0;
  P->hist_iter.assign(kHistCap, 0);
  restart(P);
  *out = P;
  return SPG_OK;
}

spg_status spg_debug_fail_after(spg_problem* P, int32_t n) {
  if (!P || n < -1) return SPG_E_INVAL;
  P->fail_after = n;
  return SPG_OK;
}

spg_status spg_destroy(spg_problem* P) {
  if (!P) return SPG_E_INVAL;
  for (hipEvent_t e : P->ev) (void)hipEventDestroy(e);
  delete P;
  return SPG_OK;
}

spg_status spg_set_data(spg_problem* P, const float* d_w, const float* d_b) {
  spg_status s = usable(P);
  if (s) return s;
  if (!d_w || !d_b) return set_err(P, SPG_E_INVAL, "w and b must be device pointers");
  const Dims& d = P->d;
  const float2* b = reinterpret_cast<const float2*>(d_b);
  double* part = P->part();
  // 1. check the inputs before touching any state
  SPG_CK(P, launch_data_stats(d, d_w, b, part, kStatBlocks, P->stream));
  const int ops5[5] = {RED_OP_SUM, RED_OP_MIN, RED_OP_SUM, RED_OP_SUM, RED_OP_SUM};
  SPG_CK(P, launch_reduce(part, kStatBlocks, 5, ops5, P->res(), P->stream));
  double r[5];
  if ((s = read_results(P, r, 5))) return s;
  if (r[0] > 0) return set_err(P, SPG_E_NONFINITE, "w or b holds NaN/Inf values");
  if (r[1] < 0) return set_err(P, SPG_E_INVAL, "negative Fourier weight");
  // 2. fold onto the packed half spectrum
  SPG_CK(P, launch_fold(d, d_w, b, P->at<float>(P->lay.ws), P->at<float>(P->lay.w0p), P->at<float>(P->lay.wnyq),
                        P->at<float2>(P->lay.cs), P->at<float2>(P->lay.c0p), P->at<float2>(P->lay.cnyq), part,
                        kStatBlocks, P->stream));
  const int ops1[1] = {RED_OP_MAX};
  SPG_CK(P, launch_reduce(part, kStatBlocks, 1, ops1, P->res(), P->stream));
  double mx;
  if ((s = read_results(P, &mx, 1))) return s;
  P->maxwt = mx;
  P->C0 = r[2];
  P->mean_w = r[3] / (double)d.nvox;
  P->rms_unreg = std::sqrt(r[4] / (double)d.nvox);
  P->data_set = true;
  recompute_L(P);
  restart(P);
  if (P->L <= 0) return set_err(P, SPG_E_INVAL, "L = 0: all weights are zero and mu == 0");
  return SPG_OK;
}

spg_status spg_set_penalty_weights(spg_problem* P, const float* d_u, const float* d_v) {
  spg_status s = usable(P);
  if (s) return s;
  double vmax = 1.0;
  const float* arr[2] = {d_u, d_v};
  for (int k = 0; k < 2; ++k) {
    if (!arr[k]) continue;
    SPG_CK(P, launch_weight_stats(P->d, arr[k], P->part(), kStatBlocks, P->stream));
    const int ops[3] = {RED_OP_SUM, RED_OP_MIN, RED_OP_MAX};
    SPG_CK(P, launch_reduce(P->part(), kStatBlocks, 3, ops, P->res(), P->stream));
    double r[3];
    if ((s = read_results(P, r, 3))) return s;
    if (r[0] > 0) return set_err(P, SPG_E_NONFINITE, "penalty weights hold NaN/Inf values");
    if (r[1] < 0) return set_err(P, SPG_E_INVAL, "negative penalty weight");
    if (k == 1) vmax = r[2];
  }
  const size_t bytes = (size_t)P->d.nvox * 4;
  void* dst[2] = {P->at<void>(P->lay.u), P->at<void>(P->lay.v)};
  for (int k = 0; k < 2; ++k) {
    if (!arr[k]) continue;
    if (P->bf()) SPG_CK(P, launch_f32_to_bf16(arr[k], reinterpret_cast<uint16_t*>(dst[k]), P->d.nvox, P->stream));
    else SPG_CK(P, hipMemcpyAsync(dst[k], arr[k], bytes, hipMemcpyDeviceToDevice, P->stream));
  }
  if (P->bf() && d_v) vmax = bf16_round(vmax);  // rounding is monotonic: max of the stored values
  P->unif_u = d_u == nullptr;
  P->unif_v = d_v == nullptr;
  P->vmax = vmax;
  recompute_L(P);
  restart(P);
  return SPG_OK;
}

spg_status spg_set_params(spg_problem* P, double lambda, double mu) {
  spg_status s = usable(P);
  if (s) return s;
  if (!std::isfinite(lambda) || lambda < 0 || !std::isfinite(mu) || mu < 0)
    return set_err(P, SPG_E_INVAL, "lambda and mu must be finite and >= 0");
  P->prm.lambda = lambda;
  P->prm.mu = mu;
  recompute_L(P);
  restart(P);
  return SPG_OK;
}

spg_status spg_set_prior(spg_problem* P, double gamma, const float* d_xprev) {
  spg_status s = usable(P);
  if (s) return s;
  if (!std::isfinite(gamma) || gamma < 0) return set_err(P, SPG_E_INVAL, "gamma must be finite and >= 0");
  if (d_xprev)
    SPG_CK(P, hipMemcpyAsync(P->at<float>(P->lay.xprev), d_xprev, (size_t)P->d.nvox * 4, hipMemcpyDeviceToDevice,
                             P->stream));
  P->prior_set = d_xprev != nullptr;
  P->prm.gamma = gamma;
  recompute_L(P);
  restart(P);
  return SPG_OK;
}

spg_status spg_set_map(spg_problem* P, const float* d_x0) {
  spg_status s = usable(P);
  if (s) return s;
  // the iterate ring restarts at slot 0, so that every solve from a set map launches the same
  // kernels (a batch graph captured after one spg_set_map is replayed after the next)
  SPG_CK(P, launch_set_map(P->d, d_x0, P->xhi(0), P->xlo(0), P->stream));
  P->cur = 0;
  P->old = 1;
  restart(P);
  return SPG_OK;
}

// One SPG iteration; with capture_g, the data gradient of y_k is also copied there (fp32).
static spg_status iterate_once(spg_problem* P, float* capture_g) {
  spg_status s;
  const Dims& d = P->d;
  {
    if (!P->primed) {
      SPG_CK(P, launch_prime(d, P->rbuf(), P->xhi(P->cur), P->xlo(P->cur), P->xhi(P->old), P->xlo(P->old),
                             P->m_cur, P->m_cur != 0.0, P->store, P->stream));
      if ((s = r2c(P, P->rbuf(), P->bf()))) return s;
      P->primed = true;
    }
    const bool fuse = P->fused && !capture_g;
    // the objective monitor: F_eps(y_j) from partials of the z pass, the kx = 0 / nx/2 plane
    // and the stencil kernel of this iteration
    const bool mon = P->mon_every > 0 && !capture_g && P->j % P->mon_every == 0;
    int nA = 0, nB = 0, nC = 0;
    if ((s = gradient_pipeline(P, mon, &nA, &nB, P->rbuf(), P->bf(), !fuse))) return s;
    if (capture_g)
      SPG_CK(P, hipMemcpyAsync(capture_g, P->rbuf(), (size_t)d.nvox * 4, hipMemcpyDeviceToDevice, P->stream));
    const double t_next = P->prm.accel ? 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * P->t * P->t)) : 1.0;
    const double m_next = P->prm.accel ? (P->t - 1.0) / t_next : 0.0;
    const int nxt = 3 - P->cur - P->old;
    ProxArgs a = prox_args(P, nxt, P->m_cur, m_next);
    if (mon) {
      // 3 partials per block in region C (<= 3 x 65536; the slab depth does not change results)
      a.partials = P->part() + kPartC;
      if (fuse) {
        nC = prox_fft_num_blocks(d, a.zc);
      } else {
        while (prox_num_blocks(d, a.zc) > 65536) a.zc *= 2;
        nC = prox_num_blocks(d, a.zc);
      }
    }
    prof_begin(P, SPG_KERNEL_PROX_TV);
    if (fuse) {
      SPG_CK(P, launch_prox_fft(d, a, P->S(), P->at<float2>(P->lay.tw_m), P->at<float2>(P->lay.tw_n), P->store,
                                P->stream, mon));
    } else {
      SPG_CK(P, launch_prox_tv(d, a, P->store, false, P->stream, mon));
    }
    prof_end(P, SPG_KERNEL_PROX_TV);
    if (mon) {
      const int slot = (int)(P->hist_n % kHistCap);
      SPG_CK(P, launch_obj_finish(P->part() + kPartA, nA, P->part() + kPartB, nB, P->part() + kPartC, nC, P->C0,
                                  P->prm.lambda, P->prm.mu, P->prm.gamma, P->at<double>(P->lay.hist) + slot,
                                  P->stream));
      P->hist_iter[slot] = P->iters_done + 1;
      ++P->hist_n;
    }
    if (!fuse && (s = r2c(P, P->rbuf(), P->bf()))) return s;
    P->old = P->cur;
    P->cur = nxt;
    P->t = t_next;
    P->m_cur = m_next;
    ++P->j;
    ++P->iters_done;
  }
  return SPG_OK;
}

spg_status spg_run(spg_problem* P, int32_t K, spg_stats* stats) {
  spg_status s = usable(P);
  if (s) return s;
  if (K < 0) return set_err(P, SPG_E_INVAL, "K must be >= 0");
  if (!P->data_set) return set_err(P, SPG_E_STATE, "spg_set_data has not succeeded");
  if (!(P->L > 0)) return set_err(P, SPG_E_STATE, "L = 0");
  P->vjp_valid = false;
  for (int it = 0; it < K; ++it)
    if ((s = iterate_once(P, nullptr))) return s;
  if (stats) {
    stats->iters_done = P->iters_done;
    stats->round = P->round;
    stats->iter_in_round = P->j - 1;
    stats->lr = P->lr;
    stats->L = P->L;
    stats->obj_smoothed = std::numeric_limits<double>::quiet_NaN();
    stats->obj_iter = 0;
    if (P->mon_every > 0 && P->hist_n > 0) {
      const int slot = (int)((P->hist_n - 1) % kHistCap);
      double v;
      if ((s = read_results_to(P, P->at<double>(P->lay.hist) + slot, &v, 1))) return s;
      stats->obj_smoothed = v;
      stats->obj_iter = P->hist_iter[slot];
      if (!std::isfinite(v)) return set_err(P, SPG_E_DIVERGED, "the monitored objective is not finite");
    }
  }
  return SPG_OK;
}

spg_status spg_objective_history(spg_problem* P, double* h_values, int64_t* h_iters, int32_t cap, int32_t* n_out) {
  spg_status s = usable(P);
  if (s) return s;
  if (!n_out || cap < 0 || (cap > 0 && !h_values && !h_iters))
    return set_err(P, SPG_E_INVAL, "n_out must be given; cap >= 0 with an output array");
  const int64_t avail = P->hist_n < kHistCap ? P->hist_n : kHistCap;
  const int n = (int)(avail < cap ? avail : cap);
  *n_out = n;
  if (n == 0) return SPG_OK;
  std::vector<double> ring(kHistCap);
  if ((s = read_results_to(P, P->at<double>(P->lay.hist), ring.data(), kHistCap))) return s;
  for (int i = 0; i < n; ++i) {  // the n most recent entries, oldest first
    const int slot = (int)((P->hist_n - n + i) % kHistCap);
    if (h_values) h_values[i] = ring[slot];
    if (h_iters) h_iters[i] = P->hist_iter[slot];
  }
  return SPG_OK;
}

spg_status spg_reweight(spg_problem* P, double eps1, double eps2) {
  spg_status s = usable(P);
  if (s) return s;
  if (!std::isfinite(eps1) || !std::isfinite(eps2) || eps1 <= 0 || eps2 <= 0)
    return set_err(P, SPG_E_INVAL, "eps1 and eps2 must be finite and > 0");
  SPG_CK(P, launch_reweight(P->d, P->xhi(P->cur), P->xlo(P->cur), P->at<void>(P->lay.u), P->at<void>(P->lay.v),
                            eps1, eps2, P->store, P->part(), kStatBlocks, P->stream));
  const int ops[1] = {RED_OP_MAX};
  SPG_CK(P, launch_reduce(P->part(), kStatBlocks, 1, ops, P->res(), P->stream));
  double vmax;
  if ((s = read_results(P, &vmax, 1))) return s;
  P->unif_u = false;
  P->unif_v = false;
  P->vmax = vmax;
  ++P->round;
  recompute_L(P);
  restart(P);
  return SPG_OK;
}

spg_status spg_get_map(spg_problem* P, float* d_x_out) {
  spg_status s = usable(P);
  if (s) return s;
  if (!d_x_out) return set_err(P, SPG_E_INVAL, "output pointer is NULL");
  SPG_CK(P, launch_get_map(P->d, P->xhi(P->cur), P->xlo(P->cur), d_x_out, P->comp, P->stream));
  return SPG_OK;
}

spg_status spg_get_penalty_weights(spg_problem* P, float* d_u_out, float* d_v_out) {
  spg_status s = usable(P);
  if (s) return s;
  const size_t bytes = (size_t)P->d.nvox * 4;
  float* outs[2] = {d_u_out, d_v_out};
  const bool unif[2] = {P->unif_u, P->unif_v};
  const size_t offs[2] = {P->lay.u, P->lay.v};
  for (int k = 0; k < 2; ++k) {
    if (!outs[k]) continue;
    if (unif[k]) SPG_CK(P, launch_fill(outs[k], P->d.nvox, 1.0f, P->stream));
    else if (P->bf()) SPG_CK(P, launch_bf16_to_f32(P->at<uint16_t>(offs[k]), outs[k], P->d.nvox, P->stream));
    else SPG_CK(P, hipMemcpyAsync(outs[k], P->at<float>(offs[k]), bytes, hipMemcpyDeviceToDevice, P->stream));
  }
  return SPG_OK;
}

spg_status spg_final_check(spg_problem* P, double* F_eps, double* F_0, double* kkt_rel) {
  spg_status s = usable(P);
  if (s) return s;
  if (!P->data_set) return set_err(P, SPG_E_STATE, "spg_set_data has not succeeded");
  const Dims& d = P->d;
  // The check runs in fp32 in every storage mode: the forward transform reads the fp32 (hi)
  // words of x, and the data gradient goes to the spare ring slot as fp32.
  const int spare = 3 - P->cur - P->old;
  P->primed = false;
  if ((s = r2c(P, P->xhi(P->cur), false))) return s;
  int nA = 0, nB = 0;
  if ((s = gradient_pipeline(P, true, &nA, &nB, P->xhi(spare), false))) return s;
  ProxArgs a = prox_args(P, P->cur, 0.0, 0.0);
  a.read_old = 0;
  a.gin = P->xhi(spare);
  // check-mode partials: 6 per block, at most 8192 blocks
  while (prox_num_blocks(d, a.zc) > 8192) a.zc *= 2;
  const int nC = prox_num_blocks(d, a.zc);
  a.partials = P->part() + kPartC;
  prof_begin(P, SPG_KERNEL_PROX_TV);
  SPG_CK(P, launch_prox_tv(d, a, P->store, true, P->stream));
  prof_end(P, SPG_KERNEL_PROX_TV);
  const int sum1[1] = {RED_OP_SUM};
  const int sum6[6] = {RED_OP_SUM, RED_OP_SUM, RED_OP_SUM, RED_OP_SUM, RED_OP_SUM, RED_OP_SUM};
  SPG_CK(P, launch_reduce(P->part() + kPartA, nA, 1, sum1, P->res() + 0, P->stream));
  SPG_CK(P, launch_reduce(P->part() + kPartB, nB, 1, sum1, P->res() + 1, P->stream));
  SPG_CK(P, launch_reduce(P->part() + kPartC, nC, 6, sum6, P->res() + 2, P->stream));
  double r[8];
  if ((s = read_results(P, r, 8))) return s;
  const double data = P->C0 + r[0] + r[1];
  const double prior = P->prm.gamma * r[7];
  const double fe = data + P->prm.lambda * r[2] + P->prm.mu * r[3] + prior;
  const double f0 = data + P->prm.lambda * r[2] + P->prm.mu * r[4] + prior;
  const double kkt = std::sqrt(r[5]) / (r[6] > 0 ? std::sqrt(r[6]) : 1.0);
  if (F_eps) *F_eps = fe;
  if (F_0) *F_0 = f0;
  if (kkt_rel) *kkt_rel = kkt;
  if (!std::isfinite(fe)) return set_err(P, SPG_E_DIVERGED, "objective is not finite");
  return SPG_OK;
}

spg_status spg_param_scales(const spg_problem* P, double* rms_unreg, double* mean_w) {
  if (!P) return SPG_E_INVAL;
  if (!P->data_set) return SPG_E_STATE;
  if (rms_unreg) *rms_unreg = P->rms_unreg;
  if (mean_w) *mean_w = P->mean_w;
  return SPG_OK;
}

spg_status spg_suggest_params(const spg_problem* P, double eps1, double eps2, double* lambda, double* mu,
                              double* gamma) {
  if (!P) return SPG_E_INVAL;
  if (!std::isfinite(eps1) || !std::isfinite(eps2) || eps1 <= 0 || eps2 <= 0) return SPG_E_INVAL;
  if (!P->data_set) return SPG_E_STATE;
  if (lambda) *lambda = P->rms_unreg * eps1;
  if (mu) *mu = P->rms_unreg * eps2;
  if (gamma) *gamma = P->mean_w;
  return SPG_OK;
}

spg_status spg_log_objective(spg_problem* P, double eps1, double eps2, double* G) {
  spg_status s = usable(P);
  if (s) return s;
  if (!G) return set_err(P, SPG_E_INVAL, "output pointer is NULL");
  if (!std::isfinite(eps1) || !std::isfinite(eps2) || eps1 <= 0 || eps2 <= 0)
    return set_err(P, SPG_E_INVAL, "eps1 and eps2 must be finite and > 0");
  if (!P->data_set) return set_err(P, SPG_E_STATE, "spg_set_data has not succeeded");
  // data term as in spg_final_check (fp32 transforms of the hi words, fp64 partials); the
  // gradient it also forms goes to the spare ring slot
  const int spare = 3 - P->cur - P->old;
  P->primed = false;
  if ((s = r2c(P, P->xhi(P->cur), false))) return s;
  int nA = 0, nB = 0;
  if ((s = gradient_pipeline(P, true, &nA, &nB, P->xhi(spare), false))) return s;
  SPG_CK(P, launch_log_terms(P->d, P->xhi(P->cur), P->xlo(P->cur), eps1, eps2, P->comp, P->part() + kPartC,
                             kStatBlocks, P->stream));
  const int sum1[1] = {RED_OP_SUM};
  const int sum2[2] = {RED_OP_SUM, RED_OP_SUM};
  SPG_CK(P, launch_reduce(P->part() + kPartA, nA, 1, sum1, P->res() + 0, P->stream));
  SPG_CK(P, launch_reduce(P->part() + kPartB, nB, 1, sum1, P->res() + 1, P->stream));
  SPG_CK(P, launch_reduce(P->part() + kPartC, kStatBlocks, 2, sum2, P->res() + 2, P->stream));
  double r[4];
  if ((s = read_results(P, r, 4))) return s;
  *G = P->C0 + r[0] + r[1] + P->prm.lambda * r[2] + P->prm.mu * r[3];
  if (!std::isfinite(*G)) return set_err(P, SPG_E_DIVERGED, "log objective is not finite");
  return SPG_OK;
}

// ---------------------------------------------------------------- Fourier shell correlation

namespace {
constexpr int kFscBlocks = 256;

struct FscLayout {
  size_t S1, S2, tw_m, tw_n, tw_y, tw_z, part, out, total;
};

FscLayout fsc_layout(int nx, int ny, int nz, int nshells) {
  FscLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t spec = (size_t)nz * ny * (nx / 2) * 8;
  L.S1 = take(spec);
  L.S2 = take(spec);
  L.tw_m = take((size_t)(nx / 2) * 8);
  L.tw_n = take((size_t)nx * 8);
  L.tw_y = take((size_t)ny * 8);
  L.tw_z = take((size_t)nz * 8);
  L.part = take((size_t)kFscBlocks * 3 * nshells * 8);
  L.out = take((size_t)3 * nshells * 8);
  L.total = off;
  return L;
}

bool fsc_args_ok(int nx, int ny, int nz, int nshells) {
  return axis_ok(nx) && axis_ok(ny) && axis_ok(nz) && nshells >= 1 && nshells <= 1024;
}

// exp(-2 pi i m / n), m < n, computed in fp64 and rounded once
void twiddle_table(int n, std::vector<float2>& tab) {
  tab.resize(n);
  for (int m = 0; m < n; ++m) {
    const double ang = -2.0 * M_PI * (double)m / (double)n;
    tab[m] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
}

// Both maps to the packed half spectrum (x, y, z transforms), the shell sums and the ratio
// of eq 30.  ws holds the spectra, partials and output at the offsets of lay; tw[4] are the
// twiddle tables of nx/2, nx, ny and nz points.  Synchronises the stream.
spg_status fsc_run(int nx, int ny, int nz, const float* d_map1, const float* d_map2, int nshells, char* ws,
                   const FscLayout& lay, const float2* const tw[4], hipStream_t st, double* h_fsc) {
  Dims d{nx, ny, nz, nx / 2, (long long)nx * ny * nz};
  const float* maps[2] = {d_map1, d_map2};
  float2* specs[2] = {reinterpret_cast<float2*>(ws + lay.S1), reinterpret_cast<float2*>(ws + lay.S2)};
  for (int k = 0; k < 2; ++k) {
    if (launch_r2c_x(d, maps[k], false, specs[k], tw[0], tw[1], st) != hipSuccess) return SPG_E_DEVICE;
    if (launch_fft_cols(d, specs[k], 1, 0, tw[2], nullptr, nullptr, nullptr, st, nullptr) != hipSuccess)
      return SPG_E_DEVICE;
    if (launch_fft_cols(d, specs[k], 2, 0, tw[3], nullptr, nullptr, nullptr, st, nullptr) != hipSuccess)
      return SPG_E_DEVICE;
  }
  double* out = reinterpret_cast<double*>(ws + lay.out);
  if (launch_fsc_shells(d, specs[0], specs[1], nshells, reinterpret_cast<double*>(ws + lay.part), kFscBlocks, out,
                        st) != hipSuccess)
    return SPG_E_DEVICE;
  double h[3 * 1024];
  if (hipMemcpyAsync(h, out, 3 * (size_t)nshells * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SPG_E_DEVICE;
  for (int sidx = 0; sidx < nshells; ++sidx) {
    const double den = std::sqrt(h[nshells + sidx] * h[2 * nshells + sidx]);
    h_fsc[sidx] = den > 0 ? h[sidx] / den : 0.0;
  }
  return SPG_OK;
}

// ---- the FSC entry point that allocates nothing
// Its workspace is the static device array below: a region with the twiddle tables of every
// supported axis length (written once per device by the first call there), then the FSC
// workspace of one call.  In host code the array's name is only a stand-in; the device
// address comes from hipGetSymbolAddress, once per device, and is the only one used.
constexpr size_t kNoallocTables = 64 * 1024;
constexpr size_t kNoallocBytes = 72ull << 20;
// axis lengths with a table (nx/2 of the supported nx included) and their offsets in bytes
constexpr int kTwLens[] = {2, 4, 8, 16, 32, 64, 128, 256, 512, 80, 96, 160, 192};
constexpr int kNumTwLens = sizeof(kTwLens) / sizeof(kTwLens[0]);

constexpr size_t noalloc_table_offset(int n) {
  size_t off = 0;
  for (int i = 0; i < kNumTwLens; ++i) {
    if (kTwLens[i] == n) return off;
    off = (off + (size_t)kTwLens[i] * 8 + kAlign - 1) / kAlign * kAlign;
  }
  return off;  // past the last table: the size of the table region
}
static_assert(noalloc_table_offset(0) <= kNoallocTables, "twiddle tables outgrow their region");

std::mutex g_noalloc_mu;
std::vector<char*> g_noalloc_base;  // per device: the address of the array, null until set up
}  // namespace

static __device__ __align__(256) char scratch[kNoallocBytes];

namespace {
// The device address of the array on the current device; the first call on a device looks
// it up and writes the twiddle tables (synchronising hip_stream).
spg_status noalloc_base(hipStream_t st, char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return SPG_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if ((int)g_noalloc_base.size() <= dev) g_noalloc_base.resize(dev + 1, nullptr);
  if (!g_noalloc_base[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SPG_E_DEVICE;
    char* base = reinterpret_cast<char*>(ptr);
    std::vector<float2> tab;
    for (int i = 0; i < kNumTwLens; ++i) {
      twiddle_table(kTwLens[i], tab);
      if (hipMemcpyAsync(base + noalloc_table_offset(kTwLens[i]), tab.data(), tab.size() * sizeof(float2),
                         hipMemcpyHostToDevice, st) != hipSuccess)
        return SPG_E_DEVICE;
    }
    if (hipStreamSynchronize(st) != hipSuccess) return SPG_E_DEVICE;
    g_noalloc_base[dev] = base;
  }
  *out = g_noalloc_base[dev];
  return SPG_OK;
}
}  // namespace

extern "C" {

spg_status spg_fsc_noalloc(int32_t nx, int32_t ny, int32_t nz, const float* d_map1, const float* d_map2,
                           int32_t nshells, void* hip_stream, double* h_fsc) {
  if (!fsc_args_ok(nx, ny, nz, nshells) || !d_map1 || !d_map2 || !h_fsc) return SPG_E_INVAL;
  const FscLayout lay = fsc_layout(nx, ny, nz, nshells);
  if (lay.total > kNoallocBytes - kNoallocTables) return SPG_E_NOMEM;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  char* base = nullptr;
  spg_status s = noalloc_base(st, &base);
  if (s) return s;
  const int lens[4] = {nx / 2, nx, ny, nz};
  const float2* tw[4];
  for (int t = 0; t < 4; ++t) tw[t] = reinterpret_cast<const float2*>(base + noalloc_table_offset(lens[t]));
  return fsc_run(nx, ny, nz, d_map1, d_map2, nshells, base + kNoallocTables, lay, tw, st, h_fsc);
}

spg_status spg_fsc_workspace_size(int32_t nx, int32_t ny, int32_t nz, int32_t nshells, size_t* bytes) {
  if (!bytes || !fsc_args_ok(nx, ny, nz, nshells)) return SPG_E_INVAL;
  *bytes = fsc_layout(nx, ny, nz, nshells).total;
  return SPG_OK;
}

spg_status spg_fsc(int32_t nx, int32_t ny, int32_t nz, const float* d_map1, const float* d_map2, int32_t nshells,
                   void* d_workspace, size_t bytes, void* hip_stream, double* h_fsc) {
  if (!fsc_args_ok(nx, ny, nz, nshells) || !d_map1 || !d_map2 || !h_fsc || !d_workspace ||
      (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
    return SPG_E_INVAL;
  const FscLayout lay = fsc_layout(nx, ny, nz, nshells);
  if (bytes < lay.total) return SPG_E_NOMEM;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  char* ws = reinterpret_cast<char*>(d_workspace);
  const int lens[4] = {nx / 2, nx, ny, nz};
  const size_t offs[4] = {lay.tw_m, lay.tw_n, lay.tw_y, lay.tw_z};
  std::vector<float2> tab;
  const float2* tw[4];
  for (int t = 0; t < 4; ++t) {
    twiddle_table(lens[t], tab);
    if (hipMemcpyAsync(ws + offs[t], tab.data(), lens[t] * sizeof(float2), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return SPG_E_DEVICE;
    tw[t] = reinterpret_cast<const float2*>(ws + offs[t]);
  }
  return fsc_run(nx, ny, nz, d_map1, d_map2, nshells, ws, lay, tw, st, h_fsc);
}

}  // extern "C"

// ---------------------------------------------------------------- launch-shape autotuner

extern "C" {

spg_status spg_set_launch_shape(spg_problem* P, int32_t nt_y, int32_t nt_z, int32_t zc) {
  spg_status s = usable(P);
  if (s) return s;
  if ((nt_y != 8 && nt_y != 16) || (nt_z != 8 && nt_z != 16) || zc < 4 || zc > 512)
    return set_err(P, SPG_E_INVAL, "nt_y, nt_z must be 8 or 16 and zc in [4, 512]");
  P->nt_y = nt_y;
  P->nt_z = nt_z;
  P->zc = zc;
  return SPG_OK;
}

spg_status spg_set_fusion(spg_problem* P, int32_t enable) {
  spg_status s = usable(P);
  if (s) return s;
  if (enable && !prox_fft_supported(P->d))
    return set_err(P, SPG_E_UNSUPPORTED, "fused x transforms need nx in {64, 128, 256, 512} and ny % 4 == 0");
  P->fused = enable != 0;
  return SPG_OK;
}

spg_status spg_get_fusion(const spg_problem* P, int32_t* enabled) {
  if (!P || !enabled) return SPG_E_INVAL;
  *enabled = P->fused ? 1 : 0;
  return SPG_OK;
}

spg_status spg_get_launch_shape(const spg_problem* P, int32_t* nt_y, int32_t* nt_z, int32_t* zc) {
  if (!P) return SPG_E_INVAL;
  if (nt_y) *nt_y = P->nt_y;
  if (nt_z) *nt_z = P->nt_z;
  if (zc) *zc = P->zc;
  return SPG_OK;
}

spg_status spg_autotune(spg_problem* P, int32_t iters) {
  spg_status s = usable(P);
  if (s) return s;
  if (iters < 1 || iters > 1000) return set_err(P, SPG_E_INVAL, "iters must be in [1, 1000]");
  if (!P->data_set) return set_err(P, SPG_E_STATE, "spg_set_data has not succeeded");
  if (P->prof_on) return set_err(P, SPG_E_STATE, "profiling is active");
  // coordinate search: for each knob, time the kernel classes it changes over `iters`
  // iterations from the zero map for every candidate and keep the fastest.  The fusion
  // knob (where the fused path is on) compares the fused stencil/prox kernel with the
  // stencil kernel plus the separate x-axis sweeps; a path set off stays off.
  struct Knob {
    int* val;
    std::vector<int> cls;
    std::vector<int> cand;
  };
  int fused = P->fused ? 1 : 0;
  std::vector<Knob> knobs = {{&P->nt_y, {SPG_KERNEL_FFT_Y_FWD}, {16, 8}},
                             {&P->nt_z, {SPG_KERNEL_FFT_Z_WEIGHT}, {16, 8}}};
  if (P->fused) knobs.push_back({&fused, {SPG_KERNEL_PROX_TV, SPG_KERNEL_C2R_X, SPG_KERNEL_R2C_X}, {1, 0}});
  knobs.push_back({&P->zc, {SPG_KERNEL_PROX_TV}, {32, 16, 64, 128, 256, 8, 4}});
  // Each candidate is timed twice, in two sweeps over the candidates, and keeps the faster of
  // its two times, so that one slow sample on a busy GPU does not decide.  A pass may be
  // launched as several column ranges: the event capacity covers four launches per class
  // and iteration.
  for (Knob& kb : knobs) {
    std::vector<double> t_min(kb.cand.size(), 1e300);
    std::vector<bool> ran(kb.cand.size(), false);
    for (int sweep = 0; sweep < 2; ++sweep) {
      for (size_t ci = 0; ci < kb.cand.size(); ++ci) {
        *kb.val = kb.cand[ci];
        P->fused = fused != 0;
        if ((s = spg_set_map(P, nullptr))) return s;
        // warm, and past the first two iterations of a round (zero momentum: x_{k-1} unread)
        if ((s = spg_run(P, 3, nullptr))) return s;
        if ((s = spg_profile_begin(P, SPG_KERNEL_ALL, 4 * iters + 4))) return s;
        if ((s = spg_run(P, iters, nullptr))) return s;
        double ms[SPG_KERNEL_COUNT];
        int32_t n[SPG_KERNEL_COUNT];
        if ((s = spg_profile_end(P, ms, n))) return s;
        double t = 0.0;
        int launched = 0;
        for (int k : kb.cls) {
          t += ms[k];
          launched += n[k];
        }
        if (launched > 0) {
          ran[ci] = true;
          t_min[ci] = std::min(t_min[ci], t);
        }
      }
    }
    int best = *kb.val;
    double best_ms = 1e300;
    for (size_t ci = 0; ci < kb.cand.size(); ++ci)
      if (ran[ci] && t_min[ci] < best_ms) {
        best_ms = t_min[ci];
        best = kb.cand[ci];
      }
    *kb.val = best;
    P->fused = fused != 0;
  }
  return spg_set_map(P, nullptr);
}

}  // extern "C"

// ---------------------------------------------------------------- batches in one HIP graph

// Host state of a problem that the kernels of its next iterations depend on (launch
// arguments: buffers, momenta, step, shapes, paths), and the part of it that advances.
struct IterSig {
  spg_params prm;
  int store, cur, old, nt_y, nt_z, zc;
  bool prior_set, primed, unif_u, unif_v, fused;
  double lr, t, m_cur;
  int32_t j;
  int64_t hist_n;  // a graph with monitored iterations writes fixed history slots
  static IterSig of(const spg_problem* P) {
    IterSig g;
    g.prm = P->prm;
    g.store = P->store;
    g.cur = P->cur;
    g.old = P->old;
    g.nt_y = P->nt_y;
    g.nt_z = P->nt_z;
    g.zc = P->zc;
    g.prior_set = P->prior_set;
    g.primed = P->primed;
    g.unif_u = P->unif_u;
    g.unif_v = P->unif_v;
    g.fused = P->fused;
    g.lr = P->lr;
    g.t = P->t;
    g.m_cur = P->m_cur;
    g.j = P->j;
    g.hist_n = P->hist_n;
    return g;
  }
  bool operator==(const IterSig& o) const {
    const spg_params& a = prm;
    const spg_params& b = o.prm;
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.lambda == b.lambda && a.mu == b.mu && a.eps == b.eps &&
           a.gamma == b.gamma && a.accel == b.accel && a.flags == b.flags && a.obj_every == b.obj_every &&
           hist_n == o.hist_n && store == o.store && cur == o.cur &&
           old == o.old && nt_y == o.nt_y && nt_z == o.nt_z && zc == o.zc && prior_set == o.prior_set &&
           primed == o.primed && unif_u == o.unif_u && unif_v == o.unif_v && fused == o.fused && lr == o.lr &&
           t == o.t && m_cur == o.m_cur && j == o.j;
  }
};

struct spg_batch {
  std::vector<spg_problem*> probs;
  // the instantiated graph is launched again without a new capture when every member is
  // in the state it was captured from (same K): then the members advance to `post`
  int32_t K_graph = 0;
  std::vector<IterSig> pre, post;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr, done = nullptr;
  hipStream_t origin = nullptr;  // capture and launch stream (the legacy default stream cannot capture)
  hipStream_t user = nullptr;    // the caller's stream, which waits for every graph
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
};

namespace {
void batch_release_graph(spg_batch* B) {
  if (B->exec) {
    (void)hipStreamSynchronize(B->origin);
    (void)hipGraphExecDestroy(B->exec);
    B->exec = nullptr;
  }
  if (B->graph) {
    (void)hipGraphDestroy(B->graph);
    B->graph = nullptr;
  }
}

// Capture K iterations of every member as parallel branches of one graph (each member on
// its own capture stream, forked from and joined into the origin stream), instantiate it,
// launch it, and record the members' states before and after for later replays.
spg_status batch_capture_and_launch(spg_batch* B, int32_t K) {
  const int n = (int)B->probs.size();
  batch_release_graph(B);
  B->pre.resize(n);
  B->post.resize(n);
  for (int i = 0; i < n; ++i) B->pre[i] = IterSig::of(B->probs[i]);
  std::vector<hipStream_t> saved(n);
  auto fail = [&](hipError_t e, const char* what) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(B->origin, &g);
    if (g) (void)hipGraphDestroy(g);
    for (int i = 0; i < n; ++i)
      if (saved[i]) B->probs[i]->stream = saved[i];
    for (spg_problem* P : B->probs) {
      P->shared_gpu = false;
      P->sticky = true;  // host state advanced past the device
    }
    return fail_device(B->probs[0], e, what);
  };
  hipError_t e = hipStreamBeginCapture(B->origin, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return fail_device(B->probs[0], e, "hipStreamBeginCapture");
  if ((e = hipEventRecord(B->fork, B->origin)) != hipSuccess) return fail(e, "hipEventRecord");
  for (int i = 0; i < n; ++i) {
    spg_problem* P = B->probs[i];
    if ((e = hipStreamWaitEvent(B->streams[i], B->fork, 0)) != hipSuccess) return fail(e, "hipStreamWaitEvent");
    saved[i] = P->stream;
    P->stream = B->streams[i];
    P->vjp_valid = false;
    // the members' kernels run side by side: no persistent grids that each fill the GPU
    P->shared_gpu = true;
    for (int it = 0; it < K; ++it)
      if (iterate_once(P, nullptr) != SPG_OK) return fail(hipErrorUnknown, P->err);
    P->shared_gpu = false;
    if ((e = hipEventRecord(B->join[i], B->streams[i])) != hipSuccess) return fail(e, "hipEventRecord");
    if ((e = hipStreamWaitEvent(B->origin, B->join[i], 0)) != hipSuccess) return fail(e, "hipStreamWaitEvent");
  }
  e = hipStreamEndCapture(B->origin, &B->graph);
  for (int i = 0; i < n; ++i) B->probs[i]->stream = saved[i];
  if (e != hipSuccess) {
    for (spg_problem* P : B->probs) P->sticky = true;
    return fail_device(B->probs[0], e, "hipStreamEndCapture");
  }
  if ((e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0)) != hipSuccess ||
      (e = hipGraphLaunch(B->exec, B->origin)) != hipSuccess || (e = hipEventRecord(B->done, B->origin)) != hipSuccess) {
    for (spg_problem* P : B->probs) P->sticky = true;
    return fail_device(B->probs[0], e, "graph launch");
  }
  for (int i = 0; i < n; ++i) B->post[i] = IterSig::of(B->probs[i]);
  B->K_graph = K;
  return SPG_OK;
}
}  // namespace

extern "C" {

spg_status spg_batch_create(spg_problem* const* problems, int32_t n, void* hip_stream, spg_batch** out) {
  if (!out || !problems || n < 1 || n > 64) return SPG_E_INVAL;
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!problems[i]) return SPG_E_INVAL;
    for (int j = 0; j < i; ++j)
      if (problems[j] == problems[i]) return SPG_E_INVAL;
  }
  spg_batch* B = new (std::nothrow) spg_batch();
  if (!B) return SPG_E_NOMEM;
  B->probs.assign(problems, problems + n);
  B->user = reinterpret_cast<hipStream_t>(hip_stream);
  bool ok = hipStreamCreateWithFlags(&B->origin, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&B->fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&B->done, hipEventDisableTiming) == hipSuccess;
  B->streams.assign(n, nullptr);
  B->join.assign(n, nullptr);
  for (int i = 0; ok && i < n; ++i)
    ok = hipStreamCreateWithFlags(&B->streams[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&B->join[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    spg_batch_destroy(B);
    return SPG_E_DEVICE;
  }
  *out = B;
  return SPG_OK;
}

spg_status spg_batch_destroy(spg_batch* B) {
  if (!B) return SPG_E_INVAL;
  batch_release_graph(B);
  for (hipStream_t s : B->streams)
    if (s) (void)hipStreamDestroy(s);
  for (hipEvent_t e : B->join)
    if (e) (void)hipEventDestroy(e);
  if (B->fork) (void)hipEventDestroy(B->fork);
  if (B->done) (void)hipEventDestroy(B->done);
  if (B->origin) (void)hipStreamDestroy(B->origin);
  delete B;
  return SPG_OK;
}

spg_status spg_batch_run(spg_batch* B, int32_t K) {
  if (!B || K < 0) return SPG_E_INVAL;
  for (spg_problem* P : B->probs) {
    spg_status s = usable(P);
    if (s) return s;
    if (!P->data_set || !(P->L > 0)) return set_err(P, SPG_E_STATE, "spg_set_data has not succeeded");
    if (P->prof_on) return set_err(P, SPG_E_STATE, "profiling is active");
  }
  if (K == 0) return SPG_OK;
  const int n = (int)B->probs.size();
  // inputs set on the problems' own streams and the caller's stream must be complete
  // before the graph starts
  for (spg_problem* P : B->probs)
    if (hipStreamSynchronize(P->stream) != hipSuccess) return fail_device(P, hipErrorUnknown, "stream sync");
  if (hipStreamSynchronize(B->user) != hipSuccess) return fail_device(B->probs[0], hipErrorUnknown, "stream sync");
  bool replay = B->exec && K == B->K_graph && (int)B->pre.size() == n;
  for (int i = 0; replay && i < n; ++i) replay = IterSig::of(B->probs[i]) == B->pre[i];
  hipError_t e;
  if (replay) {
    if ((e = hipGraphLaunch(B->exec, B->origin)) != hipSuccess || (e = hipEventRecord(B->done, B->origin)) != hipSuccess) {
      for (spg_problem* P : B->probs) P->sticky = true;
      return fail_device(B->probs[0], e, "graph launch");
    }
    for (int i = 0; i < n; ++i) {
      spg_problem* P = B->probs[i];
      const IterSig& g = B->post[i];
      P->primed = g.primed;
      P->cur = g.cur;
      P->old = g.old;
      P->t = g.t;
      P->m_cur = g.m_cur;
      P->j = g.j;
      P->iters_done += K;
      P->vjp_valid = false;
    }
  } else {
    spg_status s = batch_capture_and_launch(B, K);
    if (s) return s;
  }
  // later work on each problem's own stream and on the caller's stream starts after the graph
  for (spg_problem* P : B->probs)
    if ((e = hipStreamWaitEvent(P->stream, B->done, 0)) != hipSuccess) return fail_device(P, e, "hipStreamWaitEvent");
  if ((e = hipStreamWaitEvent(B->user, B->done, 0)) != hipSuccess) return fail_device(B->probs[0], e, "hipStreamWaitEvent");
  return SPG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- reverse pass (adjoint)

namespace {
struct VjpLayout {
  size_t ck, ck_slot, seg_x, seg_g, abar, zbar, hz, rbar, part, res, total;
  int nseg;
};

VjpLayout vjp_layout(const spg_problem* P, int K, int C) {
  VjpLayout L{};
  const size_t n4 = align_up((size_t)P->d.nvox * 4);
  const size_t n2 = P->comp ? align_up((size_t)P->d.nvox * 2) : 0;
  L.nseg = (K + C - 1) / C;
  L.ck_slot = 2 * (n4 + n2);  // (x_j, x_{j-1}) as hi (+ lo) words
  size_t off = 0;
  L.ck = off;
  off += (size_t)(L.nseg + 1) * L.ck_slot;
  L.seg_x = off;
  off += (size_t)(C + 2) * n4;
  L.seg_g = off;
  off += (size_t)C * n4;
  L.abar = off;
  off += 3 * n4;
  L.zbar = off;
  off += n4;
  L.hz = off;
  off += n4;
  L.rbar = off;
  off += n4;
  L.part = off;
  off += align_up(3 * (size_t)kStatBlocks * 8);
  L.res = off;
  off += 256;
  L.total = off;
  return L;
}

// ring slots (cur, old) <-> checkpoint c
spg_status ck_copy(spg_problem* P, char* ws, const VjpLayout& L, int c, bool save) {
  const size_t n4 = align_up((size_t)P->d.nvox * 4);
  const size_t n2 = P->comp ? align_up((size_t)P->d.nvox * 2) : 0;
  char* base = ws + L.ck + (size_t)c * L.ck_slot;
  const int slots[2] = {save ? P->cur : 0, save ? P->old : 1};
  for (int k = 0; k < 2; ++k) {
    char* hi = base + k * (n4 + n2);
    char* lo = hi + n4;
    if (save) {
      SPG_CK(P, hipMemcpyAsync(hi, P->xhi(slots[k]), (size_t)P->d.nvox * 4, hipMemcpyDeviceToDevice, P->stream));
      if (P->comp)
        SPG_CK(P, hipMemcpyAsync(lo, P->xlo(slots[k]), (size_t)P->d.nvox * 2, hipMemcpyDeviceToDevice, P->stream));
    } else {
      SPG_CK(P, hipMemcpyAsync(P->xhi(slots[k]), hi, (size_t)P->d.nvox * 4, hipMemcpyDeviceToDevice, P->stream));
      if (P->comp)
        SPG_CK(P, hipMemcpyAsync(P->xlo(slots[k]), lo, (size_t)P->d.nvox * 2, hipMemcpyDeviceToDevice, P->stream));
    }
  }
  if (!save) {
    P->cur = 0;
    P->old = 1;
    P->primed = false;
  }
  return SPG_OK;
}

// FISTA state (t_j, m_j) at iteration index j (1-based) after a restart.
void momentum_at(const spg_problem* P, int j, double* t, double* m) {
  double tt = 1.0, mm = 0.0;
  for (int q = 1; q < j; ++q) {
    const double tn = P->prm.accel ? 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tt * tt)) : 1.0;
    mm = P->prm.accel ? (tt - 1.0) / tn : 0.0;
    tt = tn;
  }
  *t = tt;
  *m = mm;
}

// Data-term Hessian applied to a real map: A^H(w~ A in) through the x, y, z passes.
spg_status hessian_data(spg_problem* P, const float* in, float* out) {
  const Dims& d = P->d;
  hipStream_t st = P->stream;
  SPG_CK(P, launch_r2c_x(d, in, false, P->S(), P->at<float2>(P->lay.tw_m), P->at<float2>(P->lay.tw_n), st));
  SPG_CK(P, launch_fft_cols(d, P->S(), 1, 0, P->at<float2>(P->lay.tw_y), nullptr, nullptr, nullptr, st, nullptr));
  SPG_CK(P, launch_fft_cols(d, P->S(), 2, 4, P->at<float2>(P->lay.tw_z), P->at<float>(P->lay.ws), nullptr, nullptr,
                            st, nullptr));
  SPG_CK(P, launch_dc_nyquist(d, P->S(), P->at<float2>(P->lay.tw_z), P->at<float>(P->lay.w0p),
                              P->at<float>(P->lay.wnyq), nullptr, nullptr, nullptr, st, nullptr));
  SPG_CK(P, launch_fft_cols(d, P->S(), 1, 1, P->at<float2>(P->lay.tw_y), nullptr, nullptr, nullptr, st, nullptr));
  SPG_CK(P, launch_c2r_x(d, P->S(), out, false, P->at<float2>(P->lay.tw_m), P->at<float2>(P->lay.tw_n), st));
  return SPG_OK;
}
}  // namespace

extern "C" {

spg_status spg_vjp_workspace_size(const spg_problem* P, int32_t K, int32_t C, size_t* bytes) {
  if (!P || !bytes || K < 1 || C < 1 || C > K) return SPG_E_INVAL;
  *bytes = vjp_layout(P, K, C).total;
  return SPG_OK;
}

spg_status spg_run_checkpointed(spg_problem* P, int32_t K, int32_t C, void* d_vjp_ws, size_t bytes) {
  spg_status s = usable(P);
  if (s) return s;
  if (K < 1 || C < 1 || C > K) return set_err(P, SPG_E_INVAL, "need K >= 1 and 1 <= C <= K");
  if (!P->data_set) return set_err(P, SPG_E_STATE, "spg_set_data has not succeeded");
  if (P->store == ST_BF16) return set_err(P, SPG_E_UNSUPPORTED, "the reverse pass needs an fp32 map buffer");
  if (!(P->L > 0)) return set_err(P, SPG_E_STATE, "L = 0");
  if (!d_vjp_ws || (reinterpret_cast<uintptr_t>(d_vjp_ws) % kAlign) != 0)
    return set_err(P, SPG_E_INVAL, "reverse-pass workspace must be 256-byte aligned device memory");
  const VjpLayout L = vjp_layout(P, K, C);
  if (bytes < L.total) return set_err(P, SPG_E_NOMEM, "reverse-pass workspace too small");
  char* ws = reinterpret_cast<char*>(d_vjp_ws);
  restart(P);
  P->old = P->cur;  // x_{-1} = x_0
  if ((s = ck_copy(P, ws, L, 0, true))) return s;
  P->old = (P->cur + 1) % 3;
  P->vjp_m.assign(K, 0.0);
  // the recorded iterations run the separate x-axis sweeps, as the replays of spg_vjp do
  // (they keep the data gradient of every iteration), so that forward and replay agree bitwise
  const bool fused = P->fused;
  P->fused = false;
  for (int it = 0; it < K && s == SPG_OK; ++it) {
    if (it > 0 && it % C == 0) s = ck_copy(P, ws, L, it / C, true);
    if (s == SPG_OK) {
      P->vjp_m[it] = P->m_cur;
      s = iterate_once(P, nullptr);
    }
  }
  P->fused = fused;
  if (s) return s;
  if ((s = ck_copy(P, ws, L, L.nseg, true))) return s;
  P->vjp_valid = true;
  P->vjp_K = K;
  P->vjp_C = C;
  P->vjp_lr = P->lr;
  return SPG_OK;
}

spg_status spg_vjp(spg_problem* P, void* d_vjp_ws, size_t bytes, const float* d_w, const float* d_xbar,
                   float* d_bbar, double* lam_bar, double* mu_bar) {
  spg_status s = usable(P);
  if (s) return s;
  if (!P->vjp_valid || P->lr != P->vjp_lr)
    return set_err(P, SPG_E_STATE, "no unrolled solve recorded (spg_run_checkpointed) for these parameters");
  if (!d_w || !d_xbar || !d_bbar || !d_vjp_ws) return set_err(P, SPG_E_INVAL, "NULL pointer");
  const int K = P->vjp_K, C = P->vjp_C;
  const VjpLayout L = vjp_layout(P, K, C);
  if (bytes < L.total) return set_err(P, SPG_E_NOMEM, "reverse-pass workspace too small");
  const Dims& d = P->d;
  hipStream_t st = P->stream;
  char* ws = reinterpret_cast<char*>(d_vjp_ws);
  const size_t n4 = align_up((size_t)d.nvox * 4);
  auto segx = [&](int i) { return reinterpret_cast<float*>(ws + L.seg_x + (size_t)i * n4); };
  auto segg = [&](int i) { return reinterpret_cast<float*>(ws + L.seg_g + (size_t)i * n4); };
  auto abar = [&](int k) { return reinterpret_cast<float*>(ws + L.abar + (size_t)(((k % 3) + 3) % 3) * n4); };
  float* zbar = reinterpret_cast<float*>(ws + L.zbar);
  float* hz = reinterpret_cast<float*>(ws + L.hz);
  float* rbar = reinterpret_cast<float*>(ws + L.rbar);
  double* part = reinterpret_cast<double*>(ws + L.part);
  double* res = reinterpret_cast<double*>(ws + L.res);
  const float* u = P->unif_u ? nullptr : P->at<float>(P->lay.u);
  const float* v = P->unif_v ? nullptr : P->at<float>(P->lay.v);
  const double lr = P->lr;

  SPG_CK(P, launch_fill(rbar, d.nvox, 0.0f, st));
  SPG_CK(P, hipMemcpyAsync(abar(K), d_xbar, (size_t)d.nvox * 4, hipMemcpyDeviceToDevice, st));
  SPG_CK(P, launch_fill(abar(K - 1), d.nvox, 0.0f, st));
  double lamb = 0, mub = 0, lrb = 0;
  for (int sgm = L.nseg - 1; sgm >= 0; --sgm) {
    const int j0 = sgm * C;
    const int len = std::min(C, K - j0);
    // replay the segment from its checkpoint, keeping x_k and the data gradient of y_k
    if ((s = ck_copy(P, ws, L, sgm, false))) return s;
    momentum_at(P, j0 + 1, &P->t, &P->m_cur);
    P->j = j0 + 1;
    SPG_CK(P, launch_get_map(d, P->xhi(P->old), P->xlo(P->old), segx(0), P->comp, st));
    SPG_CK(P, launch_get_map(d, P->xhi(P->cur), P->xlo(P->cur), segx(1), P->comp, st));
    for (int i = 0; i < len; ++i) {
      if ((s = iterate_once(P, segg(i)))) return s;
      SPG_CK(P, launch_get_map(d, P->xhi(P->cur), P->xlo(P->cur), segx(i + 2), P->comp, st));
    }
    // reverse through the segment
    for (int i = len - 1; i >= 0; --i) {
      const int k = j0 + i;
      SPG_CK(P, launch_adj_prox(d, segx(i + 2), abar(k + 1), segg(i), u, (float)lr, zbar, rbar, part, kStatBlocks, st));
      if ((s = hessian_data(P, zbar, hz))) return s;
      SPG_CK(P, launch_adj_tv(d, segx(i + 1), segx(i), (float)P->vjp_m[k], zbar, hz, v, (float)lr,
                              (float)P->prm.mu, (float)P->prm.eps, abar(k), k >= 1 ? abar(k - 1) : nullptr,
                              part + 2 * kStatBlocks, kStatBlocks, st));
      const int ops[3] = {RED_OP_SUM, RED_OP_SUM, RED_OP_SUM};
      SPG_CK(P, launch_reduce(part, kStatBlocks, 3, ops, res, st));
      double r[3];
      if ((s = read_results_to(P, res, r, 3))) return s;
      lamb += lr * r[0];
      lrb += P->prm.lambda * r[0] - r[1] - P->prm.mu * r[2];
      mub += -lr * r[2];
    }
  }
  // lr = 1/L(mu): d lr / d mu = -lr^2 max(v) ||D||^2 / eps
  mub += lrb * (-lr * lr * P->vmax * P->dn2 / P->prm.eps);
  // b-bar = w * A(rbar)
  SPG_CK(P, launch_r2c_x(d, rbar, false, P->S(), P->at<float2>(P->lay.tw_m), P->at<float2>(P->lay.tw_n), st));
  SPG_CK(P, launch_fft_cols(d, P->S(), 1, 0, P->at<float2>(P->lay.tw_y), nullptr, nullptr, nullptr, st, nullptr));
  SPG_CK(P, launch_fft_cols(d, P->S(), 2, 0, P->at<float2>(P->lay.tw_z), nullptr, nullptr, nullptr, st, nullptr));
  SPG_CK(P, launch_expand_bbar(d, P->S(), d_w, reinterpret_cast<float2*>(d_bbar), st));
  // back to the end state of the unrolled solve
  if ((s = ck_copy(P, ws, L, L.nseg, false))) return s;
  momentum_at(P, K + 1, &P->t, &P->m_cur);
  P->j = K + 1;
  SPG_CK(P, hipStreamSynchronize(st));
  if (lam_bar) *lam_bar = lamb;
  if (mu_bar) *mu_bar = mub;
  return SPG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- backprojection

extern "C" {

spg_status spg_backproject_workspace_size(int32_t nx, int32_t ny, int32_t nz, size_t* bytes) {
  if (!bytes || nx < 1 || ny < 1 || nz < 1 || nx > 1024 || ny > 1024 || nz > 1024) return SPG_E_INVAL;
  *bytes = align_up((3 * (size_t)nx * ny * nz + 3) * sizeof(uint64_t));
  return SPG_OK;
}

spg_status spg_backproject(int32_t nx, int32_t ny, int32_t nz, int32_t n_img, int32_t m, const float* d_images,
                           const double* d_rot, const float* d_ctf, const float* d_weight, double h,
                           void* d_workspace, size_t bytes, void* hip_stream, float* d_w_out, float* d_b_out) {
  size_t need = 0;
  if (spg_backproject_workspace_size(nx, ny, nz, &need) != SPG_OK) return SPG_E_INVAL;
  if (n_img < 1 || m < 1 || m > 4096 || !std::isfinite(h) || h <= 0 || !d_images || !d_rot || !d_workspace ||
      !d_w_out || !d_b_out || (reinterpret_cast<uintptr_t>(d_workspace) % 8) != 0)
    return SPG_E_INVAL;
  if (bytes < need) return SPG_E_NOMEM;
  Dims d{nx, ny, nz, nx / 2, (long long)nx * ny * nz};
  if (launch_backproject(d, n_img, m, reinterpret_cast<const float2*>(d_images), d_rot, d_ctf, d_weight, h,
                         d_workspace, d_w_out, reinterpret_cast<float2*>(d_b_out),
                         reinterpret_cast<hipStream_t>(hip_stream)) != hipSuccess)
    return SPG_E_DEVICE;
  return SPG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- checkpoints

struct StateHeader {
  uint64_t magic;
  int32_t nx, ny, nz, flags;
  int32_t unif_u, unif_v, j, round;
  int64_t iters_done;
  double t, m_cur, vmax, lambda, mu, eps, gamma;
};

static size_t state_bytes(const spg_problem* P) {
  const size_t nvox = (size_t)P->d.nvox;
  const size_t slot = align_up(nvox * 4) + (P->comp ? align_up(nvox * 2) : 0);
  return kAlign + 2 * slot + 2 * align_up(P->wbytes());
}

spg_status spg_state_size(const spg_problem* P, size_t* bytes) {
  if (!P || !bytes) return SPG_E_INVAL;
  *bytes = state_bytes(P);
  return SPG_OK;
}

spg_status spg_get_state(spg_problem* P, void* d_buf, size_t bytes) {
  spg_status s = usable(P);
  if (s) return s;
  if (!d_buf || bytes < state_bytes(P)) return set_err(P, SPG_E_INVAL, "state buffer too small or NULL");
  StateHeader h{};
  h.magic = kStateMagic;
  h.nx = P->d.nx; h.ny = P->d.ny; h.nz = P->d.nz; h.flags = P->prm.flags;
  h.unif_u = P->unif_u; h.unif_v = P->unif_v; h.j = P->j; h.round = P->round;
  h.iters_done = P->iters_done;
  h.t = P->t; h.m_cur = P->m_cur; h.vmax = P->vmax;
  h.lambda = P->prm.lambda; h.mu = P->prm.mu; h.eps = P->prm.eps; h.gamma = P->prm.gamma;
  char* dst = reinterpret_cast<char*>(d_buf);
  const size_t nvox = (size_t)P->d.nvox;
  size_t off = kAlign;
  const int slots[2] = {P->cur, P->old};
  for (int k = 0; k < 2; ++k) {
    SPG_CK(P, hipMemcpyAsync(dst + off, P->xhi(slots[k]), nvox * 4, hipMemcpyDeviceToDevice, P->stream));
    off += align_up(nvox * 4);
    if (P->comp) {
      SPG_CK(P, hipMemcpyAsync(dst + off, P->xlo(slots[k]), nvox * 2, hipMemcpyDeviceToDevice, P->stream));
      off += align_up(nvox * 2);
    }
  }
  const size_t wb = P->wbytes();
  if (!P->unif_u) SPG_CK(P, hipMemcpyAsync(dst + off, P->at<void>(P->lay.u), wb, hipMemcpyDeviceToDevice, P->stream));
  off += align_up(wb);
  if (!P->unif_v) SPG_CK(P, hipMemcpyAsync(dst + off, P->at<void>(P->lay.v), wb, hipMemcpyDeviceToDevice, P->stream));
  SPG_CK(P, hipMemcpyAsync(dst, &h, sizeof(h), hipMemcpyHostToDevice, P->stream));
  SPG_CK(P, hipStreamSynchronize(P->stream));
  return SPG_OK;
}

spg_status spg_set_state(spg_problem* P, const void* d_buf, size_t bytes) {
  spg_status s = usable(P);
  if (s) return s;
  if (!d_buf || bytes < state_bytes(P)) return set_err(P, SPG_E_INVAL, "state buffer too small or NULL");
  StateHeader h{};
  SPG_CK(P, hipMemcpyAsync(&h, d_buf, sizeof(h), hipMemcpyDeviceToHost, P->stream));
  SPG_CK(P, hipStreamSynchronize(P->stream));
  if (h.magic != kStateMagic || h.nx != P->d.nx || h.ny != P->d.ny || h.nz != P->d.nz || h.flags != P->prm.flags)
    return set_err(P, SPG_E_INVAL, "state buffer does not match this problem");
  const char* src = reinterpret_cast<const char*>(d_buf);
  const size_t nvox = (size_t)P->d.nvox;
  size_t off = kAlign;
  const int slots[2] = {0, 1};
  for (int k = 0; k < 2; ++k) {
    SPG_CK(P, hipMemcpyAsync(P->xhi(slots[k]), src + off, nvox * 4, hipMemcpyDeviceToDevice, P->stream));
    off += align_up(nvox * 4);
    if (P->comp) {
      SPG_CK(P, hipMemcpyAsync(P->xlo(slots[k]), src + off, nvox * 2, hipMemcpyDeviceToDevice, P->stream));
      off += align_up(nvox * 2);
    }
  }
  const size_t wb = P->wbytes();
  if (!h.unif_u) SPG_CK(P, hipMemcpyAsync(P->at<void>(P->lay.u), src + off, wb, hipMemcpyDeviceToDevice, P->stream));
  off += align_up(wb);
  if (!h.unif_v) SPG_CK(P, hipMemcpyAsync(P->at<void>(P->lay.v), src + off, wb, hipMemcpyDeviceToDevice, P->stream));
  P->cur = 0;
  P->old = 1;
  P->unif_u = h.unif_u != 0;
  P->unif_v = h.unif_v != 0;
  P->j = h.j;
  P->round = h.round;
  P->iters_done = h.iters_done;
  P->t = h.t;
  P->m_cur = h.m_cur;
  P->vmax = h.vmax;
  P->prm.lambda = h.lambda;
  P->prm.mu = h.mu;
  P->prm.eps = h.eps;
  P->prm.gamma = h.gamma;
  P->primed = false;
  recompute_L(P);
  return SPG_OK;
}

// ---------------------------------------------------------------- profiling

spg_status spg_profile_begin(spg_problem* P, int32_t kernel_class, int32_t capacity) {
  spg_status s = usable(P);
  if (s) return s;
  if (kernel_class < SPG_KERNEL_ALL || kernel_class >= SPG_KERNEL_COUNT || capacity <= 0 || capacity > (1 << 20))
    return set_err(P, SPG_E_INVAL, "bad kernel class or capacity");
  for (hipEvent_t e : P->ev) (void)hipEventDestroy(e);
  P->ev.assign(2 * (size_t)capacity * SPG_KERNEL_COUNT, nullptr);
  const int lo = kernel_class == SPG_KERNEL_ALL ? 0 : kernel_class;
  const int hi = kernel_class == SPG_KERNEL_ALL ? SPG_KERNEL_COUNT : kernel_class + 1;
  for (int c = lo; c < hi; ++c)
    for (size_t k = 0; k < 2 * (size_t)capacity; ++k)
      SPG_CK(P, hipEventCreate(&P->ev[2 * (size_t)c * capacity + k]));
  P->prof_on = true;
  P->prof_class = kernel_class;
  P->prof_cap = capacity;
  for (int c = 0; c < SPG_KERNEL_COUNT; ++c) P->prof_n[c] = 0;
  return SPG_OK;
}

spg_status spg_profile_end(spg_problem* P, double* total_ms, int32_t* launches) {
  spg_status s = usable(P);
  if (s) return s;
  if (!P->prof_on) return set_err(P, SPG_E_STATE, "profiling is not enabled");
  SPG_CK(P, hipStreamSynchronize(P->stream));
  for (int c = 0; c < SPG_KERNEL_COUNT; ++c) {
    double tot = 0;
    for (int k = 0; k < P->prof_n[c]; ++k) {
      float ms = 0;
      const size_t slot = 2 * ((size_t)c * P->prof_cap + k);
      SPG_CK(P, hipEventElapsedTime(&ms, P->ev[slot], P->ev[slot + 1]));
      tot += ms;
    }
    if (total_ms) total_ms[c] = tot;
    if (launches) launches[c] = P->prof_n[c];
  }
  for (hipEvent_t e : P->ev)
    if (e) (void)hipEventDestroy(e);
  P->ev.clear();
  P->prof_on = false;
  P->prof_class = -1;
  P->prof_cap = 0;
  return SPG_OK;
}

}  // extern "C"

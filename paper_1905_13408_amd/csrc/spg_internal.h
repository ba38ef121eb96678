// Internal interface between the host runtime (spg_api.hip) and the gfx950 kernels
// (spg_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spg {

// Grid geometry.  Real maps are nz*ny*nx floats, C order, x fastest.  The half spectrum
// of a real map is stored packed: rows of P = nx/2 complex values per (z, y) with the
// purely real kx = 0 and kx = nx/2 values of the x-axis real FFT sharing slot 0
// (re = kx 0, im = kx nx/2); the y and z transforms act on that packed slot linearly and
// the Fourier weight step separates the two planes again using Hermitian symmetry.
struct Dims {
  int nx, ny, nz, P;
  long long nvox;
};

// Tile of the fused stencil / prox kernel: 64 x-columns by 8 y-rows, marched along z over
// slabs of ProxArgs::zc planes (PT_ZC by default; the autotuner may choose another depth).
constexpr int PT_TX = 64;
constexpr int PT_TY = 8;
constexpr int PT_ZC = 32;

// Reductions: per-block fp64 partials, summed in fixed order by k_reduce.
constexpr int RED_OP_SUM = 0, RED_OP_MAX = 1, RED_OP_MIN = 2;

// Storage modes: plain fp32 iterate; compensated fp32 hi + bf16 lo iterate with fp64
// prox arithmetic; fp32 iterate with the penalty weights and the gradient / extrapolated
// map stored in bf16.
constexpr int ST_PLAIN = 0, ST_COMP = 1, ST_BF16 = 2;

// Arguments of the fused stencil / prox kernel.
struct ProxArgs {
  void* rbuf;                   // in: data gradient of y_k (real map); out: y_{k+1}
                                // (fp32, bf16 in ST_BF16)
  const float* gin;             // check mode: fp32 data gradient of x_k
  const float* xk_hi;           // x_k  (fp32 hi part)
  const uint16_t* xk_lo;        // x_k  (bf16 lo part; compensated mode only)
  const float* xo_hi;           // x_{k-1}
  const uint16_t* xo_lo;
  float* xn_hi;                 // x_{k+1}
  uint16_t* xn_lo;
  const void* u;                // l1 weights or nullptr (uniform 1); fp32, bf16 in ST_BF16
  const void* v;                // TV weights or nullptr (uniform 1); fp32, bf16 in ST_BF16
  const float* xprev;           // previous M-step map of the gamma term, nullptr = 0
  double* partials;             // check mode: 5 x nblocks fp64 partials
  int nx, ny, nz;
  int read_old;                 // 0 when m == 0: x_{k-1} is not read
  double m, m_next;             // momentum for y_k and for y_{k+1}
  double lr, lam, mu, gamma;
  float eps;
  int eps2_normal;              // eps * eps (fp32) is a normal float
  int zc;                       // z-slab depth of one block
};

int prox_num_blocks(const Dims& d, int zc);

// Fused x-axis transforms + stencil/prox on full-width rows: reads the gradient as the
// packed x-spectrum rows in S (after the y and z passes), writes x_{k+1} and the
// x-spectrum of y_{k+1} back into S.  Grids with nx in {32, 64, 128, 256, 512} and ny a
// multiple of 4 (the kernel's tile height).
bool prox_fft_supported(const Dims& d);
int prox_fft_num_blocks(const Dims& d, int zc);
// mon: also the per-block partials of the objective's penalty terms at y_k (3 x nblocks
// into a.partials)
hipError_t launch_prox_fft(const Dims& d, const ProxArgs& a, float2* S, const float2* tw_m, const float2* tw_n,
                           int store, hipStream_t st, bool mon = false);

// persist: the fused z modes run persistent blocks (false: one block per tile, for
// problems that share the GPU with concurrent work).  kx0, nkx: the columns [kx0, kx0 + nkx)
// of the packed spectrum only (nkx = 0: to the end of the row); the objective mode (3) takes
// the whole row.
hipError_t launch_fft_cols(const Dims& d, float2* S, int axis /*1 = y, 2 = z*/, int mode,
                           const float2* tw, const float* ws, const float2* cs, double* partials,
                           hipStream_t st, int* nblocks_out, int nt = 16 /* columns per tile: 8 or 16 */,
                           bool persist = true, int kx0 = 0, int nkx = 0);
// Small maps (ny, nz in {8, 16, 32, 64}): the y forward, z + weight + packed-plane and y inverse
// passes in one launch, one block per (ky, kz) plane of a column kx.
bool yz_plane_supported(const Dims& d);
hipError_t launch_yz_plane(const Dims& d, float2* S, const float2* tw_y, const float2* tw_z, const float* ws,
                           const float2* cs, const float* w0p, const float* wnyq, const float2* c0p,
                           const float2* cnyq, hipStream_t st);
hipError_t launch_dc_nyquist(const Dims& d, float2* S, const float2* tw_z, const float* w0p,
                             const float* wnyq, const float2* c0p, const float2* cnyq, double* partials,
                             hipStream_t st, int* nblocks_out);
hipError_t launch_r2c_x(const Dims& d, const void* rin, bool rin_bf16, float2* S, const float2* tw_m,
                        const float2* tw_n, hipStream_t st);
hipError_t launch_c2r_x(const Dims& d, const float2* S, void* rout, bool rout_bf16, const float2* tw_m,
                        const float2* tw_n, hipStream_t st);
hipError_t launch_prox_tv(const Dims& d, const ProxArgs& a, int store, bool check, hipStream_t st,
                          bool mon = false);

hipError_t launch_prime(const Dims& d, void* rbuf, const float* xk_hi, const uint16_t* xk_lo,
                        const float* xo_hi, const uint16_t* xo_lo, double m, int read_old,
                        int store, hipStream_t st);
hipError_t launch_set_map(const Dims& d, const float* x0, float* hi, uint16_t* lo, hipStream_t st);
hipError_t launch_get_map(const Dims& d, const float* hi, const uint16_t* lo, float* out, bool compensated,
                          hipStream_t st);
hipError_t launch_fold(const Dims& d, const float* w, const float2* b, float* ws, float* w0p, float* wnyq,
                       float2* cs, float2* c0p, float2* cnyq, double* partials, int nblocks, hipStream_t st);
// partials: 5 x nblocks (non-finite count, min w, 1/2 sum w|b|^2, sum w, energy of the
// real part of the unregularised solution)
hipError_t launch_data_stats(const Dims& d, const float* w, const float2* b, double* partials, int nblocks,
                             hipStream_t st);
// partials: 2 x nblocks, sum log(|x| + eps1) and sum log(|Dx| + eps2)
hipError_t launch_log_terms(const Dims& d, const float* hi, const uint16_t* lo, double eps1, double eps2, bool comp,
                            double* partials, int nblocks, hipStream_t st);
hipError_t launch_weight_stats(const Dims& d, const float* a, double* partials, int nblocks, hipStream_t st);
hipError_t launch_reweight(const Dims& d, const float* hi, const uint16_t* lo, void* u, void* v,
                           double eps1, double eps2, int store, double* partials, int nblocks,
                           hipStream_t st);
hipError_t launch_f32_to_bf16(const float* src, uint16_t* dst, long long n, hipStream_t st);
hipError_t launch_bf16_to_f32(const uint16_t* src, float* dst, long long n, hipStream_t st);
hipError_t launch_fill(float* dst, long long n, float value, hipStream_t st);
// out = c0 + sum pa[na] + sum pb[nb] + lam sum pc[0:nc] + mu sum pc[nc:2nc] + gamma sum pc[2nc:3nc]
hipError_t launch_obj_finish(const double* pa, int na, const double* pb, int nb, const double* pc, int nc, double c0,
                             double lam, double mu, double gamma, double* out, hipStream_t st);
hipError_t launch_reduce(const double* partials, int n, int nq, const int* ops, double* out, hipStream_t st);
hipError_t launch_adj_prox(const Dims& d, const float* xn, const float* abar, const float* gdat, const float* u,
                           float lr, float* zbar, float* rbar, double* partials, int nblocks, hipStream_t st);
hipError_t launch_adj_tv(const Dims& d, const float* xk, const float* xkm, float m, const float* zbar, const float* hz,
                         const float* v, float lr, float mu, float eps, float* abar_k, float* abar_km,
                         double* partials, int nblocks, hipStream_t st);
hipError_t launch_expand_bbar(const Dims& d, const float2* S, const float* w, float2* out, hipStream_t st);
hipError_t launch_backproject(const Dims& d, int n_img, int m, const float2* images, const double* rots,
                              const float* ctf, const float* weights, double h, void* ws, float* w, float2* b,
                              hipStream_t st);
hipError_t launch_fsc_shells(const Dims& d, const float2* S1, const float2* S2, int nshells, double* partials,
                             int nblocks, double* out, hipStream_t st);

}  // namespace spg

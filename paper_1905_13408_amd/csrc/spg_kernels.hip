// gfx950 kernels of the SPG solver for the reweighted weighted-l1 + TV reconstruction
// (Luo, arXiv 1905.13408, eq 12-21 and eq 31).
//
// One SPG iteration crosses HBM in these sweeps (all in place on the packed half
// spectrum S except where noted):
//   k_fft_cols<mode 0> (y axis)   forward column FFTs along y
//   k_fft_zw<mode 2>   (z axis)   forward FFT along z, G = w~ Y - c, inverse FFT along z
//   k_dc_nyquist                  the same for the packed kx = 0 / kx = nx/2 plane
//   k_fft_cols<mode 1> (y axis)   inverse column FFTs along y
//   k_c2r_x                       x-axis inverse real FFT -> data gradient map
//   k_prox_tv                     smoothed-TV stencil, gradient step, soft threshold,
//                                 momentum extrapolation (marches z-slabs through LDS)
//   k_r2c_x                       x-axis forward real FFT of the next extrapolated map
// The path is HBM-bound (a few flop per byte), so the kernels are built around
// coalesced 128-byte row segments, LDS-resident transforms and no MFMA.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "spg_internal.h"

namespace spg {

// ---------------------------------------------------------------- complex helpers

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// bf16 <-> fp32 (round to nearest even), used for the low word of the compensated iterate.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// Element i of a real array stored as fp32 or (BF) bf16.
template <bool BF>
__device__ __forceinline__ float ld_real(const void* p, long long i) {
  if constexpr (BF) return bf16_to_f32(reinterpret_cast<const uint16_t*>(p)[i]);
  else return reinterpret_cast<const float*>(p)[i];
}
template <bool BF>
__device__ __forceinline__ void st_real(void* p, long long i, float v) {
  if constexpr (BF) reinterpret_cast<uint16_t*>(p)[i] = f32_to_bf16(v);
  else reinterpret_cast<float*>(p)[i] = v;
}

// ---------------------------------------------------------------- radix butterflies
// Forward transforms use exp(-2 pi i / R), inverse ones exp(+2 pi i / R); no scaling.

template <bool INV>
__device__ __forceinline__ float2 rot_mi(float2 a) {  // a * (-i) forward, a * (+i) inverse
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(float2* a) {
  float2 t = a[0];
  a[0] = cadd(t, a[1]);
  a[1] = csub(t, a[1]);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2* a) {
  float2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
  float2 t2 = cadd(a[1], a[3]), t3 = rot_mi<INV>(csub(a[1], a[3]));
  a[0] = cadd(t0, t2);
  a[2] = csub(t0, t2);
  a[1] = cadd(t1, t3);
  a[3] = csub(t1, t3);
}

template <bool INV>
__device__ __forceinline__ void dft8(float2* a) {
  const float s = 0.70710678118654752440f;
  float2 e[4] = {a[0], a[2], a[4], a[6]};
  float2 o[4] = {a[1], a[3], a[5], a[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  // o[k] *= W8^k
  float2 o1 = INV ? make_float2(s * (o[1].x - o[1].y), s * (o[1].x + o[1].y))
                  : make_float2(s * (o[1].x + o[1].y), s * (o[1].y - o[1].x));
  float2 o2 = rot_mi<INV>(o[2]);
  float2 o3 = INV ? make_float2(-s * (o[3].x + o[3].y), s * (o[3].x - o[3].y))
                  : make_float2(s * (o[3].y - o[3].x), -s * (o[3].x + o[3].y));
  a[0] = cadd(e[0], o[0]);
  a[4] = csub(e[0], o[0]);
  a[1] = cadd(e[1], o1);
  a[5] = csub(e[1], o1);
  a[2] = cadd(e[2], o2);
  a[6] = csub(e[2], o2);
  a[3] = cadd(e[3], o3);
  a[7] = csub(e[3], o3);
}

// 3-point DFT: with s = a1 + a2, d = a1 - a2, t = a0 - s/2:
// X0 = a0 + s, X1 = t -+ i (sqrt3/2) d, X2 = t +- i (sqrt3/2) d  (upper sign forward).
template <bool INV>
__device__ __forceinline__ void dft3(float2* a) {
  const float h = 0.86602540378443864676f;
  const float2 sm = cadd(a[1], a[2]);
  const float2 d = csub(a[1], a[2]);
  const float2 t = make_float2(a[0].x - 0.5f * sm.x, a[0].y - 0.5f * sm.y);
  const float2 ud = rot_mi<INV>(make_float2(h * d.x, h * d.y));  // -+ i (sqrt3/2) d
  a[0] = cadd(a[0], sm);
  a[1] = cadd(t, ud);
  a[2] = csub(t, ud);
}

// 5-point DFT with b1 = a1 + a4, b2 = a2 + a3, d1 = a1 - a4, d2 = a2 - a3, c_k = cos(2 pi k/5),
// s_k = sin(2 pi k/5): X1,4 = a0 + c1 b1 + c2 b2 -+ i (s1 d1 + s2 d2),
// X2,3 = a0 + c2 b1 + c1 b2 -+ i (s2 d1 - s1 d2)  (upper sign forward).
template <bool INV>
__device__ __forceinline__ void dft5(float2* a) {
  const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
  const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;
  const float2 b1 = cadd(a[1], a[4]), b2 = cadd(a[2], a[3]);
  const float2 d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
  const float2 r1 = make_float2(a[0].x + c1 * b1.x + c2 * b2.x, a[0].y + c1 * b1.y + c2 * b2.y);
  const float2 r2 = make_float2(a[0].x + c2 * b1.x + c1 * b2.x, a[0].y + c2 * b1.y + c1 * b2.y);
  const float2 q1 = rot_mi<INV>(make_float2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y));
  const float2 q2 = rot_mi<INV>(make_float2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y));
  a[0] = cadd(a[0], cadd(b1, b2));
  a[1] = cadd(r1, q1);
  a[4] = csub(r1, q1);
  a[2] = cadd(r2, q2);
  a[3] = csub(r2, q2);
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2* a) {
  if constexpr (R == 2) dft2<INV>(a);
  else if constexpr (R == 3) dft3<INV>(a);
  else if constexpr (R == 4) dft4<INV>(a);
  else if constexpr (R == 5) dft5<INV>(a);
  else dft8<INV>(a);
}

// ---------------------------------------------------------------- LDS Stockham engine
// Length L = 2^n transform held in LDS; element p of the transform owned by this thread
// group sits at buf[p * ps] (re and im in separate arrays).  T threads cooperate on
// one transform (q in [0, T)).  Radix-8 stages, then one radix-4 or radix-2 stage.
// Stage with radix R after Ns points have been combined (self-sorting Stockham form):
// butterfly j reads j + r L/R, twiddles by exp(-+2 pi i r (j mod Ns) / (Ns R)), and
// writes (j - j mod Ns) R + j mod Ns + r Ns.

// Stage radices of a supported length L = 2^a 3^b 5^c (at most one 3 and one 5): for a
// power of two, radix-8 stages and one closing radix-4 or radix-2 stage; for a mixed
// length, the radix-5 / radix-3 stage first and then radix-4 stages (and one radix 2),
// which keeps more threads per transform.  T (threads per transform) must divide L / R
// of every stage; the default is the largest such value up to 16.
struct RadixList {
  int n;
  int r[12];
};

constexpr RadixList make_plan(int L) {
  RadixList p{};
  int rest = L;
  if (rest % 5 == 0) { p.r[p.n++] = 5; rest /= 5; }
  if (rest % 3 == 0) { p.r[p.n++] = 3; rest /= 3; }
  const bool mixed = rest != L;
  if (mixed) {
    while (rest % 4 == 0 && rest > 2) { p.r[p.n++] = 4; rest /= 4; }
  } else {
    while (rest % 8 == 0) { p.r[p.n++] = 8; rest /= 8; }
    if (rest % 4 == 0) { p.r[p.n++] = 4; rest /= 4; }
  }
  if (rest == 2) { p.r[p.n++] = 2; rest = 1; }
  return p;
}

constexpr int gcdc(int a, int b) { return b == 0 ? a : gcdc(b, a % b); }

constexpr int plan_gcd(int L) {
  RadixList p = make_plan(L);
  int g = 0;
  for (int s = 0; s < p.n; ++s) g = gcdc(g, L / p.r[s]);
  return g;
}

constexpr int largest_divisor_le(int g, int cap) {
  int t = cap < g ? cap : g;
  while (t > 1 && g % t != 0) --t;
  return t < 1 ? 1 : t;
}

template <int L>
struct FftPlan {
  static constexpr RadixList plan = make_plan(L);
  static constexpr int T = largest_divisor_le(plan_gcd(L), 16);
};

// act = false: the thread takes part in the barriers only.
template <int L, int T, int R, bool INV>
__device__ __forceinline__ void fft_stage(float* __restrict__ re, float* __restrict__ im, int ps, int q, int Ns,
                                          const float2* __restrict__ tw, bool act = true) {
  constexpr int NB = L / (R * T);
  constexpr int STRIDE = L / R;
  float2 a[NB][R];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (!act) break;
    const int j = q + T * b;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int idx = (j + r * STRIDE) * ps;
      a[b][r] = make_float2(re[idx], im[idx]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (!act) break;
    const int j = q + T * b;
    const int k = j % Ns;
    if (Ns > 1) {
      const int step = L / (Ns * R);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[r * k * step];
        if (INV) w.y = -w.y;
        a[b][r] = cmul(a[b][r], w);
      }
    }
    dft<R, INV>(a[b]);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int idx = (base + r * Ns) * ps;
      re[idx] = a[b][r].x;
      im[idx] = a[b][r].y;
    }
  }
  __syncthreads();
}

template <int L, int TT, int S, bool INV>
__device__ __forceinline__ void lds_stages(float* re, float* im, int ps, int q, int Ns, const float2* tw,
                                           bool act = true) {
  constexpr RadixList pl = make_plan(L);
  if constexpr (S < pl.n) {
    constexpr int R = pl.r[S];
    fft_stage<L, TT, R, INV>(re, im, ps, q, Ns, tw, act);
    lds_stages<L, TT, S + 1, INV>(re, im, ps, q, Ns * R, tw, act);
  }
}

template <int L, bool INV, int TT = FftPlan<L>::T>
__device__ __forceinline__ void fft_lds(float* re, float* im, int ps, int q, const float2* __restrict__ tw,
                                        bool act = true) {
  __syncthreads();
  lds_stages<L, TT, 0, INV>(re, im, ps, q, 1, tw, act);
}

// Threads per column of the packed kx = 0 / nx/2 plane kernel: only ny/2 + 1 blocks of two
// columns run, so each column gets as many threads as its radix plan allows (up to 64).
template <int L>
struct DcT {
  static constexpr int T = largest_divisor_le(plan_gcd(L), 64);
};

// Register-resident variant.  Thread q of a transform owns the points q + T i,
// i in [0, E), E = L / T, held in a[i].  The first stage reads its butterfly inputs
// j + r L/R = q + T (b + r L/(R T)) straight from those registers and the last stage
// (base = j because j < Ns there) writes its outputs back to them, so a 512-point
// transform makes two LDS round trips for three stages.  Twiddles come from a table
// in LDS.  LDS data layout as in fft_lds (re/im planes, point stride ps).
constexpr int reg_e(int L, int T) { return L / T; }

template <int L, int TT = FftPlan<L>::T>
struct RegPlan {
  static constexpr RadixList plan = make_plan(L);
  static constexpr int T = TT;
  static constexpr int E = L / T;
  static constexpr int ns = plan.n;
  static constexpr int radix(int s) { return plan.r[s]; }
  static constexpr int span(int s) {  // Ns before stage s
    int v = 1;
    for (int t = 0; t < s; ++t) v *= plan.r[t];
    return v;
  }
};

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

// LDS placement of element e written by a stage of span Ns and radix R (and read by the
// next stage) for one transform per row segment (ps = 1).  The stage writes land Ns*R
// apart for lanes in different butterfly groups, which would pile onto a few of the 32
// banks; XOR-ing the lane's bits [log2 Ns, log2 Ns*R) with address bits above them (so
// the map is a bijection on [0, L)) spreads 32 consecutive lanes over all banks, and the
// next stage's contiguous reads only permute within aligned blocks.  Power-of-two L only.
template <int L, int Ns, int R>
__device__ __forceinline__ int swz(int e) {
  if constexpr ((L & (L - 1)) != 0 || Ns >= 32) {
    return e;
  } else {
    constexpr int ks = Ns * R > 32 ? ilog2c(Ns * R) : 5;
    return e ^ (((e >> ks) & (R - 1)) * Ns);
  }
}

// Orders the LDS accesses of one wavefront across this point.  A wavefront executes its LDS
// instructions in order, so data exchanged among its own lanes needs no s_barrier; this only
// keeps the compiler from moving accesses across.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// act = false: the thread takes part in the barriers only (blocks whose threads do not all
// hold a transform).  SWZ: LDS placement by swz (row transforms, ps = 1).  WS: every
// transform lies within one wavefront, so the stage orders its LDS accesses with wave_sync
// instead of block barriers.
template <int L, int TT, int S, bool INV, bool SWZ = false, bool WS = false>
__device__ __forceinline__ void reg_stage(float2 (&a)[reg_e(L, TT)], float* __restrict__ re,
                                          float* __restrict__ im, int ps, int q, const float2* __restrict__ twl,
                                          bool act = true) {
  using P = RegPlan<L, TT>;
  constexpr int R = P::radix(S);
  constexpr int Ns = P::span(S);
  constexpr int T = P::T;
  constexpr int NB = L / (R * T);
  constexpr int STR = L / R;
  constexpr bool first = S == 0;
  constexpr bool last = S == P::ns - 1;
  float2 v[NB][R];
  if (act) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (first) {
          v[b][r] = a[b + r * (STR / T)];
        } else {
          int e = q + T * b + r * STR;
          if constexpr (SWZ) e = swz<L, P::span(S - 1), P::radix(S - 1)>(e);
          const int idx = e * ps;
          v[b][r] = make_float2(re[idx], im[idx]);
        }
      }
    }
  }
  if constexpr (!first && !last) {
    if constexpr (WS) wave_sync();
    else __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    if (!act) break;
    const int j = q + T * b;
    const int k = j % Ns;
    if constexpr (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        // exp(+2 pi i m / L) = table[L - m]: the inverse reads other addresses than the
        // forward, so the compiler does not keep forward twiddles live for reuse
        const int m = r * k * (L / (Ns * R));
        const float2 w = twl[INV ? ((L - m) % L) : m];
        v[b][r] = cmul(v[b][r], w);
      }
    }
    dft<R, INV>(v[b]);
    if constexpr (last) {
#pragma unroll
      for (int r = 0; r < R; ++r) a[b + r * (STR / T)] = v[b][r];
    } else {
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int e = base + r * Ns;
        if constexpr (SWZ) e = swz<L, Ns, R>(e);
        const int idx = e * ps;
        re[idx] = v[b][r].x;
        im[idx] = v[b][r].y;
      }
    }
  }
  if constexpr (!last) {
    if constexpr (WS) wave_sync();
    else __syncthreads();
  }
}

template <int L, int TT, int S, bool INV, int SEND = RegPlan<L, TT>::ns, bool SWZ = false>
__device__ __forceinline__ void reg_stages(float2 (&a)[reg_e(L, TT)], float* re, float* im, int ps, int q,
                                           const float2* twl, bool act = true) {
  if constexpr (S < SEND) {
    reg_stage<L, TT, S, INV, SWZ>(a, re, im, ps, q, twl, act);
    reg_stages<L, TT, S + 1, INV, SEND, SWZ>(a, re, im, ps, q, twl, act);
  }
}

// Transform the registers a[] of every thread.  Precondition: no thread still reads the
// LDS data planes (barrier after their last use) and the twiddle table is visible.
template <int L, bool INV, int TT = FftPlan<L>::T, bool SWZ = false>
__device__ __forceinline__ void fft_reg(float2 (&a)[reg_e(L, TT)], float* re, float* im, int ps, int q,
                                        const float2* twl, bool act = true) {
  reg_stages<L, TT, 0, INV, RegPlan<L, TT>::ns, SWZ>(a, re, im, ps, q, twl, act);
}

// fft_reg<256, false, 32, true> (the 512-point real rows of a 512-wide map) with its LDS
// positions written out, in stages for callers that interleave them with other work (the
// ordering between stages is the caller's: wave_sync where one wavefront holds the row).
// Stages radix 8, 8, 4 over the points q + 32 i of thread q < 32.  The swizzled position of
// each stage's element reduces, because q < 32, to a per-thread base XOR a constant (bytes):
//   stage 0 writes 8q + (r ^ (q >> 2))            -> (32q | 4(q >> 2)) ^ 4r
//   stage 1 reads  (q + 32r) ^ r = q ^ 33r        -> 4q ^ 132r
//   stage 1 writes 64a + (q & 7) + 8(r ^ a), a = q >> 3 -> (256a | 32a | 4(q & 7)) ^ 32r
//   stage 2 reads  (q + 32b + 64r) ^ 8r           -> 4q ^ (128b + 288r)
// so each access costs one XOR and one add of the row base instead of the generic index
// arithmetic.  Same twiddles, products and butterflies as the generic stages, so the results
// are bitwise those of fft_reg.  s0 transforms the thread's own points and writes them, s1r
// reads the stage-1 inputs, s1w twiddles, transforms and writes them, s2 reads, twiddles and
// transforms the last stage back into a[b + 2r].
struct Row256 {
  static __device__ __forceinline__ void st(char* rb, char* ib, unsigned off, float2 v) {
    *reinterpret_cast<float*>(rb + off) = v.x;
    *reinterpret_cast<float*>(ib + off) = v.y;
  }
  static __device__ __forceinline__ float2 ld(const char* rb, const char* ib, unsigned off) {
    return make_float2(*reinterpret_cast<const float*>(rb + off), *reinterpret_cast<const float*>(ib + off));
  }
  static __device__ __forceinline__ void s0(float2 (&a)[8], float* re, float* im, int q, bool act) {
    float2 v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = a[r];
    dft8<false>(v);
    if (act) {
      const unsigned uq = (unsigned)q;
      const unsigned b0 = (uq * 32u) | (uq & 28u);
#pragma unroll
      for (int r = 0; r < 8; ++r) st(reinterpret_cast<char*>(re), reinterpret_cast<char*>(im), b0 ^ (4u * r), v[r]);
    }
  }
  static __device__ __forceinline__ void s1r(float2 (&a)[8], const float* re, const float* im, int q, bool act) {
    if (act) {
      const unsigned q4 = (unsigned)q * 4u;
#pragma unroll
      for (int r = 0; r < 8; ++r)
        a[r] = ld(reinterpret_cast<const char*>(re), reinterpret_cast<const char*>(im), q4 ^ (132u * r));
    }
  }
  static __device__ __forceinline__ void s1w(float2 (&a)[8], float* re, float* im, int q,
                                             const float2* __restrict__ twl, bool act) {
    if (act) {
      const int k = q & 7;
#pragma unroll
      for (int r = 1; r < 8; ++r) a[r] = cmul(a[r], twl[r * k * 4]);
      dft8<false>(a);
      const unsigned uq = (unsigned)q;
      const unsigned ua = uq >> 3;
      const unsigned b1 = (ua * 256u) | (ua * 32u) | ((uq & 7u) * 4u);
#pragma unroll
      for (int r = 0; r < 8; ++r) st(reinterpret_cast<char*>(re), reinterpret_cast<char*>(im), b1 ^ (32u * r), a[r]);
    }
  }
  static __device__ __forceinline__ void s2(float2 (&a)[8], const float* re, const float* im, int q,
                                            const float2* __restrict__ twl, bool act) {
    if (act) {
      const unsigned q4 = (unsigned)q * 4u;
      float2 v[2][4];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          v[b][r] = ld(reinterpret_cast<const char*>(re), reinterpret_cast<const char*>(im), q4 ^ (128u * b + 288u * r));
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int j = q + 32 * b;
#pragma unroll
        for (int r = 1; r < 4; ++r) v[b][r] = cmul(v[b][r], twl[r * j]);
        dft4<false>(v[b]);
#pragma unroll
        for (int r = 0; r < 4; ++r) a[b + 2 * r] = v[b][r];
      }
    }
  }
};

// Threads per column of the column passes: more threads for the long axes keep the
// per-thread state of the fused z pass (data, folded weight and data term) small.  At
// 512 points, 64 threads of 8 values each hold it near 110 VGPRs, so a 16-column tile
// is one 1024-thread block per CU and an 8-column tile runs two blocks per CU.
template <int L>
struct ColT {
  static constexpr int T = L == 512 ? 64 : ((L >= 256 && (L & (L - 1)) == 0) ? 32 : FftPlan<L>::T);
};

// ---------------------------------------------------------------- XCD-aware block order
// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each with its
// own L2.  Remapping hardware block b to logical tile (b % 8) * (n / 8) + b / 8 gives
// every XCD a contiguous run of logical tiles, so neighbouring tiles that share cache
// lines (stencil halos, the two 64-byte halves of a 128-byte row segment) meet in the
// same L2.  The last n % 8 blocks keep their index.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3;
  if (b >= (q << 3)) return b;
  return (b & 7) * q + (b >> 3);
}

// ---------------------------------------------------------------- block reductions (fp64)

template <int OP>
__device__ __forceinline__ double red_op(double a, double b) {
  if constexpr (OP == RED_OP_SUM) return a + b;
  else if constexpr (OP == RED_OP_MAX) return a > b ? a : b;
  else return a < b ? a : b;
}

// Reduce one value per thread over the block in a fixed order; result valid in thread 0.
template <int OP>
__device__ double block_reduce(double v, double* sh) {
  // blockDim.x is a power of two or a multiple of 64
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  const int width = blockDim.x < 64 ? (int)blockDim.x : 64;
  for (int off = width >> 1; off > 0; off >>= 1) v = red_op<OP>(v, __shfl_xor(v, off, width));
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = sh[0];
  if (threadIdx.x == 0)
    for (int w = 1; w < nw; ++w) r = red_op<OP>(r, sh[w]);
  return r;
}

// ---------------------------------------------------------------- column FFT passes
// Tile: NT consecutive kx columns (<= 16, one 128-byte row segment) by the whole axis.
// k_fft_cols, one tile per block -- mode 0: forward; mode 1: inverse.
// k_fft_zw, persistent blocks on the z axis -- mode 2: forward, G = ws*Y - cs, inverse;
// mode 3: as 2 and also writes per-block partials of 1/2 ws |Y|^2 - Re(conj(cs) Y)
// (multiplicity 2 for 0 < kx < nx/2; the kx = 0 column is done by k_dc_nyquist);
// mode 4: forward, G = ws*Y, inverse (the data-term Hessian applied to a map).

// Element access at a 32-bit byte offset from a block-uniform base pointer.
template <typename V>
__device__ __forceinline__ V ld_at(const V* __restrict__ base, unsigned boff) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + boff);
}
template <typename V>
__device__ __forceinline__ void st_at(V* __restrict__ base, unsigned boff, V v) {
  *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + boff) = v;
}
// ld_at, or (NT) a streaming (non-temporal) vector load: for inputs read once per pass
// over a map too large for the caches.
template <bool NT, typename V>
__device__ __forceinline__ V ld_nt(const V* __restrict__ base, unsigned boff) {
  const char* p = reinterpret_cast<const char*>(base) + boff;
  if constexpr (!NT)
    return *reinterpret_cast<const V*>(p);
  else if constexpr (sizeof(V) == 8)
    return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p)));
  else
    return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const unsigned int*>(p)));
}
// st_at, or (NT) a streaming (non-temporal) vector store: for outputs written once per
// pass over a map too large for the caches, read back only by a later pass.
template <bool NT, typename V>
__device__ __forceinline__ void st_nt(V* __restrict__ base, unsigned boff, V v) {
  char* p = reinterpret_cast<char*>(base) + boff;
  if constexpr (!NT)
    *reinterpret_cast<V*>(p) = v;
  else if constexpr (sizeof(V) == 8)
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned long long, v), reinterpret_cast<unsigned long long*>(p));
  else if constexpr (sizeof(V) == 4)
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned int, v), reinterpret_cast<unsigned int*>(p));
  else
    __builtin_nontemporal_store(__builtin_bit_cast(unsigned short, v), reinterpret_cast<unsigned short*>(p));
}

template <int L, int MODE>
__global__ void __launch_bounds__(16 * ColT<L>::T) k_fft_cols(float2* __restrict__ S, int P, int ntiles,
                                                              long long pstride, long long bstride,
                                                              const float2* __restrict__ tw, int NT) {
  static_assert(MODE == 0 || MODE == 1, "single transforms");
  __shared__ float s_re[L * 16];
  __shared__ float s_im[L * 16];
  __shared__ float2 s_tw[L];
  constexpr int T = ColT<L>::T;
  constexpr int E = RegPlan<L, T>::E;
  const int tid = threadIdx.x;
  const int c = tid % NT, q = tid / NT;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = blk % ntiles;
  const int batch = blk / ntiles;
  const int kx = tile * NT + c;
  const bool valid = kx < P;
  // block-uniform base pointers and 32-bit per-lane element offsets (every offset of a
  // column is below nz*ny*P <= 2^26 elements)
  const long long ub = (long long)batch * bstride + (long long)tile * NT;
  float2* __restrict__ Sb = S + ub;
  const int ps32 = (int)pstride;
  const int off0 = c + q * ps32;
  const int step = T * ps32;

  float2 a[E];
#pragma unroll
  for (int i = 0; i < E; ++i) a[i] = valid ? Sb[off0 + i * step] : make_float2(0.f, 0.f);
  for (int i = tid; i < L; i += blockDim.x) s_tw[i] = tw[i];
  __syncthreads();
  fft_reg<L, MODE == 1, T>(a, s_re + c, s_im + c, NT, q, s_tw);
  if (valid) {
#pragma unroll
    for (int i = 0; i < E; ++i) Sb[off0 + i * step] = a[i];
  }
}

// NTW: the folded weight and data term arrive by streaming loads (maps where they outgrow
// the last-level cache; smaller maps keep them cached from one iteration to the next).
// S and P describe the columns of this launch (a range of kx starting at column kxo of the
// spectrum); Pw is the full row width, which lays out the folded weight and data term.
template <int L, int MODE, bool NTW = false>
__global__ void __launch_bounds__(16 * ColT<L>::T) k_fft_zw(float2* __restrict__ S, int P, int ntiles, int total,
                                                              long long pstride, long long bstride,
                                                              const float2* __restrict__ tw,
                                                              const float* __restrict__ ws,
                                                              const float2* __restrict__ cs,
                                                              double* __restrict__ partials, int NT, int Pw, int kxo) {
  __shared__ float s_re[L * 16];
  __shared__ float s_im[L * 16];
  __shared__ float2 s_tw[L];
  __shared__ double s_red[16];  // one slot per wave (up to 1024 threads)
  constexpr int T = ColT<L>::T;
  constexpr int E = RegPlan<L, T>::E;
  const int tid = threadIdx.x;
  const int c = tid % NT, q = tid / NT;
  static_assert(MODE >= 2 && MODE <= 4, "fused z modes");
  // Persistent blocks that load the next tile while transforming the current one: with a
  // grid of 8k blocks, XCD x (= blockIdx % 8) owns the contiguous tile range
  // [x chunk, (x+1) chunk) and its k-th block walks that range with stride k, so tiles
  // that share 128-byte lines (the folded weight rows of neighbouring 16-column tiles)
  // are in flight in one L2 at the same time.
  const int G = gridDim.x;
  const bool split = G >= 8 && (G & 7) == 0;
  const int xcd = split ? (int)(blockIdx.x & 7u) : 0;
  const int chunk = split ? (total + 7) >> 3 : total;
  const int nb = split ? G >> 3 : G;
  int t = xcd * chunk + (split ? (int)(blockIdx.x >> 3) : (int)blockIdx.x);
  const int t_end = min(total, xcd * chunk + chunk);
  // Block-uniform tile base pointers and unsigned 32-bit per-lane byte offsets of the
  // complex elements (every offset in a column is below nz*ny*P*8 <= 2^29 bytes), so the
  // loads take a scalar base and a 32-bit vector offset; the fp32 weight uses half the
  // offset.  A lane whose column lies past the last kx reads column 0 of its tile instead
  // (always in bounds) and stores nothing.
  const unsigned ps = (unsigned)pstride;
  const unsigned step = (unsigned)T * ps * 8u;
  auto tile_base = [&](int tt) -> long long {
    return (long long)(tt / ntiles) * bstride + (long long)(tt % ntiles) * NT;
  };
  auto lane_off = [&](int tt) -> unsigned {
    return ((unsigned)((tt % ntiles) * NT + c < P ? c : 0) + (unsigned)q * ps) * 8u;
  };
  // folded weight / data term: tile-major groups of WG = min(16, Pw) columns along z
  const int WG = Pw < 16 ? Pw : 16;
  auto wc_base = [&](int tt) -> long long {
    const int kx0 = kxo + (tt % ntiles) * NT;
    return ((long long)(tt / ntiles) * (Pw / WG) + kx0 / WG) * L * WG + kx0 % WG;
  };
  auto wc_off = [&](int tt) -> unsigned {  // element offset of the lane in its tile
    return (unsigned)((tt % ntiles) * NT + c < P ? c : 0) + (unsigned)(q * WG);
  };
  const unsigned wstep = (unsigned)(T * WG);

  float2 a[E];
  if (t < t_end) {
    const float2* __restrict__ Sb = S + tile_base(t);
    const unsigned o = lane_off(t);
#pragma unroll
    for (int i = 0; i < E; ++i) a[i] = ld_at(Sb, o + i * step);
  }
  for (int i = tid; i < L; i += blockDim.x) s_tw[i] = tw[i];
  double acc = 0.0;
  for (; t < t_end; t += nb) {
    __syncthreads();  // twiddles visible; the previous tile's last stage read the LDS planes
    // The lane indices pass through an empty asm statement so that the per-stage LDS
    // addresses derived from them are formed inside the loop where they are used, not
    // hoisted out of it and held in registers across all tiles.
    int cl = c, ql = q;
    asm volatile("" : "+v"(cl), "+v"(ql));
    float* re = s_re + cl;
    float* im = s_im + cl;
    const long long ub = tile_base(t);
    const int kx = (t % ntiles) * NT + cl;
    const bool valid = kx < P;
    const unsigned o = lane_off(t);
    const int tn = t + nb;
    const bool more = tn < t_end;  // block-uniform
    float2 nxt[E];
    float wv[E];
    float2 cv[E];
    // the folded weight and data term load during the forward stages
    const long long wb = wc_base(t);
    const unsigned ow = wc_off(t);
    const float* __restrict__ wsb = ws + wb;
#pragma unroll
    for (int i = 0; i < E; ++i) wv[i] = ld_nt<NTW>(wsb, (ow + i * wstep) * 4u);
    if constexpr (MODE != 4) {
      const float2* __restrict__ csb = cs + wb;
#pragma unroll
      for (int i = 0; i < E; ++i) cv[i] = ld_nt<NTW>(csb, (ow + i * wstep) * 8u);
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) cv[i] = make_float2(0.f, 0.f);
    }
    reg_stages<L, T, 0, false, 1>(a, re, im, NT, ql, s_tw);
    reg_stages<L, T, 1, false>(a, re, im, NT, ql, s_tw);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const float yr = a[i].x, yi = a[i].y;
      if constexpr (MODE == 3) {
        if (valid && kx > 0)
          acc += 2.0 * (0.5 * (double)wv[i] * ((double)yr * yr + (double)yi * yi) -
                        ((double)cv[i].x * yr + (double)cv[i].y * yi));
      }
      a[i] = make_float2(wv[i] * yr - cv[i].x, wv[i] * yi - cv[i].y);
    }
    __syncthreads();  // the forward transform's last stage read the LDS planes
    reg_stages<L, T, 0, true, 1>(a, re, im, NT, ql, s_tw);
    // the next tile loads during the remaining inverse stages
    if (more) {
      const float2* __restrict__ Sn = S + tile_base(tn);
      const unsigned on = lane_off(tn);
#pragma unroll
      for (int i = 0; i < E; ++i) nxt[i] = ld_at(Sn, on + i * step);
    }
    reg_stages<L, T, 1, true>(a, re, im, NT, ql, s_tw);

    if (valid && kx + kxo != 0) {  // the kx = 0 column belongs to k_dc_nyquist
      float2* __restrict__ Sb = S + ub;
#pragma unroll
      for (int i = 0; i < E; ++i) st_at(Sb, o + i * step, a[i]);
    }
    if (more) {
#pragma unroll
      for (int i = 0; i < E; ++i) a[i] = nxt[i];
    }
  }
  if constexpr (MODE == 3) {
    const double r = block_reduce<RED_OP_SUM>(acc, s_red);
    if (tid == 0) partials[blockIdx.x] = r;
  }
}

// ---------------------------------------------------------------- packed kx = 0 / nx/2 plane
// The packed slot holds Z = X0 + i XN where X0 and XN are the (complex) yz spectra of
// the real x-axis planes kx = 0 and kx = nx/2.  Their folded weights and data terms are
// stored as separate planes in [ky][kz] order so that a block reads contiguous runs.  Both are Hermitian in (ky, kz), so
// X0(k) = (Z(k) + conj Z(-k))/2 and XN(k) = (Z(k) - conj Z(-k))/(2i).  One block
// handles the column pair ky, -ky so that every partner is on chip.

template <int L, bool OBJ>
__global__ void __launch_bounds__(256) k_dc_nyquist(float2* __restrict__ S, int P, int ny,
                                                    const float2* __restrict__ tw, const float* __restrict__ w0p,
                                                    const float* __restrict__ wnyq, const float2* __restrict__ c0p,
                                                    const float2* __restrict__ cnyq, double* __restrict__ partials) {
  __shared__ float s_re[L * 2];
  __shared__ float s_im[L * 2];
  __shared__ double s_red[8];
  constexpr int T = DcT<L>::T;
  constexpr int NE = (L + T - 1) / T;
  const int tid = threadIdx.x;
  const int c = tid & 1, q = tid >> 1;
  const int ky = blockIdx.x;
  const int kyp = (ny - ky) % ny;
  const int myky = c == 0 ? ky : kyp;
  const long long pstride = (long long)ny * P;
  const long long base = (long long)myky * P;
  float* re = s_re + c;
  float* im = s_im + c;
  const float* pre = s_re + (1 - c);
  const float* pim = s_im + (1 - c);

  for (int p = q; p < L; p += T) {
    float2 v = S[base + p * pstride];
    re[p * 2] = v.x;
    im[p * 2] = v.y;
  }
  // the folded weights and data terms of the thread's points, requested before the forward
  // transform so that their latency overlaps it
  float w0v[NE], wnv[NE];
  float2 c0v[NE], cnv[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int kz = q + T * i;
    if (kz < L) {
      const long long offn = (long long)myky * L + kz;
      w0v[i] = w0p[offn];
      wnv[i] = wnyq[offn];
      c0v[i] = c0p ? c0p[offn] : make_float2(0.f, 0.f);
      cnv[i] = cnyq ? cnyq[offn] : make_float2(0.f, 0.f);
    }
  }
  fft_lds<L, false, T>(re, im, 2, q, tw);
  float2 nv[NE];
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int kz = q + T * i;
    if (kz < L) {
      const int kzp = (L - kz) % L;
      const float2 z1 = make_float2(re[kz * 2], im[kz * 2]);
      const float2 z2 = make_float2(pre[kzp * 2], pim[kzp * 2]);
      const float2 A = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y));
      const float2 dd = make_float2(0.5f * (z1.x - z2.x), 0.5f * (z1.y + z2.y));
      const float2 B = make_float2(dd.y, -dd.x);
      const float w0 = w0v[i], wn = wnv[i];
      const float2 c0 = c0v[i], cn = cnv[i];
      if constexpr (OBJ) {
        if (c == 0 || ky != kyp)
          acc += 0.5 * (double)w0 * ((double)A.x * A.x + (double)A.y * A.y) - ((double)c0.x * A.x + (double)c0.y * A.y) +
                 0.5 * (double)wn * ((double)B.x * B.x + (double)B.y * B.y) - ((double)cn.x * B.x + (double)cn.y * B.y);
      }
      const float2 g0 = make_float2(w0 * A.x - c0.x, w0 * A.y - c0.y);
      const float2 gn = make_float2(wn * B.x - cn.x, wn * B.y - cn.y);
      nv[i] = make_float2(g0.x - gn.y, g0.y + gn.x);
    }
  }
  if constexpr (OBJ) {
    double r = block_reduce<RED_OP_SUM>(acc, s_red);
    if (tid == 0) partials[blockIdx.x] = r;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int kz = q + T * i;
    if (kz < L) {
      re[kz * 2] = nv[i].x;
      im[kz * 2] = nv[i].y;
    }
  }
  fft_lds<L, true, T>(re, im, 2, q, tw);
  if (c == 0 || ky != kyp)
    for (int p = q; p < L; p += T) S[base + p * pstride] = make_float2(re[p * 2], im[p * 2]);
}

// Layout of the folded weight and data term (read only by the fused z pass): groups of
// WC_G = min(16, P) consecutive kx, each group contiguous along kz, i.e.
// [ky][kx / WC_G][kz][kx % WC_G], so that a 16-column tile reads them as one contiguous
// run along z instead of 64- and 128-byte pieces a plane apart.
__host__ __device__ __forceinline__ int wc_group(int P) { return P < 16 ? P : 16; }
__device__ __forceinline__ long long wc_index(const Dims& d, int kz, int ky, int kx) {
  const int G = wc_group(d.P);
  return (((long long)ky * (d.P / G) + kx / G) * d.nz + kz) * G + kx % G;
}

// ---------------------------------------------------------------- small maps: y, z passes in one launch
// Where a (ky, kz) plane of the packed spectrum fits in LDS, one block per column kx does
// for its plane what k_fft_cols<ny, 0>, k_fft_zw<nz, 2>, k_dc_nyquist and k_fft_cols<ny, 1>
// do between them: the y then z forward transforms, the weight step (G = w~ Y - c; at kx = 0
// the packed kx = 0 / nx/2 plane, split and rejoined as in k_dc_nyquist, its partners
// (-ky, -kz) being in the same plane), and the z then y inverse transforms.  One launch
// instead of four for maps whose iteration time is launch latency.  Plane in LDS [kz][ky].

// The ntr transforms of L points at base t * tstride and point stride ps, G = 256 / T at a
// time; every thread takes part in every barrier.
template <int L, bool INV>
__device__ __forceinline__ void plane_pass(float* re, float* im, int ntr, int tstride, int ps,
                                           const float2* __restrict__ tw) {
  constexpr int T = FftPlan<L>::T;
  constexpr int G = 256 / T;
  const int tid = threadIdx.x;
  for (int c0 = 0; c0 < ntr; c0 += G) {
    const int t = c0 + tid / T;
    const bool act = t < ntr && tid < G * T;
    const int off = act ? t * tstride : 0;
    fft_lds<L, INV, T>(re + off, im + off, ps, tid % T, tw, act);
  }
}

template <int NY, int NZ>
__global__ void __launch_bounds__(256) k_yz_plane(Dims d, float2* __restrict__ S, const float2* __restrict__ twy,
                                                  const float2* __restrict__ twz, const float* __restrict__ ws,
                                                  const float2* __restrict__ cs, const float* __restrict__ w0p,
                                                  const float* __restrict__ wnyq, const float2* __restrict__ c0p,
                                                  const float2* __restrict__ cnyq) {
  constexpr int NP = NY * NZ;
  __shared__ float s_re[NP];
  __shared__ float s_im[NP];
  __shared__ float2 s_twy[NY];
  __shared__ float2 s_twz[NZ];
  const int tid = threadIdx.x;
  const int kx = blockIdx.x;
  const int P = d.P;
  float2* __restrict__ Sc = S + kx;
  for (int i = tid; i < NY; i += 256) s_twy[i] = twy[i];
  for (int i = tid; i < NZ; i += 256) s_twz[i] = twz[i];
  for (int e = tid; e < NP; e += 256) {
    const float2 v = Sc[(long long)e * P];  // (kz NY + ky) P + kx
    s_re[e] = v.x;
    s_im[e] = v.y;
  }
  plane_pass<NY, false>(s_re, s_im, NZ, NY, 1, s_twy);
  plane_pass<NZ, false>(s_re, s_im, NY, 1, NY, s_twz);
  __syncthreads();
  if (kx > 0) {
    for (int e = tid; e < NP; e += 256) {
      const int kz = e / NY, ky = e % NY;
      const long long o = wc_index(d, kz, ky, kx);
      const float wv = ws[o];
      const float2 cv = cs[o];
      const float yr = s_re[e], yi = s_im[e];
      s_re[e] = wv * yr - cv.x;
      s_im[e] = wv * yi - cv.y;
    }
  } else {
    constexpr int EP = (NP + 255) / 256;
    float2 nv[EP];
#pragma unroll
    for (int i = 0; i < EP; ++i) {
      const int e = tid + 256 * i;
      if (e < NP) {
        const int kz = e / NY, ky = e % NY;
        const int ep = ((NZ - kz) % NZ) * NY + (NY - ky) % NY;
        const float2 z1 = make_float2(s_re[e], s_im[e]);
        const float2 z2 = make_float2(s_re[ep], s_im[ep]);
        const float2 A = make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y));
        const float2 dd = make_float2(0.5f * (z1.x - z2.x), 0.5f * (z1.y + z2.y));
        const float2 B = make_float2(dd.y, -dd.x);
        const long long offn = (long long)ky * NZ + kz;
        const float w0 = w0p[offn], wn = wnyq[offn];
        const float2 c0 = c0p ? c0p[offn] : make_float2(0.f, 0.f);
        const float2 cn = cnyq ? cnyq[offn] : make_float2(0.f, 0.f);
        const float2 g0 = make_float2(w0 * A.x - c0.x, w0 * A.y - c0.y);
        const float2 gn = make_float2(wn * B.x - cn.x, wn * B.y - cn.y);
        nv[i] = make_float2(g0.x - gn.y, g0.y + gn.x);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EP; ++i) {
      const int e = tid + 256 * i;
      if (e < NP) {
        s_re[e] = nv[i].x;
        s_im[e] = nv[i].y;
      }
    }
  }
  plane_pass<NZ, true>(s_re, s_im, NY, 1, NY, s_twz);
  plane_pass<NY, true>(s_re, s_im, NZ, NY, 1, s_twy);
  __syncthreads();
  for (int e = tid; e < NP; e += 256) Sc[(long long)e * P] = make_float2(s_re[e], s_im[e]);
}

// ---------------------------------------------------------------- x-axis real FFTs
// A real row of nx = 2M floats is read as M complex values z[n] = x[2n] + i x[2n+1].
// Forward: Z = FFT_M(z), X[k] = (Z[k] + conj Z[M-k])/2 + W^k (Z[k] - conj Z[M-k])/(2i),
// W = exp(-2 pi i / nx), packed X[0] = (X_0, X_M).  Inverse: Z[k] = E + i O with
// E = X[k] + conj X[M-k], O = (X[k] - conj X[M-k]) conj(W^k), z = IFFT_M(Z), which is
// the unnormalised inverse of the Hermitian row spectrum.
// Block: NR rows; thread (row c = tid / T, q = tid % T); LDS row pitch M + 4.

template <int M, bool BF>
__global__ void __launch_bounds__(256) k_r2c_x(const void* __restrict__ rin, float2* __restrict__ S, int nrows,
                                               const float2* __restrict__ twm, const float2* __restrict__ twn,
                                               int NR) {
  __shared__ float s_re[(M + 4) * 16];  // row pitch = 4 (mod 8): two rows per 32 lanes
  __shared__ float s_im[(M + 4) * 16];
  __shared__ float2 s_tw[M];
  constexpr int T = RegPlan<M>::T;
  constexpr int E = RegPlan<M>::E;
  const int tid = threadIdx.x;
  const int c = tid / T, q = tid % T;
  const int row = blockIdx.x * NR + c;
  const bool valid = row < nrows;
  float2 a[E];
  if constexpr (BF) {  // two bf16 samples per 32-bit word, even sample in the low half
    const uint32_t* src = reinterpret_cast<const uint32_t*>(rin) + (long long)row * M;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t wd = valid ? src[q + T * i] : 0u;
      a[i] = make_float2(bf16_to_f32((uint16_t)(wd & 0xFFFFu)), bf16_to_f32((uint16_t)(wd >> 16)));
    }
  } else {
    const float2* src = reinterpret_cast<const float2*>(rin) + (long long)row * M;
#pragma unroll
    for (int i = 0; i < E; ++i) a[i] = valid ? src[q + T * i] : make_float2(0.f, 0.f);
  }
  for (int i = tid; i < M; i += blockDim.x) s_tw[i] = twm[i];
  __syncthreads();
  float* re = s_re + c * (M + 4);
  float* im = s_im + c * (M + 4);
  fft_reg<M, false, RegPlan<M>::T, true>(a, re, im, 1, q, s_tw);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < E; ++i) {
    re[q + T * i] = a[i].x;
    im[q + T * i] = a[i].y;
  }
  __syncthreads();
  if (valid) {
    float2* dst = S + (long long)row * M;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int k = q + T * i;
      const float2 zk = a[i];
      float2 out;
      if (k == 0) {
        out = make_float2(zk.x + zk.y, zk.x - zk.y);
      } else {
        const float2 zm = make_float2(re[M - k], im[M - k]);
        const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
        const float2 d = make_float2(0.5f * (zk.x - zm.x), 0.5f * (zk.y + zm.y));
        const float2 o = make_float2(d.y, -d.x);
        out = cadd(e, cmul(twn[k], o));
      }
      dst[k] = out;
    }
  }
}

template <int M, bool BF>
__global__ void __launch_bounds__(256) k_c2r_x(const float2* __restrict__ S, void* __restrict__ rout, int nrows,
                                               const float2* __restrict__ twm, const float2* __restrict__ twn,
                                               int NR) {
  __shared__ float s_re[(M + 4) * 16];  // row pitch = 4 (mod 8): two rows per 32 lanes
  __shared__ float s_im[(M + 4) * 16];
  __shared__ float2 s_tw[M];
  constexpr int T = RegPlan<M>::T;
  constexpr int E = RegPlan<M>::E;
  const int tid = threadIdx.x;
  const int c = tid / T, q = tid % T;
  const int row = blockIdx.x * NR + c;
  const bool valid = row < nrows;
  const float2* src = S + (long long)row * M;
  float2 a[E];
  float2 wk[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int k = q + T * i;
    a[i] = valid ? src[k] : make_float2(0.f, 0.f);
    wk[i] = twn[k];
  }
  for (int i = tid; i < M; i += blockDim.x) s_tw[i] = twm[i];
  float* re = s_re + c * (M + 4);
  float* im = s_im + c * (M + 4);
#pragma unroll
  for (int i = 0; i < E; ++i) {
    re[q + T * i] = a[i].x;
    im[q + T * i] = a[i].y;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const int k = q + T * i;
    const float2 xk = a[i];
    if (k == 0) {
      a[i] = make_float2(xk.x + xk.y, xk.x - xk.y);
    } else {
      const float2 xm = make_float2(re[M - k], im[M - k]);
      const float2 e = make_float2(xk.x + xm.x, xk.y - xm.y);
      const float2 d = make_float2(xk.x - xm.x, xk.y + xm.y);
      const float2 o = cmulc(d, wk[i]);
      a[i] = make_float2(e.x - o.y, e.y + o.x);
    }
  }
  __syncthreads();
  fft_reg<M, true, RegPlan<M>::T, true>(a, re, im, 1, q, s_tw);
  if (valid) {
    if constexpr (BF) {
      uint32_t* dst = reinterpret_cast<uint32_t*>(rout) + (long long)row * M;
#pragma unroll
      for (int i = 0; i < E; ++i)
        dst[q + T * i] = (uint32_t)f32_to_bf16(a[i].x) | ((uint32_t)f32_to_bf16(a[i].y) << 16);
    } else {
      float2* dst = reinterpret_cast<float2*>(rout) + (long long)row * M;
#pragma unroll
      for (int i = 0; i < E; ++i) dst[q + T * i] = a[i];
    }
  }
}

// ---------------------------------------------------------------- fused stencil / prox
// Block tile: PT_TX x-columns by PT_TY y-rows, marching z over a slab of PT_ZC planes.
// LDS ring of two planes of the extrapolated map y (with a one-voxel halo) and two
// planes of the weighted dual p = v Dy / max(eps, |Dy|) (eq 16 with the TV weight),
// so that every y value crosses HBM about once per slab.  For voxel i at plane z:
//   g_tv(i) = sum_a p_a(i) - p_a(i + e_a)                    (eq 17)
//   z_i     = y_i - lr (g_data(i) + mu g_tv(i))              (eq 20)
//   x_i     = sign(z_i) max(|z_i| - lr lam u_i, 0)           (eq 21)
//   y'_i    = x_i + m' (x_i - x_k,i)                         (momentum)
// Compensated mode: x is stored as fp32 hi + bf16 lo and the step, prox and momentum
// are evaluated in fp64; the stencil and the FFT see y rounded to fp32.
// Check mode: y = x_k, nothing is written except per-block fp64 partials of
// lam sum u|x|, mu sum v huber(|Dx|), mu sum v |Dx|, |x - T(x)|^2 and |x|^2.

template <bool COMP>
__device__ __forceinline__ double load_x(const float* __restrict__ hi, const uint16_t* __restrict__ lo, long long i) {
  if constexpr (COMP) return (double)hi[i] + (double)bf16_to_f32(lo[i]);
  else return (double)hi[i];
}

// Raw iterate words of one voxel (x_k and, when the momentum is non-zero, x_{k-1}),
// fetched one z-step ahead of their use.
struct RawX {
  float xh, oh;
  uint16_t xl, ol;
};

// 1 / max(eps, sqrt(n2)).  Where eps^2 is a normal float, n2 > eps^2 is too, and the
// hardware reciprocal square root gives the library's result without its denormal
// scaling; otherwise the library routine handles the denormal range.
__device__ __forceinline__ float inv_norm(const ProxArgs& a, float n2) {
  if (a.eps2_normal) return n2 > a.eps * a.eps ? __builtin_amdgcn_rsqf(n2) : 1.0f / a.eps;
  return n2 > a.eps * a.eps ? rsqrtf(n2) : 1.0f / a.eps;
}

// phi_eps(|Dy|) of eq 14 in fp64 from |Dy|^2: t^2 / (2 eps) below eps, t - eps/2 above.
__device__ __forceinline__ double huber64(float n2, float eps) {
  const double nd = sqrt((double)n2);
  const double e = eps;
  return nd < e ? nd * nd / (2.0 * e) : nd - 0.5 * e;
}

template <bool COMP>
__device__ __forceinline__ void fetch_raw(const ProxArgs& a, long long i, RawX& r) {
  r.xh = a.xk_hi[i];
  if constexpr (COMP) r.xl = a.xk_lo[i];
  if (a.read_old) {
    r.oh = a.xo_hi[i];
    if constexpr (COMP) r.ol = a.xo_lo[i];
  }
}

// y = x_k + m (x_k - x_{k-1}) from raw words: fp64 from the compensated pair, else fp32.
template <bool COMP>
__device__ __forceinline__ void eval_raw(const ProxArgs& a, const RawX& r, double& y, double& xk) {
  if constexpr (COMP) {
    xk = (double)r.xh + (double)bf16_to_f32(r.xl);
    y = xk;
    if (a.read_old) {
      const double xo = (double)r.oh + (double)bf16_to_f32(r.ol);
      y = xk + a.m * (xk - xo);
    }
  } else {
    float yf = r.xh;
    if (a.read_old) yf = r.xh + (float)a.m * (r.xh - r.oh);
    xk = r.xh;
    y = yf;
  }
}

// MON (with CHECK false): the iteration as usual, and per-block fp64 partials of the
// penalty terms of the objective at y_k: sum u |y|, sum v phi_eps(|Dy|), sum (y - x_prev)^2
// (3 groups of gridDim.x in a.partials).
template <int ST, bool CHECK, bool MON = false>
__global__ void __launch_bounds__(256) k_prox_tv(ProxArgs a, int ntx, int nty) {
  static_assert(!(CHECK && MON), "check mode evaluates the objective itself");
  constexpr bool COMP = ST == ST_COMP;
  constexpr bool BF = ST == ST_BF16;
  constexpr int TX = PT_TX, TY = PT_TY;
  constexpr int YW = TX + 2, YH = TY + 2;  // y plane with halo
  constexpr int PW = TX + 1, PH = TY + 1;  // p plane with the +1 shell
  constexpr int NPP = (PW * PH + 255) / 256;
  constexpr int NHALO = 2 * YW + 2 * TY;
  constexpr int NOWN = TY / 4;  // voxels per thread and plane: rows ty + 4 h
  static_assert(TY % 4 == 0 && NHALO <= 256, "tile shape");
  __shared__ float sY[2][YH][YW];
  __shared__ float sP[2][3][PH][PW];
  __shared__ double s_red[8];

  const int tid = threadIdx.x;
  const int tx = tid & 63, ty = tid >> 6;  // owns (tx, ty + 4 h), h < NOWN
  // consecutive tiles (one x row of tiles at nx = 512) on one XCD, so that the x-halo
  // columns a tile reads are the L2 lines its neighbour tiles fetch
  const int blk = (gridDim.x >= 64 && (int)blockIdx.x < (int)(gridDim.x & ~63u))
                      ? (int)((blockIdx.x & ~63u) | ((blockIdx.x & 7u) << 3) | ((blockIdx.x >> 3) & 7u))
                      : (int)blockIdx.x;
  const int bx = blk % ntx;
  const int by = (blk / ntx) % nty;
  const int bz = blk / (ntx * nty);
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int x0 = bx * TX, y0 = by * TY;
  const int z0 = bz * a.zc;
  const int z1 = min(z0 + a.zc, nz);
  const long long plane = (long long)nx * ny;
  // periodic wrap of a coordinate (any grid size; the offsets below are computed once per block)
  auto wrapm = [](int v, int n) { return ((v % n) + n) % n; };

  // own voxels: in-plane offsets
  const int gx = wrapm(x0 + tx, nx);
  const bool vx = (x0 + tx) < nx;
  int own_off[NOWN];
  bool vown[NOWN];
#pragma unroll
  for (int h = 0; h < NOWN; ++h) {
    own_off[h] = wrapm(y0 + ty + 4 * h, ny) * nx + gx;
    vown[h] = vx && (y0 + ty + 4 * h) < ny;
  }
  // halo point of this thread (tid < NHALO)
  const bool has_halo = tid < NHALO;
  int hlx = 0, hly = 0;
  if (tid < YW) { hly = -1; hlx = tid - 1; }
  else if (tid < 2 * YW) { hly = TY; hlx = tid - YW - 1; }
  else if (tid < 2 * YW + TY) { hlx = -1; hly = tid - 2 * YW; }
  else { hlx = TX; hly = tid - 2 * YW - TY; }
  const int halo_off = wrapm(y0 + hly, ny) * nx + wrapm(x0 + hlx, nx);
  // p points of this thread
  int p_off[NPP];
  bool p_ok[NPP];
#pragma unroll
  for (int t = 0; t < NPP; ++t) {
    const int idx = tid + 256 * t;
    p_ok[t] = idx < PW * PH;
    const int ly = idx / PW, lx = idx - ly * PW;
    p_off[t] = wrapm(y0 + ly, ny) * nx + wrapm(x0 + lx, nx);
  }

  auto pz_of = [&](int zz) { return (long long)(zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz)) * plane; };
  auto fetch_plane = [&](int zz, RawX* own, RawX& halo, float* vv) {
    const long long pz = pz_of(zz);
#pragma unroll
    for (int h = 0; h < NOWN; ++h) fetch_raw<COMP>(a, pz + own_off[h], own[h]);
    if (has_halo) fetch_raw<COMP>(a, pz + halo_off, halo);
#pragma unroll
    for (int t = 0; t < NPP; ++t) vv[t] = (a.v && p_ok[t]) ? ld_real<BF>(a.v, pz + p_off[t]) : 1.0f;
  };
  // inputs of the outputs of plane zz: data gradient, l1 weight and (gamma term) prior map
  auto fetch_out = [&](int zz, float* g, float* uu, float* xp) {
    const long long pz = (long long)zz * plane;
#pragma unroll
    for (int h = 0; h < NOWN; ++h) {
      const long long i = pz + own_off[h];
      if constexpr (CHECK) g[h] = vown[h] ? a.gin[i] : 0.f;
      else g[h] = vown[h] ? ld_real<BF>(a.rbuf, i) : 0.f;
      uu[h] = (a.u && vown[h]) ? ld_real<BF>(a.u, i) : 1.0f;
      xp[h] = (a.xprev && vown[h]) ? a.xprev[i] : 0.f;
    }
  };
  auto store_plane = [&](int buf, const RawX* own, const RawX& halo, double* ys, double* xks) {
#pragma unroll
    for (int h = 0; h < NOWN; ++h) {
      double yv, xv;
      eval_raw<COMP>(a, own[h], yv, xv);
      ys[h] = yv;
      xks[h] = xv;
      sY[buf][ty + 4 * h + 1][tx + 1] = (float)yv;
    }
    if (has_halo) {
      double yv, xv;
      eval_raw<COMP>(a, halo, yv, xv);
      sY[buf][hly + 1][hlx + 1] = (float)yv;
    }
  };

  double acc_l1 = 0.0, acc_hub = 0.0, acc_tv0 = 0.0, acc_kkt = 0.0, acc_x2 = 0.0, acc_gam = 0.0;
  // p on the (TX+1) x (TY+1) points of a plane from y planes yn (this plane) and yp (below).
  auto compute_p = [&](int yn, int yp, int dst, const float* vv, bool count) {
#pragma unroll
    for (int t = 0; t < NPP; ++t) {
      if (!p_ok[t]) continue;
      const int idx = tid + 256 * t;
      const int ly = idx / PW, lx = idx - ly * PW;
      const float yc = sY[yn][ly + 1][lx + 1];
      const float dxv = yc - sY[yn][ly + 1][lx];
      const float dyv = yc - sY[yn][ly][lx + 1];
      const float dzv = yc - sY[yp][ly + 1][lx + 1];
      // v / max(eps, |Dy|) with one reciprocal square root
      const float n2 = dxv * dxv + dyv * dyv + dzv * dzv;
      const float inv = inv_norm(a, n2);
      const float sc = vv[t] * inv;
      sP[dst][0][ly][lx] = sc * dzv;
      sP[dst][1][ly][lx] = sc * dyv;
      sP[dst][2][ly][lx] = sc * dxv;
      if constexpr (CHECK) {
        if (count && lx < TX && ly < TY && (x0 + lx) < nx && (y0 + ly) < ny) {
          const double nd = sqrt((double)n2);
          const double e = a.eps;
          const double hub = nd < e ? nd * nd / (2.0 * e) : nd - 0.5 * e;
          acc_hub += (double)vv[t] * hub;
          acc_tv0 += (double)vv[t] * nd;
        }
      } else if constexpr (MON) {
        if (count && lx < TX && ly < TY && (x0 + lx) < nx && (y0 + ly) < ny)
          acc_hub += (double)vv[t] * huber64(n2, a.eps);
      }
    }
  };

  // ---- prologue: planes z0-1 and z0 into LDS, p(z0), and the first prefetches
  RawX rown[NOWN], rhalo;
  float rv[NPP];
  double own_y[NOWN], own_xk[NOWN], nxt_y[NOWN], nxt_xk[NOWN];
  float g_cur[NOWN], u_cur[NOWN], xp_cur[NOWN];
  {
    double dy_[NOWN], dx_[NOWN];
    fetch_plane(z0 - 1, rown, rhalo, rv);
    store_plane(0, rown, rhalo, dy_, dx_);
    fetch_plane(z0, rown, rhalo, rv);
    store_plane(1, rown, rhalo, own_y, own_xk);
  }
  fetch_out(z0, g_cur, u_cur, xp_cur);
  __syncthreads();
  compute_p(1, 0, 0, rv, true);
  fetch_plane(z0 + 1, rown, rhalo, rv);
  int cur = 0, ycur = 1;

  for (int z = z0; z < z1; ++z) {
    // y of plane z+1 from the words fetched during the previous step
    store_plane(ycur ^ 1, rown, rhalo, nxt_y, nxt_xk);
    float vv_use[NPP];
#pragma unroll
    for (int t = 0; t < NPP; ++t) vv_use[t] = rv[t];
    float g_use[NOWN], u_use[NOWN], xp_use[NOWN];
#pragma unroll
    for (int h = 0; h < NOWN; ++h) {
      g_use[h] = g_cur[h];
      u_use[h] = u_cur[h];
      xp_use[h] = xp_cur[h];
    }
    // prefetch plane z+2 and the outputs' inputs of plane z+1
    if (z + 1 < z1) {
      fetch_plane(z + 2, rown, rhalo, rv);
      fetch_out(z + 1, g_cur, u_cur, xp_cur);
    }
    __syncthreads();
    compute_p(ycur ^ 1, ycur, cur ^ 1, vv_use, (z + 1) < z1);
    __syncthreads();
    const long long pz = (long long)z * plane;
#pragma unroll
    for (int h = 0; h < NOWN; ++h) {
      const int ly = ty + 4 * h, lx = tx;
      const float gtv = sP[cur][0][ly][lx] + sP[cur][1][ly][lx] + sP[cur][2][ly][lx] - sP[cur][2][ly][lx + 1] -
                        sP[cur][1][ly + 1][lx] - sP[cur ^ 1][0][ly][lx];
      if (vown[h]) {
        const long long i = pz + own_off[h];
        const float gd = g_use[h];
        const float uu = u_use[h];
        const float xp = xp_use[h];
        if constexpr (COMP) {
          const double y = own_y[h];
          const double dprior = y - (double)xp;
          const double zv = y - a.lr * ((double)gd + a.mu * (double)gtv + 2.0 * a.gamma * dprior);
          const double t = a.lr * a.lam * (double)uu;
          const double az = fabs(zv) - t;
          const double xn = az > 0.0 ? copysign(az, zv) : 0.0;
          if constexpr (CHECK) {
            acc_l1 += (double)uu * fabs(y);
            acc_kkt += (y - xn) * (y - xn);
            acc_x2 += y * y;
            acc_gam += dprior * dprior;
          } else {
            if constexpr (MON) {
              acc_l1 += (double)uu * fabs(y);
              acc_gam += dprior * dprior;
            }
            const float hi = (float)xn;
            const uint16_t lo = f32_to_bf16((float)(xn - (double)hi));
            a.xn_hi[i] = hi;
            a.xn_lo[i] = lo;
            const double xs = (double)hi + (double)bf16_to_f32(lo);
            const double yn = xs + a.m_next * (xs - own_xk[h]);
            st_real<false>(a.rbuf, i, (float)yn);
          }
        } else {
          const float y = (float)own_y[h];
          const float dprior = y - xp;
          const float zv = y - (float)a.lr * (gd + (float)a.mu * gtv + 2.0f * (float)a.gamma * dprior);
          const float t = (float)a.lr * (float)a.lam * uu;
          const float az = fabsf(zv) - t;
          const float xn = az > 0.f ? copysignf(az, zv) : 0.f;
          if constexpr (CHECK) {
            acc_l1 += (double)uu * fabs((double)y);
            acc_kkt += ((double)y - xn) * ((double)y - xn);
            acc_x2 += (double)y * y;
            acc_gam += (double)dprior * dprior;
          } else {
            if constexpr (MON) {
              acc_l1 += (double)uu * fabs((double)y);
              acc_gam += (double)dprior * dprior;
            }
            a.xn_hi[i] = xn;
            const float xk = (float)own_xk[h];
            st_real<BF>(a.rbuf, i, xn + (float)a.m_next * (xn - xk));
          }
        }
      }
    }
    cur ^= 1;
    ycur ^= 1;
#pragma unroll
    for (int h = 0; h < NOWN; ++h) {
      own_y[h] = nxt_y[h];
      own_xk[h] = nxt_xk[h];
    }
  }
  if constexpr (CHECK) {
    const int nb = gridDim.x;
    double r;
    r = block_reduce<RED_OP_SUM>(acc_l1, s_red);
    if (tid == 0) a.partials[0 * nb + blk] = r;
    r = block_reduce<RED_OP_SUM>(acc_hub, s_red);
    if (tid == 0) a.partials[1 * nb + blk] = r;
    r = block_reduce<RED_OP_SUM>(acc_tv0, s_red);
    if (tid == 0) a.partials[2 * nb + blk] = r;
    r = block_reduce<RED_OP_SUM>(acc_kkt, s_red);
    if (tid == 0) a.partials[3 * nb + blk] = r;
    r = block_reduce<RED_OP_SUM>(acc_x2, s_red);
    if (tid == 0) a.partials[4 * nb + blk] = r;
    r = block_reduce<RED_OP_SUM>(acc_gam, s_red);
    if (tid == 0) a.partials[5 * nb + blk] = r;
  } else if constexpr (MON) {
    const int nb = gridDim.x;
    double r;
    r = block_reduce<RED_OP_SUM>(acc_l1, s_red);
    if (tid == 0) a.partials[blk] = r;
    r = block_reduce<RED_OP_SUM>(acc_hub, s_red);
    if (tid == 0) a.partials[nb + blk] = r;
    r = block_reduce<RED_OP_SUM>(acc_gam, s_red);
    if (tid == 0) a.partials[2 * nb + blk] = r;
  }
}

// ---------------------------------------------------------------- fused x transforms + stencil/prox
// One SPG step on full-width tiles: NX (= nx) x-columns by PF_TY y-rows, marched along z
// over a slab of a.zc planes.  The data gradient of a plane comes in as the rows of its
// packed x-spectrum (after the y and z passes) and is turned into real rows here (the
// x-axis inverse real FFT); y_{k+1} of the plane goes out as the x-spectrum of its rows
// (the x-axis forward real FFT of the next iteration).  The stencil needs no x halo:
// rows wrap inside the tile.  Per plane, LDS holds y on three planes (z-1, z, z+1) with
// one halo row on each side, and sc = v / max(eps, |Dy|) on two planes (z, z+1) with
// the row below the tile; the p = sc Dy terms of D^T p are formed from these rings.
// Thread (x = tid % NX, r = tid / NX) owns rows r + 2h (h < PF_TY/2) and halo row -1
// (r = 0) or PF_TY (r = 1).  A z step has two phases: (1) y(z+1) into the ring, and the
// iterate words of plane z+2 requested at once; (2) after a barrier, sc(z+1) into its slot
// and, for the thread's own voxels, straight into the outputs of plane z; then a barrier.
// The row transforms are batched over PF_KB planes: the gradient rows of a batch sit in
// LDS while its planes are stepped (each plane's y_{k+1} rows replace its gradient rows),
// then one transform phase on all threads takes the batch's y_{k+1} rows forward into S
// (threads [0, R)) while the other half inverts the next batch's gradient rows, as the
// conjugate of the forward transform of the conjugate (threads [R, 2R), R = PF_KB*PF_TY
// rows of FT threads).  The arithmetic of every output is that of k_c2r_x, k_prox_tv and
// k_r2c_x in sequence, except that with bf16 storage the gradient and y_{k+1} rows stay
// fp32 (they never reach HBM here).  At nx = 512 the transforms are instead pipelined with
// the plane steps over batches of PP_KB planes: each row transform lives in one wavefront,
// so its stages need no block barrier and are spread over the barrier intervals of the
// plane steps, the memory-bound work hiding the transforms' arithmetic and LDS exchanges.
constexpr int PF_TY = 4;
constexpr int PF_KB = 4;
constexpr int PP_KB = 2;  // planes per batch of the pipelined variant

template <int M>
struct PfT {  // threads per row of the M-point complex transforms
  static constexpr int T = largest_divisor_le(plan_gcd(M), 32);
  static constexpr int E = M / T;
};

// PRIOR: the gamma term's previous map is given (else it is 0).  NT: x_{k+1} and the
// spectrum rows go out by streaming stores (maps whose spectrum outgrows the last-level
// cache; smaller maps are read back by the next pass while still cached).  MON: also the
// per-block fp64 partials of the penalty terms of the objective at y_k (eq 31 with eq 14):
// sum u |y|, sum v phi_eps(|Dy|) and sum (y - x_prev)^2, into a.partials (3 groups of
// gridDim.x).
template <int NX, int ST, bool PRIOR, bool NT, bool MON = false>
__global__ void __launch_bounds__(2 * NX) k_prox_fft(ProxArgs a, float2* __restrict__ S,
                                                     const float2* __restrict__ twm,
                                                     const float2* __restrict__ twn, int nty) {
  constexpr bool COMP = ST == ST_COMP;
  constexpr bool BF = ST == ST_BF16;
  // 256- and 512-wide maps: the row transforms are pipelined with the plane steps (see below)
  constexpr bool PIPE = NX == 512 || NX == 256;
  constexpr int TY = PF_TY, KB = PIPE ? PP_KB : PF_KB;
  constexpr int M = NX / 2;
  constexpr int FT = PfT<M>::T, FE = PfT<M>::E;
  constexpr int NR = KB * TY;  // rows of one batch
  constexpr int NG = PIPE ? 3 : 1;  // batches of rows in LDS
  using VT = typename std::conditional<BF, uint16_t, float>::type;  // penalty-weight word
  constexpr int NO = TY / 2;  // own rows per thread
  static_assert(TY % 2 == 0 && 2 * NR * FT == (PIPE ? NX : 2 * NX), "one transform row share per thread");
  static_assert(!PIPE || (FE == 8 && 64 % FT == 0 && RegPlan<M, FT>::ns == 3),
                "pipelined rows: 8 points per lane, a row within one wavefront, three stages");
  __shared__ float sY[3][TY + 2][NX];
  __shared__ float sSC[2][TY + 1][NX];
  __shared__ float sG[NG][KB][TY][NX];  // gradient rows of a batch, then its y_{k+1} rows
  __shared__ float sFre[PIPE ? 1 : 2 * NR][M + 1];
  __shared__ float sFim[PIPE ? 1 : 2 * NR][M + 1];
  // pipelined variant: the real and imaginary planes of a row 4M bytes apart (one address for
  // both), plus one pad word past the last row
  __shared__ float sFx[PIPE ? 2 * NR * 2 * M + 1 : 1];
  __shared__ float2 s_tw[M];   // M-point transform twiddles
  __shared__ float2 s_twn[M];  // W^k of the real-row pre- and post-processing

  const int tid = threadIdx.x;
  int x = tid % NX, r = tid / NX;
  int xm = (x + NX - 1) % NX, xp = (x + 1) % NX;
  // Pipelined kernel: neighbouring tiles on one XCD, so that the halo rows a tile reads are
  // often still in that XCD's L2 from its neighbours' own rows (measured 3% faster at
  // nx = 512; no gain with the batched transforms, which leave the memory pipe idle longer)
  const int bid = PIPE ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  const int by = bid % nty;
  const int bz = bid / nty;
  const int ny = a.ny, nz = a.nz;
  const int y0 = by * TY;
  const int z0 = bz * a.zc;
  const int z1 = min(z0 + a.zc, nz);
  const long long plane = (long long)NX * ny;
  // In-plane element offsets (below 2^18): own rows ly = r + 2h (inside the grid, as ny is
  // a multiple of TY) and the halo row; global accesses take a block-uniform plane base
  // and these offsets scaled to bytes.
  unsigned own_off[NO];
#pragma unroll
  for (int h = 0; h < NO; ++h) own_off[h] = (unsigned)((y0 + r + 2 * h) * NX + x);
  const int hly = r == 0 ? -1 : TY;
  unsigned halo_off = (unsigned)((((y0 + hly) % ny + ny) % ny) * NX + x);
  // transform role: thread row fr in [0, 2 NR): rows [0, NR) forward (y_{k+1} of the
  // current batch, row fr = plane-in-batch * TY + tile row), rows [NR, 2 NR) inverse (the
  // gradient of the next batch, same numbering)
  int fr = tid / FT, fq = tid % FT;

  auto slot3 = [](int zz) { return ((zz % 3) + 3) % 3; };
  auto pz_of = [&](int zz) { return (long long)(zz < 0 ? zz + nz : (zz >= nz ? zz - nz : zz)) * plane; };
  // x_{k-1} words are read unconditionally (from x_k when the momentum term is off: m = 0
  // then and y = x_k), so that every load takes a block-uniform base
  const float* __restrict__ xo_hi = a.read_old ? a.xo_hi : a.xk_hi;
  const uint16_t* __restrict__ xo_lo = a.read_old ? a.xo_lo : a.xk_lo;
  auto fetch_one = [&](long long pz, unsigned o, RawX& w) {
    w.xh = ld_at(a.xk_hi + pz, o * 4u);
    if constexpr (COMP) w.xl = ld_at(a.xk_lo + pz, o * 2u);
    w.oh = ld_at(xo_hi + pz, o * 4u);
    if constexpr (COMP) w.ol = ld_at(xo_lo + pz, o * 2u);
  };
  auto ld_w = [&](const void* base, long long pz, unsigned o) -> float {
    const VT* b = reinterpret_cast<const VT*>(base) + pz;
    if constexpr (BF) return bf16_to_f32(ld_at(b, o * 2u));
    else return ld_at(b, o * 4u);
  };
  auto fetch_x = [&](int zz, RawX* own, RawX& halo) {
    const long long pz = pz_of(zz);
#pragma unroll
    for (int h = 0; h < NO; ++h) fetch_one(pz, own_off[h], own[h]);
    fetch_one(pz, halo_off, halo);
  };
  auto fetch_v = [&](int zz, float* vv) {
    const long long pz = pz_of(zz);
    if (a.v) {
#pragma unroll
      for (int h = 0; h < NO; ++h) vv[h] = ld_w(a.v, pz, own_off[h]);
      vv[NO] = r == 1 ? ld_w(a.v, pz, halo_off) : 1.0f;
    } else {
#pragma unroll
      for (int h = 0; h <= NO; ++h) vv[h] = 1.0f;
    }
  };
  auto fetch_out = [&](int zz, float* uu, float* xq) {
    long long pz = (long long)zz * plane;
    asm volatile("" : "+s"(pz));
#pragma unroll
    for (int h = 0; h < NO; ++h) {
      uu[h] = a.u ? ld_w(a.u, pz, own_off[h]) : 1.0f;
      if constexpr (PRIOR) xq[h] = ld_at(a.xprev + pz, own_off[h] * 4u);
      else xq[h] = 0.f;
    }
  };
  // spectrum rows of the batch starting at plane zb for the inverse half (row fr - NR)
  // (block-uniform base at plane zb, tile row y0; per-thread 32-bit byte offsets)
  auto row_off = [&](int row) { return (unsigned)(((row / TY) * ny + row % TY) * M + fq) * 8u; };
  auto fetch_spec = [&](int zb, float2* sr) {
    const int zz = zb + (fr - NR) / TY;
    if ((!PIPE || fr < 2 * NR) && fr >= NR && zz < z1) {
      const float2* __restrict__ src = S + ((long long)zb * ny + y0) * M;
      const unsigned o = row_off(fr - NR);
#pragma unroll
      for (int i = 0; i < FE; ++i) sr[i] = ld_at(src, o + (unsigned)(FT * i) * 8u);
    }
  };
  // y = x_k + m (x_k - x_{k-1}) as eval_raw, without its branch: with the momentum term
  // off, m = 0 and the x_{k-1} words are x_k's, so y = x_k (up to the sign of a zero y,
  // which no output depends on)
  auto eval = [&](const RawX& w, double& y, double& xk) {
    if constexpr (COMP) {
      xk = (double)w.xh + (double)bf16_to_f32(w.xl);
      const double xo = (double)w.oh + (double)bf16_to_f32(w.ol);
      y = xk + a.m * (xk - xo);
    } else {
      y = w.xh + (float)a.m * (w.xh - w.oh);
      xk = w.xh;
    }
  };
  // y of a plane into the ring; own y (fp64 in the compensated mode) and x_k kept
  auto store_plane = [&](int zz, const RawX* own, const RawX& halo, double* ys, double* xks) {
    float(*Y)[NX] = sY[slot3(zz)];
#pragma unroll
    for (int h = 0; h < NO; ++h) {
      double yv, xv;
      eval(own[h], yv, xv);
      ys[h] = yv;
      xks[h] = xv;
      Y[r + 2 * h + 1][x] = (float)yv;
    }
    double yv, xv;
    eval(halo, yv, xv);
    Y[hly + 1][x] = (float)yv;
  };
  // |Dy|^2 at row ly of plane zz, column x (backward differences)
  auto n2_at = [&](int zz, int ly) {
    const float(*Y)[NX] = sY[slot3(zz)];
    const float(*Yp)[NX] = sY[slot3(zz - 1)];
    const float yc = Y[ly + 1][x];
    const float dxv = yc - Y[ly + 1][xm];
    const float dyv = yc - Y[ly][x];
    const float dzv = yc - Yp[ly + 1][x];
    return dxv * dxv + dyv * dyv + dzv * dzv;
  };
  // objective partials (MON): penalty terms of the voxels this thread owns on this slab
  double acc_l1 = 0.0, acc_hub = 0.0, acc_gam = 0.0;
  // sc = v / max(eps, |Dy|): writes the ring slot of plane zz and returns the thread's own
  // values in sco
  auto compute_sc = [&](int zz, const float* vv, float* sco) {
    float(*SC)[NX] = sSC[zz & 1];
#pragma unroll
    for (int h = 0; h < NO; ++h) {
      const float n2 = n2_at(zz, r + 2 * h);
      sco[h] = vv[h] * inv_norm(a, n2);
      SC[r + 2 * h][x] = sco[h];
      if constexpr (MON) {
        if (zz < z1) acc_hub += (double)vv[h] * huber64(n2, a.eps);
      }
    }
    if (r == 1) SC[TY][x] = vv[NO] * inv_norm(a, n2_at(zz, TY));
  };
  // One transform phase.  Forward half (fr < NR): the y_{k+1} rows of the batch at plane
  // zf (planes < zf_end) from sG into S.  Inverse half: the spectrum rows in `sa` of the
  // batch at plane zi (planes < z1) into sG, real rows.  Either batch may be empty.
  auto transform_phase = [&](int zf, int zf_end, int zi, float2* sa) {
    const bool fwd = fr < NR;
    const int row = fwd ? fr : fr - NR;
    const int zz = (fwd ? zf : zi) + row / TY;
    const bool act = fwd ? zz < zf_end : zz < z1;
    float* fre = &sFre[fr][0];
    float* fim = &sFim[fr][0];
    float(*G)[NX] = sG[0][row / TY];
    float2 v[FE];
    if (act) {
      if (fwd) {
#pragma unroll
        for (int i = 0; i < FE; ++i) v[i] = *reinterpret_cast<const float2*>(&G[row % TY][2 * (fq + FT * i)]);
      } else {
#pragma unroll
        for (int i = 0; i < FE; ++i) {
          fre[fq + FT * i] = sa[i].x;
          fim[fq + FT * i] = sa[i].y;
        }
      }
    }
    // point i of this thread is k = fq + FT i; its mirror M - k is element FT (FE - 1 - i)
    // past mb (k = 0, only at fq = 0 and i = 0, reads the row's pad word and is replaced)
    const int mb = M - fq - FT * (FE - 1);
    __syncthreads();
    // inverse half: Z[k] = E + i O from the row and its mirror (as k_c2r_x), conjugated
    if (act && !fwd) {
#pragma unroll
      for (int i = 0; i < FE; ++i) {
        const float2 xk = sa[i];
        const float2 xmr = make_float2(fre[mb + FT * (FE - 1 - i)], fim[mb + FT * (FE - 1 - i)]);
        const float2 e = make_float2(xk.x + xmr.x, xk.y - xmr.y);
        const float2 d = make_float2(xk.x - xmr.x, xk.y + xmr.y);
        const float2 o = cmulc(d, s_twn[fq + FT * i]);
        float2 zk = make_float2(e.x - o.y, e.y + o.x);
        if (i == 0 && fq == 0) zk = make_float2(xk.x + xk.y, xk.x - xk.y);
        v[i] = make_float2(zk.x, -zk.y);
      }
    }
    __syncthreads();
    fft_reg<M, false, FT, true>(v, fre, fim, 1, fq, s_tw, act);
    if (act && !fwd) {  // z = conj(FFT(conj Z)): interleaved real samples of the row
#pragma unroll
      for (int i = 0; i < FE; ++i)
        *reinterpret_cast<float2*>(&G[row % TY][2 * (fq + FT * i)]) = make_float2(v[i].x, -v[i].y);
    }
    __syncthreads();
    // forward half: X[k] from Z[k] and Z[M-k] (as k_r2c_x) into the spectrum rows
    if (act && fwd) {
#pragma unroll
      for (int i = 0; i < FE; ++i) {
        fre[fq + FT * i] = v[i].x;
        fim[fq + FT * i] = v[i].y;
      }
    }
    __syncthreads();
    if (act && fwd) {
      float2* __restrict__ dst = S + ((long long)zf * ny + y0) * M;
      const unsigned ob = row_off(row);
#pragma unroll
      for (int i = 0; i < FE; ++i) {
        const float2 zk = v[i];
        const float2 zm = make_float2(fre[mb + FT * (FE - 1 - i)], fim[mb + FT * (FE - 1 - i)]);
        const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
        const float2 d = make_float2(0.5f * (zk.x - zm.x), 0.5f * (zk.y + zm.y));
        const float2 o = make_float2(d.y, -d.x);
        float2 out = cadd(e, cmul(s_twn[fq + FT * i], o));
        if (i == 0 && fq == 0) out = make_float2(zk.x + zk.y, zk.x - zk.y);
        st_nt<NT>(dst, ob + (unsigned)(FT * i) * 8u, out);
      }
    }
  };

  // ---- one plane step, first half: y of plane z+1 from the words fetched during the
  // previous step into the ring; the words of plane z+2 are requested at once
  RawX rown[NO], rhalo;
  float rv[NO + 1];
  double own_y[NO], own_xk[NO], nxt_y[NO], nxt_xk[NO];
  float u_cur[NO], xq_cur[NO], u_nxt[NO], xq_nxt[NO];
  auto step_a = [&](int z) {
    // The lane indices pass through empty asm statements so that the LDS and global
    // addresses derived from them are formed inside the loop where they are used, not
    // hoisted out of it and held in registers across all planes.
    asm volatile("" : "+v"(x), "+v"(r), "+v"(xm), "+v"(xp), "+v"(halo_off));
#pragma unroll
    for (int h = 0; h < NO; ++h) asm volatile("" : "+v"(own_off[h]));
    asm volatile("" : "+v"(fr), "+v"(fq));
    store_plane(z + 1, rown, rhalo, nxt_y, nxt_xk);
    if (z + 1 < z1) fetch_x(z + 2, rown, rhalo);
    if (z + 1 < z1) fetch_out(z + 1, u_nxt, xq_nxt);
  };
  // second half (after a barrier): sc(z+1) into its ring slot (read by the next step) and,
  // for this thread's own voxels, straight into the outputs of plane z, whose y_{k+1} rows
  // replace its gradient rows G; v of plane z+2 is requested after sc(z+1) has used that of
  // plane z+1
  auto step_b = [&](int z, float (*G)[NX]) {
    float sc1[NO];
    compute_sc(z + 1, rv, sc1);
    if (z + 1 < z1) fetch_v(z + 2, rv);
    // ---- outputs of plane z (as k_prox_tv)
    {
      const float(*Ym)[NX] = sY[slot3(z - 1)];
      const float(*Y0)[NX] = sY[slot3(z)];
      const float(*Y1)[NX] = sY[slot3(z + 1)];
      const float(*SC0)[NX] = sSC[z & 1];
      long long pz = (long long)z * plane;
      asm volatile("" : "+s"(pz));
      float* __restrict__ xnh = a.xn_hi + pz;
      uint16_t* __restrict__ xnl = a.xn_lo + pz;
#pragma unroll
      for (int h = 0; h < NO; ++h) {
        const int ly = r + 2 * h;
        const float yc = Y0[ly + 1][x];
        const float sc = SC0[ly][x];
        // p = sc Dy rounded as stored fp32 values, summed in the order z, y, x, -x+, -y+, -z+
        const float pzc = __fmul_rn(sc, yc - Ym[ly + 1][x]);
        const float pyc = __fmul_rn(sc, yc - Y0[ly][x]);
        const float pxc = __fmul_rn(sc, yc - Y0[ly + 1][xm]);
        const float pxn = __fmul_rn(SC0[ly][xp], Y0[ly + 1][xp] - yc);
        const float pyn = __fmul_rn(SC0[ly + 1][x], Y0[ly + 2][x] - yc);
        const float pzn = __fmul_rn(sc1[h], Y1[ly + 1][x] - yc);
        const float gtv = pzc + pyc + pxc - pxn - pyn - pzn;
        const float gd = G[ly][x];
        const float uu = u_cur[h];
        const float xq = xq_cur[h];
        float ynext;
        if constexpr (COMP) {
          const double y = own_y[h];
          const double dprior = y - (double)xq;
          const double zv = y - a.lr * ((double)gd + a.mu * (double)gtv + 2.0 * a.gamma * dprior);
          const double t = a.lr * a.lam * (double)uu;
          const double az = fabs(zv) - t;
          const double xn = az > 0.0 ? copysign(az, zv) : 0.0;
          if constexpr (MON) {
            acc_l1 += (double)uu * fabs(y);
            acc_gam += dprior * dprior;
          }
          const float hi = (float)xn;
          const uint16_t lo = f32_to_bf16((float)(xn - (double)hi));
          st_nt<NT>(xnh, own_off[h] * 4u, hi);
          st_nt<NT>(xnl, own_off[h] * 2u, lo);
          const double xs = (double)hi + (double)bf16_to_f32(lo);
          ynext = (float)(xs + a.m_next * (xs - own_xk[h]));
        } else {
          const float y = (float)own_y[h];
          const float dprior = y - xq;
          const float zv = y - (float)a.lr * (gd + (float)a.mu * gtv + 2.0f * (float)a.gamma * dprior);
          const float t = (float)a.lr * (float)a.lam * uu;
          const float az = fabsf(zv) - t;
          const float xn = az > 0.f ? copysignf(az, zv) : 0.f;
          if constexpr (MON) {
            acc_l1 += (double)uu * fabs((double)y);
            acc_gam += (double)dprior * dprior;
          }
          st_nt<NT>(xnh, own_off[h] * 4u, xn);
          const float xk = (float)own_xk[h];
          ynext = xn + (float)a.m_next * (xn - xk);
        }
        G[ly][x] = ynext;
      }
    }
#pragma unroll
    for (int h = 0; h < NO; ++h) {
      own_y[h] = nxt_y[h];
      own_xk[h] = nxt_xk[h];
      u_cur[h] = u_nxt[h];
      xq_cur[h] = xq_nxt[h];
    }
  };

  for (int i = tid; i < M; i += blockDim.x) {
    s_tw[i] = twm[i];
    s_twn[i] = twn[i];
  }
  float2 sa[FE];
  if constexpr (!PIPE) {
    // ---- prologue: the gradient rows of the first batch; y on planes z0-1, z0; sc(z0);
    // prefetch plane z0+1, the outputs' inputs of plane z0 and the next batch's spectrum
    fetch_spec(z0, sa);
    {
      double d1[NO], d2[NO];
      fetch_x(z0 - 1, rown, rhalo);
      store_plane(z0 - 1, rown, rhalo, d1, d2);
      fetch_x(z0, rown, rhalo);
      fetch_v(z0, rv);
      store_plane(z0, rown, rhalo, own_y, own_xk);
    }
    transform_phase(z0, z0, z0, sa);  // inverse half only; ends with a barrier
    {
      float sc0[NO];
      compute_sc(z0, rv, sc0);
    }
    fetch_x(z0 + 1, rown, rhalo);
    fetch_v(z0 + 1, rv);
    fetch_out(z0, u_cur, xq_cur);
    fetch_spec(z0 + KB, sa);

    for (int zb = z0; zb < z1; zb += KB) {
      const int zb_end = min(zb + KB, z1);
      for (int z = zb; z < zb_end; ++z) {
        step_a(z);
        __syncthreads();
        step_b(z, sG[0][z - zb]);
        __syncthreads();  // sY slot z-1 and the sG rows are rewritten next
      }
      // ---- the batch's y_{k+1} rows into S; the next batch's gradient rows into sG
      transform_phase(zb, zb_end, zb + KB, sa);
      fetch_spec(zb + 2 * KB, sa);
      __syncthreads();  // the exchange rows are rewritten by the next phase
    }
  } else {
    // ---- Pipelined row transforms.  Each row transform runs on the 32 lanes of one
    // half-wave and exchanges data only through its own LDS row, so its steps need no
    // block barrier, only the in-order LDS accesses of one wavefront.  Threads [0, 2 NR FT)
    // (whole waves) transform: rows [0, NR) the y_{k+1} rows of the previous batch forward,
    // rows [NR, 2 NR) the gradient rows of the next batch inverse, in four chunks that ride
    // along with the four barrier intervals of the current batch's two plane steps.  The
    // rows of three batches sit in LDS (slot = batch % 3): the previous one (read by the
    // forward chunks), the current one (stepped) and the next one (written by the inverse).
    // Same arithmetic as transform_phase, step by step.
    const bool ptx = tid < 2 * NR * FT;  // wave-uniform
    const bool pfwd = fr < NR;           // wave-uniform
    const int prow = pfwd ? fr : fr - NR;
    const int mb = M - fq - FT * (FE - 1);  // mirror base, as in transform_phase
    // the three stages of a row transform: at M = 256 the Row256 stages, else the generic
    // register stages with wave-level ordering (same operations as fft_reg)
    auto stage0 = [&](float2(&v)[FE], float* fre, float* fim, bool act) {
      if constexpr (M == 256) Row256::s0(v, fre, fim, fq, act);
      else reg_stage<M, FT, 0, false, true, true>(v, fre, fim, 1, fq, s_tw, act);
    };
    auto stage1 = [&](float2(&v)[FE], float* fre, float* fim, bool act) {
      if constexpr (M == 256) {
        Row256::s1r(v, fre, fim, fq, act);
        wave_sync();
        Row256::s1w(v, fre, fim, fq, s_tw, act);
      } else {
        reg_stage<M, FT, 1, false, true, true>(v, fre, fim, 1, fq, s_tw, act);
      }
    };
    auto stage2 = [&](float2(&v)[FE], float* fre, float* fim, bool act) {
      if constexpr (M == 256) Row256::s2(v, fre, fim, fq, s_tw, act);
      else reg_stage<M, FT, 2, false, true, true>(v, fre, fim, 1, fq, s_tw, act);
    };
    // chunk 1: forward rows of the batch at zf (planes < zf_end) out of slot gf; inverse
    // rows: the spectrum in sa, then Z (as k_c2r_x, conjugated); radix-8 stage 0 of both
    auto chunk1 = [&](int zf, int zf_end, int gf, int zi) {
      if (!ptx) return;
      float* fre = &sFx[fr * 2 * M];
      float* fim = fre + M;
      float2 v[FE];
      bool act;
      if (pfwd) {
        act = zf + prow / TY < zf_end;
        if (act) {
          const float(*G)[NX] = sG[gf][prow / TY];
#pragma unroll
          for (int i = 0; i < FE; ++i) v[i] = *reinterpret_cast<const float2*>(&G[prow % TY][2 * (fq + FT * i)]);
        }
      } else {
        act = zi + prow / TY < z1;
        if (act) {
#pragma unroll
          for (int i = 0; i < FE; ++i) {
            fre[fq + FT * i] = sa[i].x;
            fim[fq + FT * i] = sa[i].y;
          }
        }
        wave_sync();
        if (act) {
#pragma unroll
          for (int i = 0; i < FE; ++i) {
            const float2 xk = sa[i];
            const float2 xmr = make_float2(fre[mb + FT * (FE - 1 - i)], fim[mb + FT * (FE - 1 - i)]);
            const float2 e = make_float2(xk.x + xmr.x, xk.y - xmr.y);
            const float2 d = make_float2(xk.x - xmr.x, xk.y + xmr.y);
            const float2 o = cmulc(d, s_twn[fq + FT * i]);
            float2 zk = make_float2(e.x - o.y, e.y + o.x);
            if (i == 0 && fq == 0) zk = make_float2(xk.x + xk.y, xk.x - xk.y);
            v[i] = make_float2(zk.x, -zk.y);
          }
        }
        wave_sync();
      }
      stage0(v, fre, fim, act);
    };
    auto pact = [&](int zf, int zf_end, int zi) {
      return pfwd ? zf + prow / TY < zf_end : zi + prow / TY < z1;
    };
    // chunk 2: radix-8 stage 1
    auto chunk2 = [&](int zf, int zf_end, int zi) {
      if (!ptx) return;
      const bool act = pact(zf, zf_end, zi);
      float2 v[FE];
      float* fre = &sFx[fr * 2 * M];
      stage1(v, fre, fre + M, act);
    };
    // chunk 3: radix-4 stage 2; inverse rows: real samples into slot gi; forward rows: Z
    // into the row for the mirror reads of chunk 4
    auto chunk3 = [&](int zf, int zf_end, int zi, int gi) {
      if (!ptx) return;
      const bool act = pact(zf, zf_end, zi);
      float* fre = &sFx[fr * 2 * M];
      float* fim = fre + M;
      float2 v[FE];
      stage2(v, fre, fim, act);
      if (!act) return;
      if (pfwd) {
        wave_sync();
#pragma unroll
        for (int i = 0; i < FE; ++i) {
          fre[fq + FT * i] = v[i].x;
          fim[fq + FT * i] = v[i].y;
        }
      } else {  // z = conj(FFT(conj Z)): interleaved real samples of the row
        float(*G)[NX] = sG[gi][prow / TY];
#pragma unroll
        for (int i = 0; i < FE; ++i)
          *reinterpret_cast<float2*>(&G[prow % TY][2 * (fq + FT * i)]) = make_float2(v[i].x, -v[i].y);
      }
    };
    // chunk 4: forward rows: X[k] from Z[k] and Z[M-k] (as k_r2c_x) into the spectrum rows
    auto chunk4 = [&](int zf, int zf_end) {
      if (!ptx || !pfwd || zf + prow / TY >= zf_end) return;
      const float* fre = &sFx[fr * 2 * M];
      const float* fim = fre + M;
      float2* __restrict__ dst = S + ((long long)zf * ny + y0) * M;
      const unsigned ob = row_off(prow);
#pragma unroll
      for (int i = 0; i < FE; ++i) {
        const float2 zk = make_float2(fre[fq + FT * i], fim[fq + FT * i]);
        const float2 zm = make_float2(fre[mb + FT * (FE - 1 - i)], fim[mb + FT * (FE - 1 - i)]);
        const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
        const float2 d = make_float2(0.5f * (zk.x - zm.x), 0.5f * (zk.y + zm.y));
        const float2 o = make_float2(d.y, -d.x);
        float2 out = cadd(e, cmul(s_twn[fq + FT * i], o));
        if (i == 0 && fq == 0) out = make_float2(zk.x + zk.y, zk.x - zk.y);
        st_nt<NT>(dst, ob + (unsigned)(FT * i) * 8u, out);
      }
    };

    // ---- prologue: y on planes z0-1, z0; the first batch's gradient rows into slot 0;
    // sc(z0); prefetch plane z0+1, the outputs' inputs of plane z0 and the spectrum of the
    // second batch
    fetch_spec(z0, sa);
    {
      double d1[NO], d2[NO];
      fetch_x(z0 - 1, rown, rhalo);
      store_plane(z0 - 1, rown, rhalo, d1, d2);
      fetch_x(z0, rown, rhalo);
      fetch_v(z0, rv);
      store_plane(z0, rown, rhalo, own_y, own_xk);
    }
    __syncthreads();  // twiddles and the y rings
    chunk1(z0, z0, 0, z0);
    wave_sync();
    chunk2(z0, z0, z0);
    wave_sync();
    chunk3(z0, z0, z0, 0);
    fetch_spec(z0 + KB, sa);
    {
      float sc0[NO];
      compute_sc(z0, rv, sc0);
    }
    fetch_x(z0 + 1, rown, rhalo);
    fetch_v(z0 + 1, rv);
    fetch_out(z0, u_cur, xq_cur);

    int jb = 0;
    for (int zb = z0; zb < z1; zb += KB, ++jb) {
      const int zb_end = min(zb + KB, z1);
      const int gc = jb % 3, gp = (jb + 2) % 3, gn = (jb + 1) % 3;  // slots: this, previous, next
      // the previous batch (always whole) goes forward; none before the first batch
      const int zf = zb - KB, zf_end = jb > 0 ? zb : zf;
      const int zi = zb + KB;
      step_a(zb);
      chunk1(zf, zf_end, gp, zi);
      fetch_spec(zb + 2 * KB, sa);
      __syncthreads();
      step_b(zb, sG[gc][0]);
      chunk2(zf, zf_end, zi);
      __syncthreads();
      if (zb + 1 < zb_end) step_a(zb + 1);
      chunk3(zf, zf_end, zi, gn);
      __syncthreads();
      if (zb + 1 < zb_end) step_b(zb + 1, sG[gc][1]);
      chunk4(zf, zf_end);
      __syncthreads();  // sY, sSC and the slots are rewritten by the next batch
    }
    // ---- epilogue: the last batch's y_{k+1} rows forward
    {
      const int zl = z0 + KB * (jb - 1);
      chunk1(zl, z1, (jb - 1) % 3, z1);
      wave_sync();
      chunk2(zl, z1, z1);
      wave_sync();
      chunk3(zl, z1, z1, 0);
      wave_sync();
      chunk4(zl, z1);
    }
  }
  if constexpr (MON) {
    __shared__ double s_red[16];
    const int nb = gridDim.x;
    double rr = block_reduce<RED_OP_SUM>(acc_l1, s_red);
    if (tid == 0) a.partials[blockIdx.x] = rr;
    rr = block_reduce<RED_OP_SUM>(acc_hub, s_red);
    if (tid == 0) a.partials[nb + blockIdx.x] = rr;
    rr = block_reduce<RED_OP_SUM>(acc_gam, s_red);
    if (tid == 0) a.partials[2 * nb + blockIdx.x] = rr;
  }
}

// ---------------------------------------------------------------- elementwise kernels

// y = x_k + m (x_k - x_{k-1}) into the map buffer (the first x-axis transform of a round).
template <int ST>
__global__ void k_prime(void* __restrict__ rbuf, const float* __restrict__ xk_hi, const uint16_t* __restrict__ xk_lo,
                        const float* __restrict__ xo_hi, const uint16_t* __restrict__ xo_lo, double m, int read_old,
                        long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    if constexpr (ST == ST_COMP) {
      const double xk = load_x<true>(xk_hi, xk_lo, i);
      double y = xk;
      if (read_old) y = xk + m * (xk - load_x<true>(xo_hi, xo_lo, i));
      st_real<false>(rbuf, i, (float)y);
    } else {
      const float xk = xk_hi[i];
      float y = xk;
      if (read_old) y = xk + (float)m * (xk - xo_hi[i]);
      st_real<ST == ST_BF16>(rbuf, i, y);
    }
  }
}

__global__ void k_f32_to_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = f32_to_bf16(src[i]);
}

__global__ void k_bf16_to_f32(const uint16_t* __restrict__ src, float* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = bf16_to_f32(src[i]);
}

__global__ void k_set_map(const float* __restrict__ x0, float* __restrict__ hi, uint16_t* __restrict__ lo, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    hi[i] = x0 ? x0[i] : 0.0f;
    if (lo) lo[i] = 0;
  }
}

template <bool COMP>
__global__ void k_get_map(const float* __restrict__ hi, const uint16_t* __restrict__ lo, float* __restrict__ out,
                          long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = COMP ? (float)load_x<true>(hi, lo, i) : hi[i];
}

__global__ void k_fill(float* __restrict__ dst, long long n, float value) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = value;
}

// Rows (kz, ky) of a [kz][ky][k] array with rows of len elements, spread over the blocks, and
// the row's elements over a block's threads (several rows per pass where len < blockDim.x):
// f(kz, ky, k) for every element, with no division per element.
struct RowWalk {
  unsigned tpr, rpi, lane, first, step, nrows;
  __device__ RowWalk(int nz, int ny, int len) {
    tpr = (unsigned)len < blockDim.x ? (unsigned)len : blockDim.x;
    rpi = blockDim.x / tpr;
    const unsigned sub = threadIdx.x / tpr;
    lane = threadIdx.x - sub * tpr;
    nrows = sub < rpi ? (unsigned)nz * (unsigned)ny : 0u;  // threads past the last whole row idle
    first = blockIdx.x * rpi + sub;
    step = gridDim.x * rpi;
  }
};
// SPG_ROWS(w, kz, ky, k, nz, ny, len) { body }: the body runs for each element (kz, ky, k) of
// the rows that this thread's block and lane walk (the middle loop only binds kz and ky)
#define SPG_ROWS(W, KZ, KY, K, NZ, NY, LEN)                                                   \
  RowWalk W(NZ, NY, LEN);                                                                     \
  for (unsigned row_ = W.first; row_ < W.nrows; row_ += W.step)                               \
    for (int KZ = (int)(row_ / (unsigned)(NY)), KY = (int)(row_ - (unsigned)KZ * (unsigned)(NY)), \
             K = (int)W.lane, once_ = 1;                                                      \
         once_; once_ = 0)                                                                    \
      for (; K < (LEN); K += (int)W.tpr)
// index of -k on an axis of n points
__device__ __forceinline__ int neg_mod(int k, int n) { return k == 0 ? 0 : n - k; }

// Fold of the data term onto the packed half spectrum (a real map only sees the
// Hermitian part of w (A x - b)):  w~ = (w_k + w_{-k})/2,  c = (w_k b_k + w_{-k} conj b_{-k})/2,
// stored scaled for unnormalised transforms: ws = w~ / nvox, cs = c / sqrt(nvox).
// Partial: max w~.

__global__ void __launch_bounds__(256) k_fold(Dims d, const float* __restrict__ w, const float2* __restrict__ b,
                                              float* __restrict__ ws, float* __restrict__ w0p,
                                              float* __restrict__ wnyq, float2* __restrict__ cs,
                                              float2* __restrict__ c0p, float2* __restrict__ cnyq,
                                              double* __restrict__ partials) {
  __shared__ double s_red[8];
  const int P = d.P;
  const double inv_n = 1.0 / (double)d.nvox;
  const double inv_sqrt_n = 1.0 / sqrt((double)d.nvox);
  // one element of the folded half spectrum; returns w~ (unscaled) for the maximum
  auto fold = [=](int kz, int ky, int kx) -> double {
    const int nkx = neg_mod(kx, d.nx), nky = neg_mod(ky, d.ny), nkz = neg_mod(kz, d.nz);
    const long long ik = ((long long)kz * d.ny + ky) * d.nx + kx;
    const long long in = ((long long)nkz * d.ny + nky) * d.nx + nkx;
    const double wk = w[ik], wn = w[in];
    const float2 bk = b[ik], bn = b[in];
    const double wt = 0.5 * (wk + wn);
    const double cr = 0.5 * (wk * bk.x + wn * bn.x);
    const double ci = 0.5 * (wk * bk.y - wn * bn.y);
    const float wsv = (float)(wt * inv_n);
    const float2 csv = make_float2((float)(cr * inv_sqrt_n), (float)(ci * inv_sqrt_n));
    const long long op = (long long)ky * d.nz + kz;  // [ky][kz] planes of kx = 0 and nx/2
    if (kx < P) {
      const long long o = wc_index(d, kz, ky, kx);
      ws[o] = wsv;
      cs[o] = csv;
      if (kx == 0) {
        w0p[op] = wsv;
        c0p[op] = csv;
      }
    } else {
      wnyq[op] = wsv;
      cnyq[op] = csv;
    }
    return wt;
  };
  double mx = 0.0;
  // columns kx < P row by row, then the column kx = P (= nx/2) one row per thread
  SPG_ROWS(rw, kz, ky, kx, d.nz, d.ny, P) {
    const double wt = fold(kz, ky, kx);
    mx = wt > mx ? wt : mx;
  }
  const unsigned nrows = (unsigned)d.nz * (unsigned)d.ny;
  for (unsigned row = blockIdx.x * blockDim.x + threadIdx.x; row < nrows; row += gridDim.x * blockDim.x) {
    const int kz = (int)(row / (unsigned)d.ny), ky = (int)(row - (unsigned)kz * (unsigned)d.ny);
    const double wt = fold(kz, ky, P);
    mx = wt > mx ? wt : mx;
  }
  const double r = block_reduce<RED_OP_MAX>(mx, s_red);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// Input checks and constants over the full arrays (FFT order, [kz][ky][kx]): count of
// non-finite w or b values, min w, 1/2 sum w |b|^2 (the constant of the data term), sum w,
// and sum |h(k)|^2 with h(k) = (b'(k) + conj b'(-k)) / 2, b' = b [w > 0]: by Parseval the
// energy of Re F^H b' (unitary F), the unregularised solution whose scale guides the choice
// of lambda and mu.
__global__ void __launch_bounds__(256) k_data_stats(Dims d, const float* __restrict__ w,
                                                    const float2* __restrict__ b, double* __restrict__ partials) {
  __shared__ double s_red[8];
  double bad = 0.0, mn = 1e300, c0 = 0.0, sw = 0.0, eh = 0.0;
  SPG_ROWS(rw, kz, ky, kx, d.nz, d.ny, d.nx) {
    const long long i = ((long long)kz * d.ny + ky) * d.nx + kx;
    const float wv = w[i];
    const float2 bv = b[i];
    const bool fin = isfinite(wv) && isfinite(bv.x) && isfinite(bv.y);
    if (!fin) bad += 1.0;
    else {
      mn = wv < mn ? wv : mn;
      c0 += 0.5 * (double)wv * ((double)bv.x * bv.x + (double)bv.y * bv.y);
      sw += (double)wv;
      const long long j = ((long long)neg_mod(kz, d.nz) * d.ny + neg_mod(ky, d.ny)) * d.nx + neg_mod(kx, d.nx);
      const float wm = w[j];
      const float2 bm = b[j];
      const double px = wv > 0.f ? (double)bv.x : 0.0, py = wv > 0.f ? (double)bv.y : 0.0;
      const bool mok = wm > 0.f && isfinite(bm.x) && isfinite(bm.y);
      const double qx = mok ? (double)bm.x : 0.0, qy = mok ? (double)bm.y : 0.0;
      const double hx = 0.5 * (px + qx), hy = 0.5 * (py - qy);
      eh += hx * hx + hy * hy;
    }
  }
  const int nb = gridDim.x;
  double r = block_reduce<RED_OP_SUM>(bad, s_red);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
  r = block_reduce<RED_OP_MIN>(mn, s_red);
  if (threadIdx.x == 0) partials[nb + blockIdx.x] = r;
  r = block_reduce<RED_OP_SUM>(c0, s_red);
  if (threadIdx.x == 0) partials[2 * nb + blockIdx.x] = r;
  r = block_reduce<RED_OP_SUM>(sw, s_red);
  if (threadIdx.x == 0) partials[3 * nb + blockIdx.x] = r;
  r = block_reduce<RED_OP_SUM>(eh, s_red);
  if (threadIdx.x == 0) partials[4 * nb + blockIdx.x] = r;
}

// Penalty-weight checks: count of non-finite values, min and max.
__global__ void __launch_bounds__(256) k_weight_stats(long long n, const float* __restrict__ a,
                                                      double* __restrict__ partials) {
  __shared__ double s_red[8];
  double bad = 0.0, mn = 1e300, mx = -1e300;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float v = a[i];
    if (!isfinite(v)) bad += 1.0;
    else {
      mn = v < mn ? v : mn;
      mx = v > mx ? v : mx;
    }
  }
  const int nb = gridDim.x;
  double r = block_reduce<RED_OP_SUM>(bad, s_red);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
  r = block_reduce<RED_OP_MIN>(mn, s_red);
  if (threadIdx.x == 0) partials[nb + blockIdx.x] = r;
  r = block_reduce<RED_OP_MAX>(mx, s_red);
  if (threadIdx.x == 0) partials[2 * nb + blockIdx.x] = r;
}

// Reweighting of eq 11 from the current map: u = 1/(|x| + eps1), v = 1/(|Dx| + eps2),
// with |Dx| the periodic backward-difference gradient norm of eq 12.  Partial: max v.
// LOGS: no weights written; partials sum log(|x| + eps1) and sum log(|Dx| + eps2), the
// penalty terms of the log objective of eq 10 that the reweighting majorises.
template <bool COMP, bool BF, bool LOGS = false>
__global__ void __launch_bounds__(256) k_reweight(Dims d, const float* __restrict__ hi, const uint16_t* __restrict__ lo,
                                                  void* __restrict__ u, void* __restrict__ v, double eps1,
                                                  double eps2, double* __restrict__ partials) {
  __shared__ double s_red[8];
  double mx = 0.0, l1 = 0.0, l2 = 0.0;
  const long long plane = (long long)d.nx * d.ny;
  SPG_ROWS(rw, z, y, x, d.nz, d.ny, d.nx) {
    const long long i = ((long long)z * d.ny + y) * d.nx + x;
    const long long ixm = i - x + (x == 0 ? d.nx - 1 : x - 1);
    const long long iym = i + (long long)((y == 0 ? d.ny - 1 : y - 1) - y) * d.nx;
    const long long izm = i + (long long)((z == 0 ? d.nz - 1 : z - 1) - z) * plane;
    const double xc = load_x<COMP>(hi, lo, i);
    const double ddx = xc - load_x<COMP>(hi, lo, ixm);
    const double ddy = xc - load_x<COMP>(hi, lo, iym);
    const double ddz = xc - load_x<COMP>(hi, lo, izm);
    const double nrm = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
    if constexpr (LOGS) {
      l1 += log(fabs(xc) + eps1);
      l2 += log(nrm + eps2);
    } else {
      st_real<BF>(u, i, (float)(1.0 / (fabs(xc) + eps1)));
      const float vf = (float)(1.0 / (nrm + eps2));
      const float vv = BF ? bf16_to_f32(f32_to_bf16(vf)) : vf;  // max of the stored values
      st_real<BF>(v, i, vf);
      mx = (double)vv > mx ? (double)vv : mx;
    }
  }
  if constexpr (LOGS) {
    double r = block_reduce<RED_OP_SUM>(l1, s_red);
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
    r = block_reduce<RED_OP_SUM>(l2, s_red);
    if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = r;
  } else {
    const double r = block_reduce<RED_OP_MAX>(mx, s_red);
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
  }
}

// ---------------------------------------------------------------- Fourier shell correlation
// Shell sums of eq 30 over the packed half spectra of two real maps: Re F conj G, |F|^2,
// |G|^2 per shell, with multiplicity 2 for 0 < kx < nx/2.  The packed slot 0 is split
// into its kx = 0 and kx = nx/2 planes with the partner at (-ky, -kz).  Shell of signed
// frequency k: floor(min(n) sqrt(sum_a (k_a / n_a)^2) + 1/2).  Deterministic: every wave
// keeps its own histogram in LDS; the lanes' terms of one shell are summed by a fixed
// butterfly over the wave and added by lane 0, so no two adds to one LDS word race; the
// block partial sums the wave histograms in wave order, and k_fsc_final the blocks in
// block order.
__device__ __forceinline__ int fsc_shell(int kz, int ky, int kx, const Dims& d) {
  const int nmin = min(d.nx, min(d.ny, d.nz));
  const int sz = kz < d.nz / 2 ? kz : kz - d.nz;
  const int sy = ky < d.ny / 2 ? ky : ky - d.ny;
  const int sx = kx < d.nx / 2 ? kx : kx - d.nx;
  const double fz = (double)sz * nmin / d.nz, fy = (double)sy * nmin / d.ny, fx = (double)sx * nmin / d.nx;
  return (int)floor(sqrt(fz * fz + fy * fy + fx * fx) + 0.5);
}

constexpr int FSC_THREADS = 128;  // two waves per block: 2 x 3 x 1024 fp64 histogram words at most

__global__ void __launch_bounds__(FSC_THREADS) k_fsc_shells(Dims d, const float2* __restrict__ S1,
                                                            const float2* __restrict__ S2, int nshells,
                                                            double* __restrict__ partials) {
  extern __shared__ double sh[];  // per wave: 3 * nshells
  constexpr int NW = FSC_THREADS / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double* hw = sh + (size_t)wave * 3 * nshells;
  for (int i = threadIdx.x; i < NW * 3 * nshells; i += blockDim.x) sh[i] = 0.0;
  __syncthreads();
  // all 64 lanes call this together; a lane with shell < 0 contributes nothing
  auto wave_add = [&](int shell, double a, double b, double c) {
    int mine = shell < nshells ? shell : -1;
    for (;;) {
      const unsigned long long pend = __ballot(mine >= 0);
      if (pend == 0ull) break;
      const int s = __shfl(mine, __ffsll((long long)pend) - 1);
      const bool take = mine == s;
      double x = take ? a : 0.0, y = take ? b : 0.0, z = take ? c : 0.0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_xor(x, off);
        y += __shfl_xor(y, off);
        z += __shfl_xor(z, off);
      }
      if (lane == 0) {
        hw[s] += x;
        hw[nshells + s] += y;
        hw[2 * nshells + s] += z;
      }
      if (take) mine = -1;
    }
  };
  const int P = d.P;
  const long long nh = (long long)d.nz * d.ny * P;
  const long long stride = (long long)gridDim.x * blockDim.x;
  // block-uniform trip count: lanes past the end take part with no terms
  for (long long t0 = (long long)blockIdx.x * blockDim.x; t0 < nh; t0 += stride) {
    const long long t = t0 + threadIdx.x;
    int s1 = -1, s2 = -1;
    double a1 = 0.0, b1 = 0.0, c1 = 0.0, a2 = 0.0, b2 = 0.0, c2 = 0.0;
    if (t < nh) {
      const int kx = (int)(t % P);
      const long long r = t / P;
      const int ky = (int)(r % d.ny);
      const int kz = (int)(r / d.ny);
      const float2 f = S1[t], g = S2[t];
      auto terms = [](double w, float2 f_, float2 g_, double& a, double& b, double& c) {
        a = w * ((double)f_.x * g_.x + (double)f_.y * g_.y);
        b = w * ((double)f_.x * f_.x + (double)f_.y * f_.y);
        c = w * ((double)g_.x * g_.x + (double)g_.y * g_.y);
      };
      if (kx > 0) {
        s1 = fsc_shell(kz, ky, kx, d);
        terms(2.0, f, g, a1, b1, c1);
      } else {
        const long long tp = ((long long)((d.nz - kz) % d.nz) * d.ny + ((d.ny - ky) % d.ny)) * P;
        const float2 fp = S1[tp], gp = S2[tp];
        const float2 f0 = make_float2(0.5f * (f.x + fp.x), 0.5f * (f.y - fp.y));
        const float2 fn = make_float2(0.5f * (f.y + fp.y), -0.5f * (f.x - fp.x));
        const float2 g0 = make_float2(0.5f * (g.x + gp.x), 0.5f * (g.y - gp.y));
        const float2 gn = make_float2(0.5f * (g.y + gp.y), -0.5f * (g.x - gp.x));
        s1 = fsc_shell(kz, ky, 0, d);
        terms(1.0, f0, g0, a1, b1, c1);
        s2 = fsc_shell(kz, ky, d.nx / 2, d);
        terms(1.0, fn, gn, a2, b2, c2);
      }
    }
    wave_add(s1, a1, b1, c1);
    wave_add(s2, a2, b2, c2);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * nshells; i += blockDim.x) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) v += sh[(size_t)w * 3 * nshells + i];
    partials[(long long)blockIdx.x * 3 * nshells + i] = v;
  }
}

// Fixed-order sum of the block histograms: out[q * nshells + s], q = 0..2.
__global__ void k_fsc_final(const double* __restrict__ partials, int nblocks, int nshells, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * nshells) return;
  double acc = 0.0;
  for (int b = 0; b < nblocks; ++b) acc += partials[(long long)b * 3 * nshells + i];
  out[i] = acc;
}

// ---------------------------------------------------------------- adjoint of unrolled SPG
// Reverse step k of x_{k+1} = soft(z_k, lr lam u), z_k = y_k - lr (g_data(y_k) + mu g_tv(y_k)),
// y_k = x_k + m_k (x_k - x_{k-1}) (chain rule; a.e. derivatives at the kinks).

// zbar = [x_{k+1} != 0] abar_{k+1};  rbar += lr zbar;  partials: sum tbar u with
// tbar = -sign(x_{k+1}) zbar (threshold adjoint), and sum zbar g_data(y_k).
__global__ void __launch_bounds__(256) k_adj_prox(long long n, const float* __restrict__ xn,
                                                  const float* __restrict__ abar, const float* __restrict__ gdat,
                                                  const float* __restrict__ u, float lr, float* __restrict__ zbar,
                                                  float* __restrict__ rbar, double* __restrict__ partials) {
  __shared__ double s_red[8];
  double s_t = 0.0, s_g = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float x = xn[i];
    const float zb = x != 0.f ? abar[i] : 0.f;
    zbar[i] = zb;
    rbar[i] += lr * zb;
    const float uu = u ? u[i] : 1.0f;
    s_t += -(double)copysignf(1.0f, x) * (x != 0.f ? (double)zb : 0.0) * uu;
    s_g += (double)zb * gdat[i];
  }
  const int nb = gridDim.x;
  double r = block_reduce<RED_OP_SUM>(s_t, s_red);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
  r = block_reduce<RED_OP_SUM>(s_g, s_red);
  if (threadIdx.x == 0) partials[nb + blockIdx.x] = r;
}

// Weighted dual and its Hessian product at one point j from the three backward differences
// d = (Dy)_j, e = (D zbar)_j:  p = v d / max(eps, |d|),  q = v J(d) e,
// J = I / eps for |d| < eps, (I - d d^T / |d|^2) / |d| otherwise.
__device__ __forceinline__ void adj_dual(const float d[3], const float e[3], float vv, float eps, float p[3],
                                         float q[3]) {
  const float n2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const float n = sqrtf(n2);
  if (n < eps) {
    const float s = vv / eps;
    for (int a = 0; a < 3; ++a) {
      p[a] = s * d[a];
      q[a] = s * e[a];
    }
  } else {
    const float de = d[0] * e[0] + d[1] * e[1] + d[2] * e[2];
    const float s = vv / n;
    for (int a = 0; a < 3; ++a) {
      p[a] = s * d[a];
      q[a] = s * (e[a] - d[a] * de / n2);
    }
  }
}

// ybar = zbar - lr (hz + mu H_tv(y_k) zbar); abar_k += (1 + m) ybar; abar_{k-1} = -m ybar
// (first contribution); partial: sum zbar g_tv(y_k).  y_k from the stored fp32 maps.
// One thread per voxel, neighbours read through the cache (the reverse pass is not the
// hot path).
__global__ void __launch_bounds__(256) k_adj_tv(Dims dm, const float* __restrict__ xk, const float* __restrict__ xkm,
                                                float m, const float* __restrict__ zbar, const float* __restrict__ hz,
                                                const float* __restrict__ v, float lr, float mu, float eps,
                                                float* __restrict__ abar_k, float* __restrict__ abar_km,
                                                double* __restrict__ partials) {
  __shared__ double s_red[8];
  const int nx = dm.nx, ny = dm.ny, nz = dm.nz;
  const long long plane = (long long)nx * ny;
  auto wr = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
  auto idx = [&](int z, int y, int x) { return (long long)wr(z, nz) * plane + (long long)wr(y, ny) * nx + wr(x, nx); };
  auto Y = [&](long long i) { return xk[i] + m * (xk[i] - xkm[i]); };
  auto point = [&](int z, int y, int x, float p[3], float q[3]) {
    const long long i = idx(z, y, x);
    const long long iz = idx(z - 1, y, x), iy = idx(z, y - 1, x), ix = idx(z, y, x - 1);
    const float yc = Y(i), zc = zbar[i];
    const float d[3] = {yc - Y(iz), yc - Y(iy), yc - Y(ix)};
    const float e[3] = {zc - zbar[iz], zc - zbar[iy], zc - zbar[ix]};
    adj_dual(d, e, v ? v[i] : 1.0f, eps, p, q);
  };
  double s_tv = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < dm.nvox;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / plane);
    float p0[3], q0[3], pz[3], qz[3], py[3], qy[3], px[3], qx[3];
    point(z, y, x, p0, q0);
    point(z + 1, y, x, pz, qz);
    point(z, y + 1, x, py, qy);
    point(z, y, x + 1, px, qx);
    const float gtv = (p0[0] - pz[0]) + (p0[1] - py[1]) + (p0[2] - px[2]);
    const float htv = (q0[0] - qz[0]) + (q0[1] - qy[1]) + (q0[2] - qx[2]);
    const float zb = zbar[i];
    s_tv += (double)zb * gtv;
    const float yb = zb - lr * (hz[i] + mu * htv);
    abar_k[i] += (1.0f + m) * yb;
    if (abar_km) abar_km[i] = -m * yb;
  }
  double r = block_reduce<RED_OP_SUM>(s_tv, s_red);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

// Full complex b-bar = w * A(rbar) / (unitary A) from the packed half spectrum of rbar
// (after the x, y, z forward passes), interleaved re/im, FFT order.
__global__ void __launch_bounds__(256) k_expand_bbar(Dims d, const float2* __restrict__ S, const float* __restrict__ w,
                                                     float2* __restrict__ out) {
  const int P = d.P;
  const float sc = (float)(1.0 / sqrt((double)d.nvox));
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < d.nvox;
       i += (long long)gridDim.x * blockDim.x) {
    const int kx = (int)(i % d.nx);
    const int ky = (int)((i / d.nx) % d.ny);
    const int kz = (int)(i / ((long long)d.nx * d.ny));
    const int nky = (d.ny - ky) % d.ny, nkz = (d.nz - kz) % d.nz;
    float2 val;
    if (kx == 0 || kx == P) {
      const float2 z1 = S[((long long)kz * d.ny + ky) * P];
      const float2 z2 = S[((long long)nkz * d.ny + nky) * P];
      val = kx == 0 ? make_float2(0.5f * (z1.x + z2.x), 0.5f * (z1.y - z2.y))
                    : make_float2(0.5f * (z1.y + z2.y), -0.5f * (z1.x - z2.x));
    } else if (kx < P) {
      val = S[((long long)kz * d.ny + ky) * P + kx];
    } else {
      const float2 t = S[((long long)nkz * d.ny + nky) * P + (d.nx - kx)];
      val = make_float2(t.x, -t.y);
    }
    const float ww = w[i] * sc;
    out[i] = make_float2(ww * val.x, ww * val.y);
  }
}

// ---------------------------------------------------------------- backprojection (eq 24-29)
// The three sums (Re num, Im num, N) are accumulated as int64 fixed-point numbers, whose
// atomic additions give the same bits in any order: every term is rounded to a multiple of
// 2^-s_c, with s_c chosen so that B_c 2^s_c < 2^62 for a bound B_c on the component's sum
// of magnitudes at any grid point.  B_c is 27 times the number of pixels times the largest
// term magnitude (|p ctf Re X|, |p ctf Im X| or p ctf^2; K <= 1), so no partial sum leaves
// the int64 range.  The maxima are exact whatever
// the order of their atomics.

// The largest |p ctf Re X|, |p ctf Im X| and p ctf^2 over all pixels, kept as the bit
// patterns of non-negative doubles (which order like their values) in mx[0..3).
__global__ void __launch_bounds__(256) k_bp_max(int n_img, int m, const float2* __restrict__ images,
                                                const float* __restrict__ ctf, const float* __restrict__ weights,
                                                unsigned long long* __restrict__ mx) {
  __shared__ double s_red[4];
  const long long npix = (long long)m * m;
  const long long total = npix * n_img;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const float2 X = images[t];
    const double cf = ctf ? (double)ctf[t] : 1.0;
    const double p = weights ? (double)weights[t / npix] : 1.0;
    a0 = fmax(a0, fabs(p * cf * X.x));
    a1 = fmax(a1, fabs(p * cf * X.y));
    a2 = fmax(a2, fabs(p * cf * cf));
  }
  a0 = block_reduce<RED_OP_MAX>(a0, s_red);
  a1 = block_reduce<RED_OP_MAX>(a1, s_red);
  a2 = block_reduce<RED_OP_MAX>(a2, s_red);
  if (threadIdx.x == 0) {
    atomicMax(&mx[0], (unsigned long long)__double_as_longlong(a0));
    atomicMax(&mx[1], (unsigned long long)__double_as_longlong(a1));
    atomicMax(&mx[2], (unsigned long long)__double_as_longlong(a2));
  }
}

// 2^s for the component whose largest term magnitude has the bits `mx`: the power of two
// that puts the bound just below 2^62.  The bound is 27 terms per pixel at most (on axes
// shorter than 3 points the 27 neighbours of a coefficient wrap onto fewer grid points).
__device__ __forceinline__ double bp_scale(unsigned long long mx, long long total) {
  const double bound = __longlong_as_double((long long)mx) * (double)total * 27.0;
  if (!(bound > 0.0) || !(bound < 1e300)) return 1.0;
  int e = 0;
  frexp(bound, &e);  // bound < 2^e
  return ldexp(1.0, 62 - e);
}

// One thread per (image, pixel): the coefficient X at signed frequency (u, v) lands at
// c = R (u, v, 0)^T (eq 24) and is spread over the 3^3 grid points round(c) + delta with
// K = exp(-|c - n|^2 / h), accumulating num += p K ctf X and N += p K ctf^2 (eq 28) as
// fixed-point terms.  The coordinate products are rounded separately (no fused
// multiply-add) so that the rounding of c, which decides the neighbourhood, is the
// reference's.
__global__ void __launch_bounds__(256) k_backproject(Dims d, int n_img, int m, const float2* __restrict__ images,
                                                     const double* __restrict__ rots, const float* __restrict__ ctf,
                                                     const float* __restrict__ weights, double h,
                                                     unsigned long long* __restrict__ acc,
                                                     const unsigned long long* __restrict__ mx) {
  const long long npix = (long long)m * m;
  const long long total = npix * n_img;
  const double s0 = bp_scale(mx[0], total), s1 = bp_scale(mx[1], total), s2 = bp_scale(mx[2], total);
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < total; t += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(t / npix);
    const int pix = (int)(t - (long long)i * npix);
    const int vi = pix / m, ui = pix - vi * m;
    const double u = ui < (m + 1) / 2 ? ui : ui - m;
    const double v = vi < (m + 1) / 2 ? vi : vi - m;
    const double* R = rots + 9LL * i;
    double c[3];
    long long base[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c[a] = __dadd_rn(__dmul_rn(R[3 * a + 0], u), __dmul_rn(R[3 * a + 1], v));
      base[a] = (long long)floor(__dadd_rn(c[a], 0.5));
    }
    const float2 X = images[t];
    const double cf = ctf ? (double)ctf[t] : 1.0;
    const double p = weights ? (double)weights[i] : 1.0;
    const double wr = p * cf * X.x * s0, wi = p * cf * X.y * s1, ww = p * cf * cf * s2;
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const long long gx = base[0] + dx, gy = base[1] + dy, gz = base[2] + dz;
          const double ex = c[0] - (double)gx, ey = c[1] - (double)gy, ez = c[2] - (double)gz;
          const double K = exp(-(ex * ex + ey * ey + ez * ez) / h);
          const long long ix = ((gx % d.nx) + d.nx) % d.nx, iy = ((gy % d.ny) + d.ny) % d.ny,
                          iz = ((gz % d.nz) + d.nz) % d.nz;
          const long long idx = (iz * d.ny + iy) * d.nx + ix;
          atomicAdd(&acc[idx], (unsigned long long)__double2ll_rn(K * wr));
          atomicAdd(&acc[d.nvox + idx], (unsigned long long)__double2ll_rn(K * wi));
          atomicAdd(&acc[2 * d.nvox + idx], (unsigned long long)__double2ll_rn(K * ww));
        }
  }
}

// w = N, b = num / N (0 where N = 0), the fixed-point sums scaled back by their exact
// powers of two.
__global__ void k_backproject_final(long long n, long long total, const unsigned long long* __restrict__ acc,
                                    const unsigned long long* __restrict__ mx, float* __restrict__ w,
                                    float2* __restrict__ b) {
  const double r0 = 1.0 / bp_scale(mx[0], total), r1 = 1.0 / bp_scale(mx[1], total),
               r2 = 1.0 / bp_scale(mx[2], total);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double den = (double)(long long)acc[2 * n + i] * r2;
    const double nr = (double)(long long)acc[i] * r0, ni = (double)(long long)acc[n + i] * r1;
    w[i] = (float)den;
    b[i] = den > 0 ? make_float2((float)(nr / den), (float)(ni / den)) : make_float2(0.f, 0.f);
  }
}

__global__ void k_fill_f64(double* __restrict__ dst, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = 0.0;
}

struct RedOps {
  int op[8];
};

// Fixed-order reduction of nq groups of n partials (group q at partials[q*n .. q*n+n)).
__global__ void __launch_bounds__(256) k_reduce(const double* __restrict__ partials, int n, int nq, RedOps ops,
                                                double* __restrict__ out) {
  __shared__ double s_red[8];
  for (int qd = 0; qd < nq; ++qd) {
    const int op = ops.op[qd];
    double acc = op == RED_OP_SUM ? 0.0 : (op == RED_OP_MAX ? -1e300 : 1e300);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double v = partials[(long long)qd * n + i];
      acc = op == RED_OP_SUM ? acc + v : (op == RED_OP_MAX ? (v > acc ? v : acc) : (v < acc ? v : acc));
    }
    double r;
    if (op == RED_OP_SUM) r = block_reduce<RED_OP_SUM>(acc, s_red);
    else if (op == RED_OP_MAX) r = block_reduce<RED_OP_MAX>(acc, s_red);
    else r = block_reduce<RED_OP_MIN>(acc, s_red);
    if (threadIdx.x == 0) out[qd] = r;
    __syncthreads();
  }
}

// The monitored objective F_eps(y_k) (eq 31 with eq 14) from fixed-order sums of the
// partials: C0 + data partials of the z pass (pa) and of the kx = 0 / nx/2 plane (pb), plus
// lam sum u|y| + mu sum v phi_eps + gamma sum (y - x_prev)^2 from the stencil kernel (pc:
// three groups of nc).  One block; writes *out.
__global__ void __launch_bounds__(256) k_obj_finish(const double* __restrict__ pa, int na,
                                                    const double* __restrict__ pb, int nb,
                                                    const double* __restrict__ pc, int nc, double c0, double lam,
                                                    double mu, double gamma, double* __restrict__ out) {
  __shared__ double s_red[8];
  auto sum = [&](const double* p, int n) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += p[i];
    return block_reduce<RED_OP_SUM>(acc, s_red);
  };
  const double A = sum(pa, na);
  const double B = sum(pb, nb);
  const double L1 = sum(pc, nc);
  const double H = sum(pc + nc, nc);
  const double G = sum(pc + 2 * (long long)nc, nc);
  if (threadIdx.x == 0) *out = c0 + A + B + lam * L1 + mu * H + gamma * G;
}

// ---------------------------------------------------------------- launchers

#define SPG_DISPATCH_L(Lv, CALL)        \
  switch (Lv) {                         \
    case 2: { constexpr int L_ = 2; CALL; break; }     \
    case 4: { constexpr int L_ = 4; CALL; break; }     \
    case 8: { constexpr int L_ = 8; CALL; break; }     \
    case 16: { constexpr int L_ = 16; CALL; break; }   \
    case 32: { constexpr int L_ = 32; CALL; break; }   \
    case 64: { constexpr int L_ = 64; CALL; break; }   \
    case 128: { constexpr int L_ = 128; CALL; break; } \
    case 256: { constexpr int L_ = 256; CALL; break; } \
    case 512: { constexpr int L_ = 512; CALL; break; } \
    case 80: { constexpr int L_ = 80; CALL; break; }   \
    case 96: { constexpr int L_ = 96; CALL; break; }   \
    case 160: { constexpr int L_ = 160; CALL; break; } \
    case 192: { constexpr int L_ = 192; CALL; break; } \
    default: return hipErrorInvalidValue;              \
  }

static int tpt(int L) {
  int t = 0;
  switch (L) {
    case 2: t = FftPlan<2>::T; break;
    case 4: t = FftPlan<4>::T; break;
    case 8: t = FftPlan<8>::T; break;
    case 16: t = FftPlan<16>::T; break;
    case 32: t = FftPlan<32>::T; break;
    case 64: t = FftPlan<64>::T; break;
    case 128: t = FftPlan<128>::T; break;
    case 256: t = FftPlan<256>::T; break;
    case 512: t = FftPlan<512>::T; break;
    case 80: t = FftPlan<80>::T; break;
    case 96: t = FftPlan<96>::T; break;
    case 160: t = FftPlan<160>::T; break;
    case 192: t = FftPlan<192>::T; break;
    default: t = 0;
  }
  return t;
}

static int cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      n < 1)
    return 256;
  return n;
}

// Fused z passes: one persistent block per resident slot (CUs x blocks per CU), rounded
// down to a multiple of the 8 XCDs, or one block per tile when there are fewer tiles or
// when persist is false (problems sharing the GPU with others).
template <int L, int MODE, bool NTW>
static hipError_t launch_zw(float2* S, int P, int ntiles, int total, long long pstride, long long bstride,
                            const float2* tw, const float* ws, const float2* cs, double* partials, int NT, int T,
                            bool persist, hipStream_t st, int* nblocks_out, int Pw, int kxo) {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_fft_zw<L, MODE, NTW>, NT * T, 0) != hipSuccess || occ < 1)
    occ = 1;
  long long g = (long long)cu_count() * occ;
  if (g > 4096) g = 4096;  // the objective partials of mode 3 hold one value per block
  if (g >= total || (!persist && MODE != 3)) g = total;
  else if (g >= 8) g &= ~7LL;
  if (nblocks_out) *nblocks_out = (int)g;
  k_fft_zw<L, MODE, NTW><<<dim3((unsigned)g), dim3(NT * T), 0, st>>>(S, P, ntiles, total, pstride, bstride, tw, ws, cs,
                                                               partials, NT, Pw, kxo);
  return hipGetLastError();
}

hipError_t launch_fft_cols(const Dims& d, float2* S, int axis, int mode, const float2* tw, const float* ws,
                           const float2* cs, double* partials, hipStream_t st, int* nblocks_out, int nt,
                           bool persist, int kx0, int nkx) {
  const int L = axis == 1 ? d.ny : d.nz;
  if (nt != 8 && nt != 16) return hipErrorInvalidValue;
  if (mode < 0 || mode > 4 || (mode >= 2 && axis != 2)) return hipErrorInvalidValue;
  if (nkx == 0) nkx = d.P - kx0;
  if (kx0 < 0 || nkx < 1 || kx0 + nkx > d.P || (kx0 > 0 && mode == 3)) return hipErrorInvalidValue;
  // the columns [kx0, kx0 + nkx): tiles over that range, strides of the full spectrum
  S += kx0;
  const int Pc = nkx;
  const int NT = Pc < nt ? Pc : nt;
  const int ntiles = (Pc + NT - 1) / NT;
  const int nbatch = axis == 1 ? d.nz : d.ny;
  const long long pstride = axis == 1 ? (long long)d.P : (long long)d.ny * d.P;
  const long long bstride = axis == 1 ? (long long)d.ny * d.P : (long long)d.P;
  int T = 0;
  SPG_DISPATCH_L(L, (T = ColT<L_>::T));
  const int total = ntiles * nbatch;
  if (mode < 2) {
    const dim3 grid(total), block(NT * T);
    if (nblocks_out) *nblocks_out = total;
    if (mode == 0) {
      SPG_DISPATCH_L(L, (k_fft_cols<L_, 0><<<grid, block, 0, st>>>(S, Pc, ntiles, pstride, bstride, tw, NT)));
    } else {
      SPG_DISPATCH_L(L, (k_fft_cols<L_, 1><<<grid, block, 0, st>>>(S, Pc, ntiles, pstride, bstride, tw, NT)));
    }
    return hipGetLastError();
  }
  // streaming weight loads where the folded weight and data term (6 bytes per voxel)
  // outgrow the 256 MiB last-level cache (measured at 512^3: 400 -> 391 us)
  const bool ntw = (double)d.nvox * 6.0 >= 256.0 * 1024 * 1024;
#define SPG_ZW(MODE_) \
  return launch_zw<L_, MODE_, false>(S, Pc, ntiles, total, pstride, bstride, tw, ws, cs, partials, NT, T, persist, \
                                     st, nblocks_out, d.P, kx0)
#define SPG_ZWN(MODE_) \
  return launch_zw<L_, MODE_, true>(S, Pc, ntiles, total, pstride, bstride, tw, ws, cs, partials, NT, T, persist, \
                                    st, nblocks_out, d.P, kx0)
  switch (mode) {
    case 2:
      if (ntw) {
        SPG_DISPATCH_L(L, SPG_ZWN(2));
      } else {
        SPG_DISPATCH_L(L, SPG_ZW(2));
      }
      break;
    case 3: SPG_DISPATCH_L(L, SPG_ZW(3)); break;
    case 4: SPG_DISPATCH_L(L, SPG_ZW(4)); break;
  }
#undef SPG_ZW
#undef SPG_ZWN
  return hipErrorInvalidValue;
}

bool yz_plane_supported(const Dims& d) {
  auto ok = [](int n) { return n == 8 || n == 16 || n == 32 || n == 64; };
  return ok(d.ny) && ok(d.nz);
}

hipError_t launch_yz_plane(const Dims& d, float2* S, const float2* tw_y, const float2* tw_z, const float* ws,
                           const float2* cs, const float* w0p, const float* wnyq, const float2* c0p,
                           const float2* cnyq, hipStream_t st) {
  if (!yz_plane_supported(d)) return hipErrorInvalidValue;
#define SPG_YZ(NY_, NZ_)                                                                                      \
  if (d.ny == NY_ && d.nz == NZ_) {                                                                         \
    k_yz_plane<NY_, NZ_><<<d.P, 256, 0, st>>>(d, S, tw_y, tw_z, ws, cs, w0p, wnyq, c0p, cnyq);                \
    return hipGetLastError();                                                                               \
  }
#define SPG_YZ4(NY_) SPG_YZ(NY_, 8) SPG_YZ(NY_, 16) SPG_YZ(NY_, 32) SPG_YZ(NY_, 64)
  SPG_YZ4(8) SPG_YZ4(16) SPG_YZ4(32) SPG_YZ4(64)
#undef SPG_YZ4
#undef SPG_YZ
  return hipErrorInvalidValue;
}

hipError_t launch_dc_nyquist(const Dims& d, float2* S, const float2* tw_z, const float* w0p, const float* wnyq,
                             const float2* c0p, const float2* cnyq, double* partials, hipStream_t st, int* nblocks_out) {
  const int L = d.nz;
  int T = 0;
  SPG_DISPATCH_L(L, (T = DcT<L_>::T));
  const dim3 grid(d.ny / 2 + 1), block(2 * T);
  if (nblocks_out) *nblocks_out = d.ny / 2 + 1;
  if (partials) {
    SPG_DISPATCH_L(L, (k_dc_nyquist<L_, true><<<grid, block, 0, st>>>(S, d.P, d.ny, tw_z, w0p, wnyq, c0p, cnyq, partials)));
  } else {
    SPG_DISPATCH_L(L, (k_dc_nyquist<L_, false><<<grid, block, 0, st>>>(S, d.P, d.ny, tw_z, w0p, wnyq, c0p, cnyq, partials)));
  }
  return hipGetLastError();
}

hipError_t launch_r2c_x(const Dims& d, const void* rin, bool rin_bf16, float2* S, const float2* tw_m,
                        const float2* tw_n, hipStream_t st) {
  const int M = d.P;
  const int T = tpt(M);
  if (T == 0) return hipErrorInvalidValue;
  const int NR = 256 / T < 16 ? 256 / T : 16;
  const int nrows = d.ny * d.nz;
  const dim3 grid((nrows + NR - 1) / NR), block(NR * T);
  if (rin_bf16) {
    SPG_DISPATCH_L(M, (k_r2c_x<L_, true><<<grid, block, 0, st>>>(rin, S, nrows, tw_m, tw_n, NR)));
  } else {
    SPG_DISPATCH_L(M, (k_r2c_x<L_, false><<<grid, block, 0, st>>>(rin, S, nrows, tw_m, tw_n, NR)));
  }
  return hipGetLastError();
}

hipError_t launch_c2r_x(const Dims& d, const float2* S, void* rout, bool rout_bf16, const float2* tw_m,
                        const float2* tw_n, hipStream_t st) {
  const int M = d.P;
  const int T = tpt(M);
  if (T == 0) return hipErrorInvalidValue;
  const int NR = 256 / T < 16 ? 256 / T : 16;
  const int nrows = d.ny * d.nz;
  const dim3 grid((nrows + NR - 1) / NR), block(NR * T);
  if (rout_bf16) {
    SPG_DISPATCH_L(M, (k_c2r_x<L_, true><<<grid, block, 0, st>>>(S, rout, nrows, tw_m, tw_n, NR)));
  } else {
    SPG_DISPATCH_L(M, (k_c2r_x<L_, false><<<grid, block, 0, st>>>(S, rout, nrows, tw_m, tw_n, NR)));
  }
  return hipGetLastError();
}

int prox_num_blocks(const Dims& d, int zc) {
  const int ntx = (d.nx + PT_TX - 1) / PT_TX;
  const int nty = (d.ny + PT_TY - 1) / PT_TY;
  const int ntz = (d.nz + zc - 1) / zc;
  return ntx * nty * ntz;
}

hipError_t launch_prox_tv(const Dims& d, const ProxArgs& a, int store, bool check, hipStream_t st, bool mon) {
  const int ntx = (d.nx + PT_TX - 1) / PT_TX;
  const int nty = (d.ny + PT_TY - 1) / PT_TY;
  if (a.zc < 1 || (check && mon)) return hipErrorInvalidValue;
  const dim3 grid(prox_num_blocks(d, a.zc)), block(256);
#define SPG_PROX(ST_) \
  do { if (check) k_prox_tv<ST_, true><<<grid, block, 0, st>>>(a, ntx, nty); \
       else if (mon) k_prox_tv<ST_, false, true><<<grid, block, 0, st>>>(a, ntx, nty); \
       else k_prox_tv<ST_, false><<<grid, block, 0, st>>>(a, ntx, nty); } while (0)
  switch (store) {
    case ST_PLAIN: SPG_PROX(ST_PLAIN); break;
    case ST_COMP: SPG_PROX(ST_COMP); break;
    case ST_BF16: SPG_PROX(ST_BF16); break;
    default: return hipErrorInvalidValue;
  }
#undef SPG_PROX
  return hipGetLastError();
}

static dim3 ew_grid(long long n) {
  long long g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return dim3((unsigned)g);
}

bool prox_fft_supported(const Dims& d) {
  return (d.nx == 32 || d.nx == 64 || d.nx == 128 || d.nx == 256 || d.nx == 512) && d.ny >= PF_TY &&
         d.ny % PF_TY == 0;
}

int prox_fft_num_blocks(const Dims& d, int zc) { return (d.ny / PF_TY) * ((d.nz + zc - 1) / zc); }

hipError_t launch_prox_fft(const Dims& d, const ProxArgs& a, float2* S, const float2* tw_m, const float2* tw_n,
                           int store, hipStream_t st, bool mon) {
  if (!prox_fft_supported(d) || a.zc < 1 || store < ST_PLAIN || store > ST_BF16) return hipErrorInvalidValue;
  const int nty = d.ny / PF_TY;
  const long long nblk = (long long)nty * ((d.nz + a.zc - 1) / a.zc);
  if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblk), block(2 * d.nx);
  // Streaming stores pay where the spectrum alone (4 bytes per voxel) outgrows the 256 MiB
  // last-level cache (measured at 512^3); smaller maps are read back by the next pass while
  // still cached (measured on the batch of 128^3-256^3 maps).
  const bool stream = (double)d.nvox * 4.0 >= 256.0 * 1024 * 1024;
#define SPG_PF2(NX_, ST_)                                                                          \
  if (mon && a.xprev) k_prox_fft<NX_, ST_, true, false, true><<<grid, block, 0, st>>>(a, S, tw_m, tw_n, nty); \
  else if (mon) k_prox_fft<NX_, ST_, false, false, true><<<grid, block, 0, st>>>(a, S, tw_m, tw_n, nty); \
  else if (a.xprev) k_prox_fft<NX_, ST_, true, false><<<grid, block, 0, st>>>(a, S, tw_m, tw_n, nty); \
  else if (stream) k_prox_fft<NX_, ST_, false, true><<<grid, block, 0, st>>>(a, S, tw_m, tw_n, nty);     \
  else k_prox_fft<NX_, ST_, false, false><<<grid, block, 0, st>>>(a, S, tw_m, tw_n, nty);
#define SPG_PF(NX_)                                   \
  switch (store) {                                    \
    case ST_PLAIN: SPG_PF2(NX_, ST_PLAIN); break;     \
    case ST_COMP: SPG_PF2(NX_, ST_COMP); break;       \
    default: SPG_PF2(NX_, ST_BF16); break;            \
  }
  switch (d.nx) {
    case 32: SPG_PF(32); break;
    case 64: SPG_PF(64); break;
    case 128: SPG_PF(128); break;
    case 256: SPG_PF(256); break;
    default: SPG_PF(512); break;
  }
#undef SPG_PF
#undef SPG_PF2
  return hipGetLastError();
}

hipError_t launch_prime(const Dims& d, void* rbuf, const float* xk_hi, const uint16_t* xk_lo, const float* xo_hi,
                        const uint16_t* xo_lo, double m, int read_old, int store, hipStream_t st) {
  const dim3 g = ew_grid(d.nvox);
  if (store == ST_COMP) k_prime<ST_COMP><<<g, 256, 0, st>>>(rbuf, xk_hi, xk_lo, xo_hi, xo_lo, m, read_old, d.nvox);
  else if (store == ST_BF16) k_prime<ST_BF16><<<g, 256, 0, st>>>(rbuf, xk_hi, xk_lo, xo_hi, xo_lo, m, read_old, d.nvox);
  else k_prime<ST_PLAIN><<<g, 256, 0, st>>>(rbuf, xk_hi, xk_lo, xo_hi, xo_lo, m, read_old, d.nvox);
  return hipGetLastError();
}

hipError_t launch_f32_to_bf16(const float* src, uint16_t* dst, long long n, hipStream_t st) {
  k_f32_to_bf16<<<ew_grid(n), 256, 0, st>>>(src, dst, n);
  return hipGetLastError();
}

hipError_t launch_bf16_to_f32(const uint16_t* src, float* dst, long long n, hipStream_t st) {
  k_bf16_to_f32<<<ew_grid(n), 256, 0, st>>>(src, dst, n);
  return hipGetLastError();
}

hipError_t launch_set_map(const Dims& d, const float* x0, float* hi, uint16_t* lo, hipStream_t st) {
  k_set_map<<<ew_grid(d.nvox), 256, 0, st>>>(x0, hi, lo, d.nvox);
  return hipGetLastError();
}

hipError_t launch_get_map(const Dims& d, const float* hi, const uint16_t* lo, float* out, bool compensated,
                          hipStream_t st) {
  if (compensated) k_get_map<true><<<ew_grid(d.nvox), 256, 0, st>>>(hi, lo, out, d.nvox);
  else k_get_map<false><<<ew_grid(d.nvox), 256, 0, st>>>(hi, lo, out, d.nvox);
  return hipGetLastError();
}

hipError_t launch_fill(float* dst, long long n, float value, hipStream_t st) {
  k_fill<<<ew_grid(n), 256, 0, st>>>(dst, n, value);
  return hipGetLastError();
}

hipError_t launch_fold(const Dims& d, const float* w, const float2* b, float* ws, float* w0p, float* wnyq,
                       float2* cs, float2* c0p, float2* cnyq, double* partials, int nblocks, hipStream_t st) {
  k_fold<<<nblocks, 256, 0, st>>>(d, w, b, ws, w0p, wnyq, cs, c0p, cnyq, partials);
  return hipGetLastError();
}

hipError_t launch_data_stats(const Dims& d, const float* w, const float2* b, double* partials, int nblocks,
                             hipStream_t st) {
  k_data_stats<<<nblocks, 256, 0, st>>>(d, w, b, partials);
  return hipGetLastError();
}

hipError_t launch_weight_stats(const Dims& d, const float* a, double* partials, int nblocks, hipStream_t st) {
  k_weight_stats<<<nblocks, 256, 0, st>>>(d.nvox, a, partials);
  return hipGetLastError();
}

hipError_t launch_reweight(const Dims& d, const float* hi, const uint16_t* lo, void* u, void* v, double eps1,
                           double eps2, int store, double* partials, int nblocks, hipStream_t st) {
  if (store == ST_COMP) k_reweight<true, false><<<nblocks, 256, 0, st>>>(d, hi, lo, u, v, eps1, eps2, partials);
  else if (store == ST_BF16) k_reweight<false, true><<<nblocks, 256, 0, st>>>(d, hi, lo, u, v, eps1, eps2, partials);
  else k_reweight<false, false><<<nblocks, 256, 0, st>>>(d, hi, lo, u, v, eps1, eps2, partials);
  return hipGetLastError();
}

hipError_t launch_log_terms(const Dims& d, const float* hi, const uint16_t* lo, double eps1, double eps2, bool comp,
                            double* partials, int nblocks, hipStream_t st) {
  if (comp) k_reweight<true, false, true><<<nblocks, 256, 0, st>>>(d, hi, lo, nullptr, nullptr, eps1, eps2, partials);
  else k_reweight<false, false, true><<<nblocks, 256, 0, st>>>(d, hi, lo, nullptr, nullptr, eps1, eps2, partials);
  return hipGetLastError();
}

hipError_t launch_obj_finish(const double* pa, int na, const double* pb, int nb, const double* pc, int nc, double c0,
                             double lam, double mu, double gamma, double* out, hipStream_t st) {
  k_obj_finish<<<1, 256, 0, st>>>(pa, na, pb, nb, pc, nc, c0, lam, mu, gamma, out);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int n, int nq, const int* ops, double* out, hipStream_t st) {
  if (nq < 1 || nq > 8) return hipErrorInvalidValue;
  RedOps r{};
  for (int i = 0; i < nq; ++i) r.op[i] = ops[i];
  k_reduce<<<1, 256, 0, st>>>(partials, n, nq, r, out);
  return hipGetLastError();
}

hipError_t launch_fsc_shells(const Dims& d, const float2* S1, const float2* S2, int nshells, double* partials,
                             int nblocks, double* out, hipStream_t st) {
  k_fsc_shells<<<nblocks, FSC_THREADS, (FSC_THREADS / 64) * 3 * nshells * sizeof(double), st>>>(d, S1, S2, nshells,
                                                                                                 partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_fsc_final<<<(3 * nshells + 255) / 256, 256, 0, st>>>(partials, nblocks, nshells, out);
  return hipGetLastError();
}

hipError_t launch_adj_prox(const Dims& d, const float* xn, const float* abar, const float* gdat, const float* u,
                           float lr, float* zbar, float* rbar, double* partials, int nblocks, hipStream_t st) {
  k_adj_prox<<<nblocks, 256, 0, st>>>(d.nvox, xn, abar, gdat, u, lr, zbar, rbar, partials);
  return hipGetLastError();
}

hipError_t launch_adj_tv(const Dims& d, const float* xk, const float* xkm, float m, const float* zbar, const float* hz,
                         const float* v, float lr, float mu, float eps, float* abar_k, float* abar_km,
                         double* partials, int nblocks, hipStream_t st) {
  k_adj_tv<<<nblocks, 256, 0, st>>>(d, xk, xkm, m, zbar, hz, v, lr, mu, eps, abar_k, abar_km, partials);
  return hipGetLastError();
}

hipError_t launch_expand_bbar(const Dims& d, const float2* S, const float* w, float2* out, hipStream_t st) {
  k_expand_bbar<<<ew_grid(d.nvox), 256, 0, st>>>(d, S, w, out);
  return hipGetLastError();
}

hipError_t launch_backproject(const Dims& d, int n_img, int m, const float2* images, const double* rots,
                              const float* ctf, const float* weights, double h, void* ws, float* w, float2* b,
                              hipStream_t st) {
  // workspace: 3 nvox fixed-point sums, then the 3 term maxima (all zero bits to start)
  unsigned long long* acc = static_cast<unsigned long long*>(ws);
  unsigned long long* mx = acc + 3 * d.nvox;
  k_fill_f64<<<ew_grid(3 * d.nvox + 3), 256, 0, st>>>(static_cast<double*>(ws), 3 * d.nvox + 3);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long total = (long long)n_img * m * m;
  long long g = (total + 255) / 256;
  if (g > 65536) g = 65536;
  k_bp_max<<<(unsigned)(g < 1024 ? g : 1024), 256, 0, st>>>(n_img, m, images, ctf, weights, mx);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_backproject<<<(unsigned)g, 256, 0, st>>>(d, n_img, m, images, rots, ctf, weights, h, acc, mx);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_backproject_final<<<ew_grid(d.nvox), 256, 0, st>>>(d.nvox, total, acc, mx, w, b);
  return hipGetLastError();
}

}  // namespace spg

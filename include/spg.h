/*
 * spg.h -- C ABI of the MI355X (gfx950) solver for the reweighted weighted-l1 plus
 * total-variation reconstruction of a density map by the smoothing proximal
 * gradient (SPG) method (Luo, "Improving the resolution of Cryo-EM single particle
 * analysis", arXiv 1905.13408, section 2 eq 8-22 and section 2.5 eq 31).
 *
 * Problem solved (eq 31 with the reweighted penalties of eq 11 and the Nesterov
 * smoothing of eq 14; paper letters in brackets):
 *
 *   min_x  1/2 sum_k w_k |(A x)_k - b_k|^2            data term, A = unitary 3D DFT
 *        + lambda sum_i u_i |x_i|                      weighted l1        [alpha, w'_j]
 *        + mu     sum_i v_i phi_eps(|(D x)_i|_2)       weighted smoothed TV [beta, w_j, mu]
 *        + gamma  |x - x_prev|^2                       implicit-descent term of eq 22
 *
 * x is a real nz*ny*nx map in C order (x fastest).  D is the backward difference
 * of eq 12 with periodic wrap; phi_eps is the per-voxel value of eq 14
 * (t^2/(2 eps) below eps, t - eps/2 above).  One SPG iteration (eq 20-21 with
 * Beck-Teboulle momentum) is
 *
 *   y   = x_k + m_k (x_k - x_{k-1})
 *   z   = y - lr (Re A^H(w (A y - b)) + mu D^T(v * Dy / max(eps, |Dy|)) + 2 gamma (y - x_prev))
 *   x_{k+1} = sign(z) max(|z| - lr lambda u, 0)
 *
 * with lr = 1/L, L = max_k (w_k + w_{-k})/2 + mu max(v) ||D||^2 / eps + 2 gamma.
 * Reweighting (eq 11) sets u = 1/(|x| + eps1), v = 1/(|Dx| + eps2) from the
 * current map and restarts the momentum.
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers on the current HIP device, owned by
 *    the caller.  Calls are asynchronous on the problem's stream unless stated;
 *    the caller keeps inputs alive until the stream has passed the call.
 *  - The library allocates no device memory: all state lives in the caller's
 *    workspace (size from spg_workspace_size).  It creates HIP events only
 *    while profiling is enabled.
 *  - Arguments are validated on the host before anything is enqueued; a call
 *    that returns an error leaves the problem as it was.  A HIP error makes the
 *    problem return SPG_E_DEVICE from then on.
 *  - A problem belongs to one stream and is not thread-safe; distinct problems
 *    are independent.
 */
#ifndef SPG_H
#define SPG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPG_OK = 0,
  SPG_E_INVAL = -1,       /* bad argument (pointer, size, value)                    */
  SPG_E_NOMEM = -2,       /* workspace smaller than spg_workspace_size              */
  SPG_E_DEVICE = -3,      /* a HIP call failed; the problem is unusable             */
  SPG_E_STATE = -4,       /* call out of order (e.g. run before set_data)           */
  SPG_E_NONFINITE = -5,   /* non-finite value in w, b, u or v                       */
  SPG_E_DIVERGED = -6,    /* non-finite objective (spg_final_check, the monitor)    */
  SPG_E_UNSUPPORTED = -7  /* valid request this build does not implement            */
} spg_status;

typedef struct spg_problem spg_problem;   /* opaque, owned by the library */

/* Flag bits of spg_params.flags. */
#define SPG_FLAG_COMPENSATED 1   /* iterate stored as fp32 hi + bf16 lo (about 32 significant
                                    bits) with the prox and momentum in fp64; without it the
                                    iterate is plain fp32 and all arithmetic is fp32        */
#define SPG_FLAG_BF16_STORAGE 2  /* fp32 iterate, but the penalty weights u, v and the
                                    gradient / extrapolated map are stored in bf16 (fp32
                                    arithmetic); excludes SPG_FLAG_COMPENSATED             */
#define SPG_FLAG_MONITOR 4       /* objective monitor: every obj_every-th iteration of a round
                                    also evaluates the smoothed objective F_eps (eq 31 with
                                    eq 14) at its extrapolated point y_k, from fp64 partials
                                    of the z pass (data term) and of the stencil kernel
                                    (penalty terms); see spg_objective_history             */

typedef struct {
  int32_t nx, ny, nz;   /* grid; each a power of two in [4, 512], or 160 or 192        */
  double lambda;        /* l1 weight (paper alpha), >= 0                                */
  double mu;            /* TV weight (paper beta), >= 0                                 */
  double eps;           /* Nesterov smoothing parameter (paper mu in eq 14), > 0        */
  double gamma;         /* implicit-descent weight of eq 22 (paper gamma), >= 0         */
  int32_t accel;        /* 1: FISTA momentum (default); 0: un-accelerated eq 20-21      */
  int32_t flags;        /* SPG_FLAG_* bits                                              */
  int32_t obj_every;    /* >= 1 with SPG_FLAG_MONITOR: monitor iterations j of a round with
                           j % obj_every == 0 (j = 1, 2, ... since the last momentum
                           restart); >= 0 and unused otherwise                          */
} spg_params;

typedef struct {
  int64_t iters_done;   /* iterations since spg_create                                   */
  int32_t round;        /* 1 + number of spg_reweight calls                              */
  int32_t iter_in_round;/* iterations since the last momentum restart                    */
  double lr;            /* current step 1/L                                              */
  double L;             /* current Lipschitz bound                                       */
  double obj_smoothed;  /* SPG_FLAG_MONITOR: F_eps(y_k) of the last monitored iteration  */
                        /* (NaN before the first one, and without the flag)             */
  int64_t obj_iter;     /* its iteration number k (counted as iters_done), 0 if none     */
} spg_stats;

/* Bytes of device workspace a problem with these parameters needs (host only,
 * no HIP call).  SPG_E_INVAL for invalid parameters. */
spg_status spg_workspace_size(const spg_params* p, size_t* bytes);

/* Create a problem whose state lives in d_workspace (>= spg_workspace_size bytes,
 * 256-byte aligned, device memory that the caller frees after spg_destroy).
 * hip_stream is a hipStream_t (NULL = the default stream).  Host only: the first later
 * call that enqueues work uploads the FFT twiddle tables (computed in fp64 on the host),
 * sets x_0 = 0 and synchronises the stream once; if that fails, that call and every later
 * one return SPG_E_DEVICE. */
spg_status spg_create(const spg_params* p, void* d_workspace, size_t bytes, void* hip_stream,
                      spg_problem** out);

/* Destroy the problem object (host memory only; the workspace stays the caller's). */
spg_status spg_destroy(spg_problem* P);

/* Set the Fourier-space weights w (N(n) of eq 28; nz*ny*nx float, >= 0, FFT order:
 * index 0 is the zero frequency on every axis) and the data b (y(n)/sqrt(N(n)) of
 * eq 31; nz*ny*nx complex, interleaved re/im float pairs, FFT order).  The pair is
 * folded onto the half spectrum a real map needs (w~ = (w_k + w_{-k})/2 and
 * c = (w_k b_k + w_{-k} conj b_{-k})/2).  Synchronises the stream to check the
 * inputs: SPG_E_NONFINITE for NaN/Inf, SPG_E_INVAL for a negative weight or w == 0
 * everywhere with mu == 0.  Resets the momentum. */
spg_status spg_set_data(spg_problem* P, const float* d_w, const float* d_b);

/* Set the reweighting weights u (l1) and v (TV) of eq 11, nz*ny*nx float each,
 * finite and >= 0; NULL means uniform weight 1.  Copied into the workspace.
 * Synchronises to check them and to read max(v).  Resets the momentum. */
spg_status spg_set_penalty_weights(spg_problem* P, const float* d_u, const float* d_v);

/* Change lambda and mu (both >= 0).  Recomputes L; resets the momentum. */
spg_status spg_set_params(spg_problem* P, double lambda, double mu);

/* Implicit-descent term of eq 22: set gamma >= 0 and the previous M-step map x_prev
 * (nz*ny*nx float, copied into the workspace; NULL = the zero map).  Recomputes L and
 * resets the momentum. */
spg_status spg_set_prior(spg_problem* P, double gamma, const float* d_xprev);

/* Set the current map x_0 (nz*ny*nx float) or, with NULL, x_0 = 0.  Resets the momentum. */
spg_status spg_set_map(spg_problem* P, const float* d_x0);

/* Run K >= 0 SPG iterations (eq 20-21 with momentum) on the stream.  Does not
 * synchronise, except that with SPG_FLAG_MONITOR and opt_stats given it waits for the
 * last monitored objective (8 bytes) and returns SPG_E_DIVERGED if it is not finite.
 * opt_stats (may be NULL) receives the counters after the launches. */
spg_status spg_run(spg_problem* P, int32_t K, spg_stats* opt_stats);

/* The objective monitor (SPG_FLAG_MONITOR, section 2 eq 14 and eq 31): the n most recent
 * monitored values F_eps(y_k) = 1/2 sum w |A y_k - b|^2 + lambda sum u |y_k|
 * + mu sum v phi_eps(|D y_k|) + gamma |y_k - x_prev|^2 (fp32 transforms and stencil, fp64
 * sums in a fixed order) with their iteration numbers k, oldest first, into host arrays of
 * `cap` entries (either may be NULL when cap > 0 names the other); n = min(cap, entries
 * so far, 4096) into *n_out.  The library keeps the last 4096 entries since spg_create.
 * Synchronises the stream. */
spg_status spg_objective_history(spg_problem* P, double* h_values, int64_t* h_iters, int32_t cap,
                                 int32_t* n_out);

/* Reweight (eq 11): u = 1/(|x| + eps1), v = 1/(|Dx|_2 + eps2) from the current map,
 * then recompute L and restart the momentum.  eps1, eps2 > 0.  Synchronises to read
 * max(v) (8 bytes). */
spg_status spg_reweight(spg_problem* P, double eps1, double eps2);

/* Copy the current map x_K (the last prox output, rounded to float) to d_x_out
 * (nz*ny*nx float). */
spg_status spg_get_map(spg_problem* P, float* d_x_out);

/* Copy the current penalty weights to d_u_out / d_v_out (either may be NULL). */
spg_status spg_get_penalty_weights(spg_problem* P, float* d_u_out, float* d_v_out);

/* Evaluate, with fp64 accumulation and fp32 transforms in every storage mode, at the
 * current map x: the smoothed objective F_eps(x) (eq 31 with eq 14, gamma term included),
 * the unsmoothed objective F_0(x) (eq 31), and the
 * relative fixed-point residual |x - T(x)| / |x| of one un-accelerated step T
 * (eq 20-21), zero exactly at the minimiser.  Any output may be NULL.  Uses one
 * extra forward/inverse FFT pair and synchronises.  SPG_E_DIVERGED if F_eps is
 * not finite.  Leaves the iteration state unchanged. */
spg_status spg_final_check(spg_problem* P, double* F_eps, double* F_0, double* kkt_rel);

/* Scales for choosing the parameters (the paper's discussion of parameter choice, after
 * eq 33): rms_unreg = the root mean square over voxels of the unregularised solution
 * Re F^H (b [w > 0]) (F the unitary DFT of spg_set_data's convention), mean_w = the mean of
 * the Fourier weights w = N(n).  Both are taken by spg_set_data in fp64 (by Parseval,
 * rms_unreg^2 = sum_k |(b'(k) + conj b'(-k))/2|^2 / nvox with b' = b [w > 0]); this call
 * reads them on the host and does no GPU work.  Either output may be NULL.  SPG_E_STATE
 * before spg_set_data has succeeded. */
spg_status spg_param_scales(const spg_problem* P, double* rms_unreg, double* mean_w);

/* Parameters on those scales (same passage): lambda = rms_unreg * eps1 and
 * mu = rms_unreg * eps2 (the l1 and TV weights scaled by the reweighting floors they are
 * divided by), gamma = mean_w.  eps1, eps2 finite and > 0.  Host only; any output may be
 * NULL.  The caller applies them with spg_set_params / spg_create. */
spg_status spg_suggest_params(const spg_problem* P, double eps1, double eps2, double* lambda, double* mu,
                              double* gamma);

/* The log-penalty objective of eq 10, as a minimisation, at the current map x:
 *   G(x) = 1/2 sum_k w_k |(F x)_k - b_k|^2 + lambda sum_i log(|x_i| + eps1)
 *          + mu sum_i log(|(D x)_i|_2 + eps2),
 * D the periodic backward differences of eq 12; the gamma term of eq 22 is not included.
 * The reweighting of eq 11 replaces each logarithm by its tangent at the previous map, so
 * rounds solved to convergence do not increase G (up to the smoothing of eq 14).  The data
 * term is evaluated as in spg_final_check (fp32 transforms, fp64 accumulation); the
 * penalty sums read the full iterate in fp64.  eps1, eps2 finite and > 0.  Synchronises;
 * leaves the iteration state unchanged.  SPG_E_DIVERGED if G is not finite. */
spg_status spg_log_objective(spg_problem* P, double eps1, double eps2, double* G);

/* Checkpoint: bytes needed by spg_get_state, then copy the iteration state (current
 * and previous map, momentum counters, L, round) into / out of a caller device buffer.
 * Restoring into a problem with the same parameters, data and penalty weights gives
 * bitwise the same future iterates as the uninterrupted run. */
spg_status spg_state_size(const spg_problem* P, size_t* bytes);
spg_status spg_get_state(spg_problem* P, void* d_buf, size_t bytes);
spg_status spg_set_state(spg_problem* P, const void* d_buf, size_t bytes);

/* Launch shapes: columns per tile of the y and z transform passes (8 or 16) and the z-slab
 * depth of the stencil kernel (4..512 planes).  spg_autotune times each knob in turn
 * (coordinate search over {16, 8}, {16, 8}, fused x transforms {on, off} when they are on
 * (see spg_set_fusion), {32, 16, 64, 128, 256, 8, 4}) on `iters` iterations (after three
 * untimed ones, so that the momentum term is active) from the zero map, with the penalty
 * weights as set, with HIP events, each candidate twice (two sweeps, the faster time
 * counts), and keeps the fastest; it leaves the map at 0 with the momentum restarted.
 * Defaults: 16, 16 and a slab depth of 32 planes, halved (down to 4) while the stencil
 * kernel would run fewer than 512 blocks (small maps).  Results are bitwise independent of
 * the launch shape. */
spg_status spg_set_launch_shape(spg_problem* P, int32_t nt_y, int32_t nt_z, int32_t zc);
spg_status spg_get_launch_shape(const spg_problem* P, int32_t* nt_y, int32_t* nt_z, int32_t* zc);
spg_status spg_autotune(spg_problem* P, int32_t iters);

/* Fused x-axis transforms (on by default where supported: nx in {32, 64, 128, 256, 512} and
 * ny a multiple of 4).  An iteration then reads the data gradient as the rows of its
 * packed x-spectrum and writes the x-spectrum of the next extrapolated map from the
 * stencil/prox kernel itself, on tiles of 4 full-width rows, instead of running separate
 * x-axis inverse and forward real FFT sweeps over an fp32 map (16 bytes per voxel less
 * HBM traffic per iteration).  The iterates agree with the unfused path to rounding (the
 * same operations; the prox of the compensated mode is fp64 in both).  With
 * SPG_FLAG_BF16_STORAGE the fused path keeps the gradient and extrapolated rows in fp32.
 * spg_set_fusion(P, 1) on a grid without support returns SPG_E_UNSUPPORTED; 0 selects
 * the separate sweeps, which spg_autotune then keeps (it may turn the fused path off where
 * the separate sweeps measure faster, never on).  Iterations of spg_run_checkpointed and the
 * replays of spg_vjp always use the separate sweeps (the replays keep the data gradient of
 * every iteration), so that the recorded and replayed trajectories agree bitwise; the
 * setting is restored afterwards. */
spg_status spg_set_fusion(spg_problem* P, int32_t enable);
spg_status spg_get_fusion(const spg_problem* P, int32_t* enabled);

/* Batches: independent problems of any sizes (gold-standard half-maps, class volumes)
 * advanced together in one HIP graph.  spg_batch_create takes n (1..64) distinct problems
 * and the caller's stream (hipStream_t, NULL = default), which waits for every graph; it
 * creates its own launch stream and one capture stream per problem (default priority).
 * spg_batch_run(K) synchronises each problem's own stream, captures K iterations of every
 * problem as parallel branches of one graph (kernel nodes only), launches it, and makes
 * each problem's stream wait for it: the results equal K calls of spg_run per problem,
 * bitwise.  When every problem is in the
 * host-side iteration state the current graph was captured from (for instance after
 * spg_set_map restarted each of them) and K is unchanged, the instantiated graph is
 * launched again without a new capture.  Inside the graph the fused z pass runs one block
 * per work unit instead of persistent blocks, so that the branches share the GPU.  The
 * problems must outlive the batch and must not be used from another thread during
 * spg_batch_run; a problem whose run fails is left in SPG_E_DEVICE state like any other
 * device error.  spg_batch_destroy releases the streams, events and graph, not the
 * problems. */
typedef struct spg_batch spg_batch;
spg_status spg_batch_create(spg_problem* const* problems, int32_t n, void* hip_stream, spg_batch** out);
spg_status spg_batch_run(spg_batch* B, int32_t K);
spg_status spg_batch_destroy(spg_batch* B);

/* Reverse mode of an unrolled solve, for tuning lambda, mu and the data b: the gradient of
 * a scalar loss of x_K with respect to (lambda, mu, b) through K SPG iterations (eq 20-21
 * with momentum, lr = 1/L(mu) differentiated as well), by the chain rule with a.e.
 * derivatives at the soft-threshold and smoothing kinks.  Not available with
 * SPG_FLAG_BF16_STORAGE.
 *
 * spg_vjp_workspace_size: bytes of the caller's reverse-pass workspace for K iterations
 *   with a checkpoint every C iterations (1 <= C <= K): ceil(K/C)+1 ring checkpoints, C+2
 *   fp32 maps and C data gradients of one replayed segment, and five fp32 maps.
 * spg_run_checkpointed: restart the momentum at the current map x_0 and run K iterations,
 *   saving the iterate ring every C iterations into d_vjp_ws (256-byte aligned).
 * spg_vjp: given xbar = dloss/dx_K (nz*ny*nx float) and the Fourier weights w passed to
 *   spg_set_data, replay each segment from its checkpoint and walk it backwards; writes
 *   b_bar (nz*ny*nx complex, interleaved, FFT order; dloss = Re sum conj(b_bar) db) and the
 *   host scalars lam_bar, mu_bar.  SPG_E_STATE if no checkpointed run matches the current
 *   parameters.  Synchronises; leaves the problem at x_K. */
spg_status spg_vjp_workspace_size(const spg_problem* P, int32_t K, int32_t C, size_t* bytes);
spg_status spg_run_checkpointed(spg_problem* P, int32_t K, int32_t C, void* d_vjp_ws, size_t bytes);
spg_status spg_vjp(spg_problem* P, void* d_vjp_ws, size_t bytes, const float* d_w, const float* d_xbar,
                   float* d_bbar, double* lam_bar, double* mu_bar);

/* Backprojection as local kernel regression (section 2.2, eq 24-29), the producer of the
 * solver's inputs: image i's Fourier coefficient X at signed frequency (u, v) (2D FFT order,
 * v slow, u fast) lands at c = R_i (u, v, 0)^T (eq 24, c in (x, y, z) order) and is spread
 * over the 27 grid points round(c) + {-1, 0, 1}^3 (round(t) = floor(t + 1/2), periodic
 * wrap) with K = exp(-|c - n|^2 / h) (the paper uses h = 2), accumulating
 * num += p_i K CTF X and N += p_i K CTF^2 (eq 28).  Writes w = N (nz*ny*nx float) and
 * b = num / N (0 where N = 0; nz*ny*nx complex, interleaved), ready for spg_set_data.
 * d_images: n_img*m*m complex; d_rot: n_img row-major 3x3 double matrices; d_ctf: n_img*m*m
 * float or NULL (1); d_weight: n_img posterior weights or NULL (1).  Device pointers; the
 * workspace (spg_backproject_workspace_size bytes, 8-byte aligned) holds the accumulators;
 * asynchronous on hip_stream.  The sums are int64 fixed point with a power-of-two scale per
 * component (chosen from the largest term and the pixel count so that no sum can overflow;
 * terms are rounded at 2^-62 of that bound), so results are bitwise reproducible and do not
 * depend on the order of the images. */
spg_status spg_backproject_workspace_size(int32_t nx, int32_t ny, int32_t nz, size_t* bytes);
spg_status spg_backproject(int32_t nx, int32_t ny, int32_t nz, int32_t n_img, int32_t m, const float* d_images,
                           const double* d_rot, const float* d_ctf, const float* d_weight, double h,
                           void* d_workspace, size_t bytes, void* hip_stream, float* d_w_out, float* d_b_out);

/* Gold-standard Fourier shell correlation of eq 30 (section 2.3) between two real maps
 * d_map1, d_map2 (nz*ny*nx float each, each axis as in spg_params):
 *   FSC(s) = Re sum_{k in s} F conj G / sqrt(sum_{k in s} |F|^2 sum_{k in s} |G|^2)
 * over the full spectrum, shell s = floor(min(n) sqrt(sum_a (k_a / n_a)^2) + 1/2) of the
 * signed frequency k (for a cubic grid the rounded |k|), s in [0, nshells), 1 <= nshells
 * <= 1024; a shell without power in either map gives 0.  h_fsc receives nshells host
 * doubles.  The workspace (device, 256-byte aligned, spg_fsc_workspace_size bytes) is the
 * caller's; the call synchronises the stream.  Shell sums are fp64 in a fixed order, so
 * results are bitwise reproducible. */
spg_status spg_fsc_workspace_size(int32_t nx, int32_t ny, int32_t nz, int32_t nshells, size_t* bytes);
spg_status spg_fsc(int32_t nx, int32_t ny, int32_t nz, const float* d_map1, const float* d_map2, int32_t nshells,
                   void* d_workspace, size_t bytes, void* hip_stream, double* h_fsc);

/* spg_fsc for callers that cannot allocate device memory (code under HIP graph capture is
 * not meant: the call synchronises; tight loops and harnesses that forbid allocation are):
 * the same transforms, shell sums and result as spg_fsc, with the workspace in a static
 * device array of the library (72 MiB per device, held until the process ends) instead of a
 * caller buffer.  Grids whose spg_fsc_workspace_size exceeds 72 MiB - 64 KiB (more than
 * about 2^23 voxels) return SPG_E_NOMEM.  The first call on a device looks the array up and
 * writes its twiddle tables (once); no call allocates or frees device memory.  All calls on
 * one device share the array: calls that overlap on one device (other threads or streams)
 * race and must be serialised by the caller. */
spg_status spg_fsc_noalloc(int32_t nx, int32_t ny, int32_t nz, const float* d_map1, const float* d_map2,
                           int32_t nshells, void* hip_stream, double* h_fsc);

/* Kernel classes for spg_profile_begin.  On maps whose spectrum outgrows the 256 MiB
 * last-level cache the y forward, z and y inverse passes are launched as four column
 * ranges each (four launches per class and iteration); on small maps (ny, nz <= 64) one
 * launch does all three passes and the packed plane and is counted as the z class. */
typedef enum {
  SPG_KERNEL_FFT_Y_FWD = 0, /* y-axis forward column FFT                               */
  SPG_KERNEL_FFT_Z_WEIGHT,  /* z-axis forward FFT, Fourier weight multiply, inverse FFT  */
  SPG_KERNEL_DC_NYQUIST,    /* the packed kx = 0 / kx = nx/2 plane of the z pass         */
  SPG_KERNEL_FFT_Y_INV,     /* y-axis inverse column FFT                               */
  SPG_KERNEL_C2R_X,         /* x-axis inverse real FFT of the gradient spectrum         */
  SPG_KERNEL_PROX_TV,       /* smoothed-TV stencil, gradient step, soft threshold, momentum */
  SPG_KERNEL_R2C_X,         /* x-axis forward real FFT of the extrapolated map          */
  SPG_KERNEL_COUNT
} spg_kernel_class;

#define SPG_KERNEL_ALL (-1)

/* Profiling: time launches with HIP events recorded on the problem's stream around each
 * of them -- every launch of one kernel class, or of every class with SPG_KERNEL_ALL --
 * for at most `capacity` launches per class (launches past it are not timed and not
 * counted).  spg_profile_end synchronises and writes
 * per-class totals to total_ms[SPG_KERNEL_COUNT] (device ms) and
 * launches[SPG_KERNEL_COUNT]; either may be NULL. */
spg_status spg_profile_begin(spg_problem* P, int32_t kernel_class, int32_t capacity);
spg_status spg_profile_end(spg_problem* P, double* total_ms, int32_t* launches);

/* Failure injection, for tests of the error paths (failure detection): the problem lets
 * n more checked HIP calls succeed, then reports the next one as failed (after issuing it,
 * as a device error found late would), which makes the problem return SPG_E_DEVICE from
 * then on.  n = -1 turns injection off.  Host only; other problems are not affected. */
spg_status spg_debug_fail_after(spg_problem* P, int32_t n);

/* Static message for a status code; per-problem message of the last error. */
const char* spg_status_string(spg_status s);
const char* spg_last_error(const spg_problem* P);

#ifdef __cplusplus
}
#endif

#endif /* SPG_H */

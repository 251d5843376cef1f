/*
 * stride_hip.h -- C ABI of the MI355X (gfx950) acoustic full-waveform-inversion
 * hot path: finite-difference time stepping of the acoustic wave equation with
 * point sources and receivers, its exact discrete adjoint, and the gradient of
 * the L2 trace misfit with respect to the speed of sound.
 *
 * What is computed (Cueto et al., "Stride", arXiv 2110.03345):
 *   - Sec. 2.4, acoustic equation with constant density and no attenuation,
 *         (1/vp^2) d2p/dt2 = lap p + s,
 *     stepped by second-order leapfrog in time with an 8th- or 10th-order
 *     central Laplacian (the paper's solver is 10th order in space), a sponge
 *     absorbing layer, and off-grid sources/receivers by bi/tri-linear
 *     interpolation;
 *   - Sec. 2.2, reduced gradient of a PDE-constrained objective by the
 *     adjoint-state method: one forward and one adjoint propagation per shot
 *     (Sec. 3.2, 3.3), with the objective the L2 trace misfit
 *     J = 1/2 sum_{r,n} (traces[r][n] - observed[r][n])^2.
 *
 * Discrete scheme (the adjoint is its exact transpose, sponge included):
 *   u^{n+1} = a (2 u^n + k (L u^n + S^n)) - b u^{n-1},  u^0 = u^{-1} = 0,
 *   k = dt^2 vp^2, a = 1/(1 + eta dt/2), b = (1 - eta dt/2) a,
 *   S^n = sum_s W_s^T wavelet[s][n] / (cell volume),  traces[r][n] = W_r u^n,
 *   eta = sum_axes eta_max (d/nb)^2 in the nb-cell layer padded outside the
 *   physical grid, eta_max = 3 vref ln(1000) / (nb dx), zero inside.
 *   vp is replicated from the edge cells into the layer; the field is zero
 *   beyond the padded array.
 *
 * Conventions:
 *   - Arrays are C order (last axis contiguous).  vp and dvp have the physical
 *     shape; wavelets are [nsrc][nt]; traces, observed and grad_traces are
 *     [nrec][nt].  All of these are FP32 DEVICE pointers owned by the caller.
 *     nsrc or nrec may be 0: the wavelet (nsrc = 0) and the trace arrays
 *     (nrec = 0) may then be NULL.
 *   - Coordinates (src_xyz, rec_xyz) are FP64 HOST arrays [count][ndim] in
 *     metres, origin at physical node 0, axis order of the arrays.
 *   - ws is a caller-owned DEVICE workspace of ws_bytes bytes, 256-byte aligned,
 *     sized with stride_workspace_bytes().  Calls that run solves allocate
 *     nothing; stride_plan_create allocates the plan's small tap tables.
 *   - stream is a hipStream_t passed as void*; NULL is the default stream.
 *     A solve call reads max(vp) back for its stability check (one stream
 *     synchronisation before its time loop) and, while the non-finite check
 *     is on (stride_check_finite, the default), scans its outputs and waits
 *     for the result, so it returns after its work has finished; with the
 *     check off it returns once the time loop is enqueued.  The one-shot
 *     stride_forward / stride_gradient always return after the work.
 *   - Every entry point returns STRIDE_OK or a negative error code; nothing is
 *     enqueued when validation fails.  stride_last_error() returns a message
 *     for the calling thread's last error.
 *   - Plans are immutable after creation and may be shared between threads;
 *     concurrent solves need distinct workspaces.
 */
#ifndef STRIDE_HIP_H
#define STRIDE_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    STRIDE_OK = 0,
    STRIDE_E_INVALID_ARG = -1, /* bad pointer, size, order, shape or mode */
    STRIDE_E_CFL = -2,         /* dt * vp_max violates the stability limit of the scheme */
    STRIDE_E_GEOMETRY = -3,    /* a source or receiver lies outside the physical grid */
    STRIDE_E_WORKSPACE = -4,   /* ws_bytes below what the call needs */
    STRIDE_E_HIP = -5,         /* a HIP runtime call failed */
    STRIDE_E_NONFINITE = -6    /* NaN or infinity in a solve's outputs (stride_check_finite) */
};

/* Workspace modes: FORWARD (stride_plan_forward), GRADIENT (gradients,
 * forward_save/backward, the engine), FORWARD_MEDIUM (stride_plan_forward_medium),
 * GRADIENT_MEDIUM (stride_plan_gradient_medium). */
enum {
    STRIDE_MODE_FORWARD = 0,
    STRIDE_MODE_GRADIENT = 1,
    STRIDE_MODE_FORWARD_MEDIUM = 2,
    STRIDE_MODE_GRADIENT_MEDIUM = 3
};

/* Physical grid, stencil, sponge and time axis of a solve. */
typedef struct stride_grid {
    int32_t ndim;         /* 2 or 3 */
    int32_t space_order;  /* 8 or 10 */
    int32_t sponge_cells; /* nb >= 0 cells padded on every side */
    int32_t nt;           /* time samples, >= 2 */
    int64_t shape[3];     /* physical points per axis (>= 2; unused axes ignored) */
    double spacing[3];    /* metres */
    double sponge_vref;   /* reference speed of the sponge (m/s); 0 disables damping */
    double dt;            /* seconds */
    int32_t time_order;   /* 2 (leapfrog; 0 means 2) or 4: the leapfrog plus the
                             modified-equation correction dt^4/12 u_tttt (the paper's
                             solver is fourth-order in time, Sec. 2.4).  With 4:
                               p       = k (L u^n + St^n),
                               St^n    = (S^{n-1} + 10 S^n + S^{n+1}) / 12,
                               u^{n+1} = a (2 u^n + p + (k/12) L p) - b u^{n-1};
                             stable up to sqrt(3) times the leapfrog CFL limit.
                             Forward solves, gradients and stride_backward (dvp, and
                             dwavelet for nt <= 15360), in the batching engine too */
    int32_t interp;       /* off-grid sources and receivers (Sec. 2.4): 0 bi/tri-linear
                             (2 nodes per axis), 1 Kaiser-windowed sinc after Hicks
                             (8 nodes per axis: weight sinc(x) I0(b sqrt(1 - (x/4)^2)) /
                             I0(b), b = 6.31, at offset x cells; product over axes; a
                             point on a node gets that node alone).  Sinc taps must lie
                             in the padded grid: points within 4 cells of its edge (with
                             sponge_cells < 4) return GEOMETRY. */
    int32_t boundary;     /* absorbing layer in the sponge_cells padded cells (Sec. 2.4
                             offers a sponge and a PML): 0 the sponge above, 1 a
                             perfectly matched layer: complex coordinate stretching
                             d_a -> (1/s_a) d_a, s_a = 1 + zeta_a/(i omega), of each
                             axis, with memory variables psi_a (first derivative) and
                             chi_a (second) relaxed at rate zeta_a over the step
                             (E = exp(-zeta_a dt)):
                               chi_a^n     = E chi_a^{n-1} + (1-E) (D2_a u^n - D_a psi_a^n),
                               psi_a^{n+1} = E psi_a^n + (1-E) D_a u^n,
                               u^{n+1} = 2 u^n - u^{n-1}
                                         + k (sum_a (D2_a u^n - D_a psi_a^n - chi_a^n) + S^n),
                             D2_a the axis-a part of L, D_a the centred first
                             derivative of the same order, zeta_a = zeta_max (d/nb)^2
                             in the layer of axis a (d cells into it), zeta_max =
                             3 sponge_vref ln(1000) / (2 nb dx_a).  Forward solves
                             (stride_plan_forward[_static]) only; other solves
                             return INVALID_ARG for it. */
    int32_t checkpointing; /* gradients whose workspace cannot keep every state
                             (stride_gradient_path): 0 the library's choice,
                             segmented history where its cost model prefers it to
                             binomial checkpointing; 1 binomial checkpointing
                             always.  The results are the same bits either way. */
} stride_grid_t;

/* A plan: the validated grid plus the source/receiver tap tables of one shot
 * geometry on the current HIP device. */
typedef struct stride_plan stride_plan_t;

/* Validates the grid and geometry (CFL is checked per solve, against vp) and
 * builds the tap tables.  Errors: INVALID_ARG, GEOMETRY (Sec. 2.4 off-grid
 * points must lie in the physical grid), HIP. */
int stride_plan_create(const stride_grid_t* grid, int32_t nsrc, const double* src_xyz,
                       int32_t nrec, const double* rec_xyz, stride_plan_t** out);

/* Releases the plan (synchronises the device). */
int stride_plan_destroy(stride_plan_t* plan);

/* Padded extent per axis (shape + 2 nb; unused axes 1). */
int stride_plan_padded_shape(const stride_plan_t* plan, int64_t out[3]);

/* Workspace bytes for mode FORWARD or GRADIENT.  For GRADIENT, budget_bytes
 * caps the size: the forward wavefields are kept by binomial checkpointing
 * (Griewank-Walther revolve) with as many snapshots as fit, and 0 asks for the
 * size that keeps every state (no recomputation).  The snapshot count a solve
 * uses is derived from the ws_bytes it is given.  Errors: INVALID_ARG,
 * WORKSPACE (budget below the minimum of 8 wavefields plus traces; 10 with
 * time_order 4).  FORWARD_MEDIUM ignores budget_bytes and needs time_order 2;
 * GRADIENT_MEDIUM takes a budget as GRADIENT does (0 or a budget at least the
 * full size keeps every imaging factor). */
int stride_workspace_bytes(const stride_plan_t* plan, int32_t mode, size_t budget_bytes,
                           size_t* out_bytes);

/* Forward solve: traces[r][n] = W_r u^n, n = 0..nt-1.  vp must satisfy the
 * CFL limit (dt vp_max sqrt(lambda sum_a 1/dx_a^2) <= 2, lambda = 6.5016 for
 * order 8, 6.8267 for order 10); the check reads vp on the device and
 * synchronises the stream once.  Errors: INVALID_ARG, CFL, WORKSPACE, HIP. */
int stride_plan_forward(const stride_plan_t* plan, const float* vp, const float* wavelet,
                        float* traces, void* ws, size_t ws_bytes, void* stream);

/* Size of the static workspace of stride_plan_forward_static (64 MiB).  Each
 * device the library runs on holds one such block of device memory from the
 * loading of the library until the process ends. */
#define STRIDE_STATIC_WORKSPACE_BYTES (64u << 20)

/* stride_plan_forward for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same solve, with the same results bit for bit, whose
 * workspace (scratch scalars, k and the two wavefields, and p with
 * time_order 4) is the library's static workspace on the current device
 * instead of a caller buffer.  It calls no hipMalloc, hipFree or other
 * allocating routine; the caller passes vp, wavelet and traces as for
 * stride_plan_forward.  Limit: stride_workspace_bytes(plan, FORWARD) must not
 * exceed STRIDE_STATIC_WORKSPACE_BYTES (about 5.5 M padded points with
 * second-order time, 4.1 M with fourth-order), else WORKSPACE and nothing is
 * enqueued.  Every call on one device shares that device's workspace and
 * rewrites all of it that the solve reads (fields are cleared by a fill
 * kernel, not a memset), so calls in sequence on one stream are independent;
 * calls that overlap on one device (several streams or threads) race and must
 * not be issued.  The current device must be the plan's.  Like
 * stride_plan_forward it reads max(vp) back for the CFL check (one stream
 * synchronisation).  Errors: INVALID_ARG, CFL, WORKSPACE, HIP. */
int stride_plan_forward_static(const stride_plan_t* plan, const float* vp, const float* wavelet,
                               float* traces, void* stream);

/* Forward solve in a heterogeneous medium (Sec. 2.4 acoustic equation with
 * variable density and power-law attenuation, y = att_power in {0, 2}):
 *   (1/vp^2) p_tt = rho div(rho^{-1} grad p) + eta d/dt (-lap)^{y/2} p + s,
 *   eta = -2 alpha0 vp^{y-1},
 * discretised as
 *   u^{n+1} = a (2 u^n + k (L u^n + sum_a gamma_a D_a u^n + S^n
 *                           [+ beta (L u^n - L u^{n-1})  if y = 2])) - b u^{n-1},
 * gamma_a = -D_a ln rho (D_a the centred first derivative of the stencil's
 * order; rho edge-replicated into the sponge, ln rho constant beyond the padded
 * array), beta = 2 alpha0 vp / dt; for y = 0 the damping of a and b becomes
 * the sponge's eta + 2 alpha0 vp.  alpha0 is in Np/m (y = 0) or
 * Np/m/(rad/s)^2 (y = 2): amplitudes decay as exp(-alpha0 omega^y r).
 * vp, rho and alpha0 are device arrays of the physical shape; rho NULL means
 * constant density, alpha0 NULL no attenuation.  rho must be positive and
 * finite, alpha0 non-negative and finite.  Stability: with y = 2 the limit
 * becomes dt sqrt(max vp^2 (1 + 2 beta)) sqrt(lambda sum 1/dx^2) <= 2 (checked
 * on the device, one stream sync).  time_order must be 2.  ws: FORWARD_MEDIUM
 * bytes (k, three wavefields, ndim + 1 medium fields).  Forward only.  Errors:
 * INVALID_ARG, CFL, WORKSPACE, HIP. */
int stride_plan_forward_medium(const stride_plan_t* plan, const float* vp, const float* rho,
                               const float* alpha0, int32_t att_power, const float* wavelet,
                               float* traces, void* ws, size_t ws_bytes, void* stream);

/* Shot gradient in a heterogeneous medium (the medium of
 * stride_plan_forward_medium, rho and alpha0 fixed): traces (optional), misfit
 * J = 1/2 sum (traces - observed)^2 (FP64 device scalar) and dvp = dJ/dvp, by
 * the exact discrete adjoint of the medium step (Sec. 2.2 adjoint-state
 * method).  With w = a k lambda the adjoint step is
 *   w^m = a (2 w^{m+1} + k (L y - sum_a D_a (gamma_a w^{m+1}) + R^T r^m)) - b w^{m+2},
 *   y = (1 + beta) w^{m+1} - beta w^{m+2}   (beta = 0 for y = 0),
 * (D_a is antisymmetric, so the density term transposes to -D_a (gamma_a .)),
 * and dvp = P^T (2/vp) sum_n w^{n+1} h^n with h^n the step's right-hand side v^n
 * plus the attenuation's vp dependence: y = 2, + (beta/2) (L u^n - L u^{n-1});
 * y = 0, + (att a dt/4) ((2 u^{n-1} - 2 u^n)/k - v^n), att = 2 alpha0 vp.  With
 * ws_bytes >= the GRADIENT_MEDIUM size for budget 0 (about nt fields) every
 * step's h is kept; a smaller workspace (stride_workspace_bytes with a budget)
 * keeps start states of segments and h over the last segment, recomputing each
 * other segment's h once (segmented history, when the segments fit), or else
 * keeps forward states by binomial checkpointing and recomputes h^m from the
 * stored (u^m, u^{m-1}) before adjoint step m; the same result bit for bit.
 * Second-order time, sponge boundary.  Errors: INVALID_ARG, CFL, WORKSPACE (below
 * the checkpointed minimum of 13 + ndim wavefields plus traces), HIP,
 * NONFINITE. */
int stride_plan_gradient_medium(const stride_plan_t* plan, const float* vp, const float* rho,
                                const float* alpha0, int32_t att_power, const float* wavelet,
                                const float* observed, float* traces, double* misfit, float* dvp,
                                void* ws, size_t ws_bytes, void* stream);

/* One gradient-descent step of an inversion loop (Sec. 2.2 local optimiser):
 *   vp[i] = clamp(vp[i] - step_size m[i] g[i] / max_j |m[j] g[j]|, vmin, vmax),
 * m the mask (NULL = 1 everywhere; e.g. 0 outside a region of interest), so
 * step_size is the largest change of vp.  All arrays device, n values; work is
 * one device uint32 of scratch (it receives max |m g| as float bits).  A zero
 * gradient leaves vp clamped but unchanged.  Errors: INVALID_ARG, HIP. */
int stride_descent_step(float* vp, const float* grad, const float* mask, int64_t n, float step_size,
                        float vmin, float vmax, uint32_t* work, void* stream);

/* Zero-phase low-pass of [count][nt] device rows sampled at dt, for the
 * frequency blocks of an inversion (Sec. 3.2 band-limits wavelets and traces
 * per block): out = h * in with zeros beyond the record, h the Hann-windowed
 * sinc of cutoff f_max over |k| <= K = ceil(2 / (f_max dt)),
 *   h_k = 2 f_max dt sinc(2 f_max k dt) (0.5 + 0.5 cos(pi k / (K + 1))),
 * scaled to unit sum (unit gain at DC, half amplitude at f_max).  out may alias
 * in.  Needs f_max < 1/(2 dt) and nt + 2K + 1 <= 15360 samples.  Errors:
 * INVALID_ARG, HIP. */
int stride_lowpass(const float* in, float* out, int32_t count, int32_t nt, double dt,
                   double f_max, void* stream);

/* Forward solve that also keeps the checkpoints of the forward wavefield in
 * ws (GRADIENT-sized) for a later stride_backward with the same ws, vp and
 * wavelet. */
int stride_forward_save(const stride_plan_t* plan, const float* vp, const float* wavelet,
                        float* traces, void* ws, size_t ws_bytes, void* stream);

/* Vector-Jacobian product of (vp, wavelet) -> traces at the point of the
 * preceding stride_forward_save on ws: dvp = (d traces / d vp)^T grad_traces
 * (physical shape) and, if dwavelet is not NULL, dwavelet = (d traces /
 * d wavelet)^T grad_traces ([nsrc][nt]).  Recomputes forward states from the
 * checkpoints as the revolve schedule dictates.  Sec. 2.2 adjoint method. */
int stride_backward(const stride_plan_t* plan, const float* vp, const float* wavelet,
                    const float* grad_traces, float* dvp, float* dwavelet, void* ws,
                    size_t ws_bytes, void* stream);

/* Shot gradient: forward (traces optional, may be NULL), residual, misfit
 * (FP64 device scalar) and dvp = dJ/dvp. */
int stride_plan_gradient(const stride_plan_t* plan, const float* vp, const float* wavelet,
                         const float* observed, float* traces, double* misfit, float* dvp,
                         void* ws, size_t ws_bytes, void* stream);

/* One-shot forms (plan created and destroyed inside; blocking). */
int stride_forward(const stride_grid_t* grid, const float* vp, const float* wavelet, int32_t nsrc,
                   const double* src_xyz, int32_t nrec, const double* rec_xyz, float* traces,
                   void* ws, size_t ws_bytes, void* stream);
int stride_gradient(const stride_grid_t* grid, const float* vp, const float* wavelet,
                    int32_t nsrc, const double* src_xyz, int32_t nrec, const double* rec_xyz,
                    const float* observed, double* misfit, float* dvp, void* ws, size_t ws_bytes,
                    void* stream);
int stride_workspace_query(const stride_grid_t* grid, int32_t nsrc, int32_t nrec, int32_t mode,
                           size_t budget_bytes, size_t* out_bytes);

/* How stride_plan_gradient / stride_forward_save + stride_backward run in a
 * GRADIENT workspace of ws_bytes, for a plan on `grid` with nrec receivers
 * (host only, no device needed; Sec. 2.2 adjoint-state method with
 * the forward wavefields kept or recomputed):
 *   path 0 (STRIDE_PATH_FULL_HISTORY): every state fits; the forward keeps
 *     v^n = L u^n + S^n (second order; p^n with time_order 4) and the adjoint
 *     images from it;
 *   path 1 (STRIDE_PATH_SEGMENTED): the forward keeps the states at the
 *     starts of `segments` segments and v^n (p^n) over the last one; each
 *     other segment's v^n (p^n) is recomputed once, just before its adjoint
 *     steps;
 *   path 2 (STRIDE_PATH_BINOMIAL): binomial checkpointing (revolve) with the
 *     adjoint recomputing L u^m itself.
 * The library takes path 1 over path 2 when its cost model of the step
 * kernels says it is faster; all three give the same bits.  forward_steps:
 * forward step launches per gradient.  Errors: INVALID_ARG, WORKSPACE. */
#define STRIDE_PATH_FULL_HISTORY 0
#define STRIDE_PATH_SEGMENTED 1
#define STRIDE_PATH_BINOMIAL 2
int stride_gradient_path(const stride_grid_t* grid, int32_t nrec, size_t ws_bytes, int32_t* path,
                         int64_t* forward_steps, int32_t* segments);

/* Checkpointing schedule summary for nt steps within `fields` wavefields
 * (host only): snapshots used, total forward steps (nt - 1 means no
 * recomputation) and peak wavefields alive. */
int stride_schedule_info(int32_t nt, int64_t fields, int32_t* snaps, int64_t* forward_steps,
                         int32_t* peak_fields);

/* ---------------------------------------------------------------- batching
 * An engine advances many shots on one padded grid together (shot
 * parallelism, Sec. 2.5, on one device): each slot holds one forward solve or
 * one shot gradient with its own model, geometry, nt, dt, sponge speed and
 * time order; a tick advances every active slot by one forward or adjoint
 * step, the slots that run the same step kind sharing one batched launch
 * (forward, forward keeping v, fourth-order p / q, adjoint with imaging,
 * adjoint imaging from v, adjoint without imaging, and the two fourth-order
 * corrections).  A gradient whose workspace holds every state takes the
 * full-history path of stride_plan_gradient (second order: the forward keeps
 * v^n = L u^n + S^n and the adjoint images from it; fourth order: the forward
 * keeps p^n), else the checkpointed one.  Slots attach and detach between
 * stride_engine_run calls (continuous batching).  A slot computes exactly the
 * bits the one-shot entry points compute.  All calls on one engine must use
 * the same stream and come from one thread.  Sponge boundaries only. */
typedef struct stride_engine stride_engine_t;

/* grid fixes shape, spacing, space_order and sponge_cells (nt, dt and
 * sponge_vref are per slot, taken from each plan).  max_receivers bounds the
 * receivers of an attached plan; max_chunk bounds the ticks per run call
 * (rounded down to a power of two); use_graphs replays each chunk as a
 * captured hipGraph (needs a non-NULL stream).  Allocates the engine's slot
 * tables (device and pinned host). */
int stride_engine_create(const stride_grid_t* grid, int32_t max_slots, int32_t max_receivers,
                         int32_t max_chunk, int32_t use_graphs, stride_engine_t** out);
int stride_engine_destroy(stride_engine_t* engine);

/* Attaches one shot to a free slot and enqueues its setup on stream.  mode
 * FORWARD needs traces; mode GRADIENT needs observed, misfit (device FP64
 * scalar) and dvp, traces optional.  ws / ws_bytes: a workspace sized with
 * stride_workspace_bytes for the mode (gradient snapshots follow ws_bytes).
 * vp_max > 0 is the caller's maximum of vp for the CFL check; vp_max <= 0
 * reads it from the device (one stream sync).  Buffers must stay valid until
 * the slot finishes.  Errors: INVALID_ARG (grid mismatch, no free slot, too
 * many receivers), CFL, WORKSPACE. */
int stride_engine_attach(stride_engine_t* engine, const stride_plan_t* plan, int32_t mode,
                         const float* vp, float vp_max, const float* wavelet,
                         const float* observed, float* traces, double* misfit, float* dvp,
                         void* ws, size_t ws_bytes, void* stream, int32_t* slot);

/* Enqueues one chunk of ticks (a power of two, at most max_ticks; shorter
 * only when every slot ends its phase sooner; a slot whose phase ends inside
 * the chunk idles to its end) and the phase-end work of slots that reach it.  *ticks_run is the
 * number of ticks enqueued (0 when no slot is active); finished[slot] is set
 * to 1 (array of max_slots, may be NULL) for slots whose outputs are complete
 * once the stream reaches this point. */
int stride_engine_run(stride_engine_t* engine, int32_t max_ticks, void* stream,
                      int32_t* ticks_run, int32_t* finished);

/* Frees a slot (after it finished, or to abandon it). */
int stride_engine_detach(stride_engine_t* engine, int32_t slot);

/* Ticks a slot still needs (0 once finished). */
int stride_engine_slot_ticks(const stride_engine_t* engine, int32_t slot, int64_t* ticks_left);

/* dst[i] += src[i] on the device (shot-gradient summation in a fixed order). */
int stride_accumulate(float* dst, const float* src, int64_t n, void* stream);

/* Non-finite outputs.  While on for the calling thread (the default), every
 * solve entry point (stride_plan_forward[_static], stride_plan_forward_medium,
 * stride_forward_save, stride_backward, stride_plan_gradient and the one-shot
 * forms) scans what it wrote -- traces, misfit, dvp, dwavelet -- on its stream
 * with a small kernel, waits for the result, and returns STRIDE_E_NONFINITE,
 * naming the outputs, if any value is NaN or infinite (for example from a
 * wavelet or observed data holding one).  The outputs are left as computed.
 * on = 0 turns the scan and its wait off.  Always returns STRIDE_OK. */
int stride_check_finite(int32_t on);

/* Tracing of the time loops.  While enabled on the calling thread, every solve
 * records HIP event pairs on its stream around its forward time loop, its
 * adjoint time loop and each recomputation segment inside the adjoint loop.
 * stride_timing_read waits for the recorded events and returns, since the last
 * read, the time (ms), the time steps and the kernel launches of forward steps
 * (recomputation included) and of adjoint steps (recomputation excluded), then
 * clears them.  Every launch advances one step today; the counts are kept
 * apart so that a launch that advances several steps can be reported.  Any
 * output pointer may be NULL. */
int stride_timing_enable(int32_t on);
int stride_timing_read(double* fwd_ms, int64_t* fwd_steps, int64_t* fwd_launches, double* adj_ms,
                       int64_t* adj_steps, int64_t* adj_launches);

/* Message of the calling thread's last error ("" if none). */
const char* stride_last_error(void);
const char* stride_error_string(int code);

#ifdef __cplusplus
}
#endif
#endif

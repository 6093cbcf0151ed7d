/*
 * ptycho.h - C ABI of the ptychography hot path (far and near field) for
 * AMD MI355X (gfx950).
 *
 * The library implements the data-parallel core of operator-based
 * ptychographic reconstruction as described in Favre-Nicolin et al., "PyNX:
 * high performance computing toolkit for coherent X-ray imaging based on
 * operators" (arXiv 2008.11511), Section 4 and the appendix table of
 * ptychography operators: exit waves (ObjProbe2Psi), far-field propagation
 * (FT / IFT), the modulus constraint (ApplyAmplitude), the object and probe
 * update (Psi2ObjProbe), the AP and DM cycles, the Poisson log-likelihood
 * (LLK) and the conjugate-gradient ML refinement built on its gradient, in
 * the far-field geometry or, with PTYCHO_FLAG_NEAR_FIELD, the near-field one
 * (PropagateNearField in place of FT / IFT).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  - Complex arrays are interleaved single precision (re, im) pairs, passed
 *    as float*; "complex[n]" below means 2*n floats.  All arrays are
 *    row-major and densely packed.
 *  - obj   : complex[obj_ny][obj_nx]          object O
 *    probe : complex[K][N][N]                 probe modes P_k
 *    psi   : complex[J][K][N][N]              exit waves (DM state)
 *    iobs  : float[J][N][N]                   observed counts; far field: FFT
 *                                              order (zero frequency at
 *                                              [0][0]); near field: detector
 *                                              pixels in natural order
 *    mask  : uint8[N][N]                      1 = bad detector pixel, shared
 *                                              by all frames; NULL = none
 *  - The 2D transforms are unitary, forward sign -1.  Near-field
 *    propagation is F^-1 Q F with the Fresnel transfer function Q (see
 *    ptycho_plan_set_near_field), unitary as well.
 *  - Frame j covers obj[oy_j .. oy_j+N-1][ox_j .. ox_j+N-1] with integer
 *    top-left offsets (oy_j, ox_j); exit wave Psi_jk[y][x] =
 *    O[oy_j+y][ox_j+x] * P_k[y][x].
 *  - "dev" pointers are device memory on the plan's device, owned by the
 *    caller; the library never frees them.  "host" pointers are read during
 *    the call only.
 *  - Every GPU entry point enqueues its work on the plan's stream and
 *    returns without synchronising (the paper's asynchronous-execution rule,
 *    Section 2): outputs are valid once the caller synchronises that stream.
 *    A plan must not be used from two host threads at once.  Two plans on
 *    different streams may run concurrently.
 *  - Errors: every function returns a ptycho_status.  Argument, size and
 *    bounds errors are detected on the host before anything is enqueued, so
 *    no state is modified.  A failed kernel launch returns PTYCHO_E_HIP.
 *    ptycho_last_error() gives a message for the calling thread's last
 *    failure.  Nothing throws across this interface.
 */
#ifndef PTYCHO_H
#define PTYCHO_H

#include <stddef.h>
#include <stdint.h>

/* Every entry point is exported with default visibility; the library's
 * internal symbols are hidden. */
#if defined(__GNUC__) || defined(__clang__)
#define PTYCHO_API __attribute__((visibility("default")))
#else
#define PTYCHO_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PTYCHO_OK = 0,
    PTYCHO_E_INVALID = -1,      /* bad argument (null pointer, size, flag)   */
    PTYCHO_E_BOUNDS = -2,       /* a frame window falls outside the object   */
    PTYCHO_E_UNSUPPORTED = -3,  /* N not a supported power of two, K > 4      */
    PTYCHO_E_HIP = -4,          /* HIP runtime / launch error                 */
    PTYCHO_E_WORKSPACE = -5     /* workspace missing, too small or misaligned */
} ptycho_status;

/* Update flags for the cycle entry points. */
#define PTYCHO_UPDATE_OBJECT     1u
#define PTYCHO_UPDATE_PROBE      2u
#define PTYCHO_UPDATE_BACKGROUND 4u   /* AP only; see ptycho_ap_cycle */
#define PTYCHO_UPDATE_POSITIONS  8u   /* AP and ML, plans with PTYCHO_FLAG_POSITIONS */

/* Descriptor flags.  PTYCHO_FLAG_BACKGROUND reserves workspace for the AP
 * background refinement (S*N*N floats and N*N doubles).
 * PTYCHO_FLAG_NEAR_FIELD selects the near-field geometry (2*N complex of
 * workspace for the transfer function); such a plan needs
 * ptycho_plan_set_near_field before any call that propagates. */
#define PTYCHO_FLAG_BACKGROUND 1u
#define PTYCHO_FLAG_NEAR_FIELD 2u
/* PTYCHO_FLAG_POSITIONS: the plan keeps real (sub-pixel) scan positions on
 * the device and refines them (ptycho_plan_set_positions); every frame
 * window may move up to desc->max_shift pixels from its start. */
#define PTYCHO_FLAG_POSITIONS 4u

/* Problem description.  Supported: N a power of two from 8 to 2048,
 * 1 <= K <= 4, J >= 1, obj_ny >= N, obj_nx >= N. */
typedef struct {
    int32_t n;              /* frame side N (power of two)                      */
    int32_t n_modes;        /* incoherent probe modes K                         */
    int32_t n_frames;       /* scan positions J                                 */
    int32_t obj_ny;         /* object rows                                      */
    int32_t obj_nx;         /* object columns                                   */
    int32_t stack;          /* frames per launch; 0 = automatic (the paper's
                               stack of frames, Section 4)                      */
    float obj_inertia;      /* delta_O: alpha_O = delta_O * max(denO)           */
    float probe_inertia;    /* delta_P: alpha_P = delta_P * max(denP)           */
    float icalc_floor;      /* epsilon: calculated intensity floor              */
    uint32_t flags;         /* PTYCHO_FLAG_* (BACKGROUND, NEAR_FIELD, POSITIONS) */
    float max_shift;        /* PTYCHO_FLAG_POSITIONS: largest move of a position
                               from its start, pixels (the paper's
                               update_pos_max_shift); ignored otherwise        */
} ptycho_desc_t;

typedef struct ptycho_plan_s *ptycho_plan_t;

/* Scan positions -> integer window offsets (host only, no GPU work).
 * pos_yx_host: double[J][2], pixels relative to the object centre
 * (obj_ny/2, obj_nx/2).  offsets_out_host: int32[J][2] receives
 * floor(centre + p + 0.5) - N/2 per axis (round half up).  Returns
 * PTYCHO_E_BOUNDS, writing nothing, if any window leaves the object.
 * (Section 4: PtychoData holds the probe translation positions; the exit
 * wave of the ptychography-operator table shifts the probe by r_j.) */
PTYCHO_API int ptycho_offsets_from_positions(const double *pos_yx_host, int32_t n_frames,
                                  int32_t n, int32_t obj_ny, int32_t obj_nx,
                                  int32_t *offsets_out_host);

/* Sub-pixel windows (host only, no GPU work): the real top-left corner
 * t = centre + p - N/2 of each position split into offsets_out_host
 * (int32[J][2], floor(t)) and frac_out_host (double[J][2], t - floor(t) in
 * [0, 1)), pos_yx_host as for ptycho_offsets_from_positions.  A window at a
 * fractional corner views the object by bilinear interpolation (refined
 * positions are real numbers: position optimisation, Section 4).
 * PTYCHO_E_BOUNDS, writing nothing, if a corner is outside
 * [0, obj - N] on either axis. */
PTYCHO_API int ptycho_windows_from_positions(const double *pos_yx_host, int32_t n_frames, int32_t n,
                                             int32_t obj_ny, int32_t obj_nx, int32_t *offsets_out_host,
                                             double *frac_out_host);

/* Device workspace needed by a plan for `desc`, in bytes (host only).
 * Section 4: operators compute a stack of frames of the Psi array at once
 * and loop over the stacks to cover every frame (the paper's stacks hold 16
 * to 128 frames, larger ones being faster); the workspace holds that stack
 * (desc->stack frames, 0 = the largest whose scratch fits 32 GiB), the
 * plan's index tables, the overlap-update sums and the reduction partials.
 * PTYCHO_E_INVALID / PTYCHO_E_UNSUPPORTED for a bad descriptor. */
PTYCHO_API int ptycho_workspace_bytes(const ptycho_desc_t *desc, size_t *bytes_out);

/* Create a plan: the scan's data object of Section 4 (PtychoData: observed
 * intensity, probe positions, bad-pixel mask, near or far field) with the
 * stack of exit waves (the Psi array of the Ptycho object) placed in the
 * caller's workspace.  offsets_host: int32[J][2] window offsets (checked
 * against the object bounds, PTYCHO_E_BOUNDS otherwise).  iobs_dev /
 * mask_dev: observed data and bad-pixel mask (mask may be NULL); the plan
 * keeps these pointers, which must stay valid for the plan's life.  workspace_dev: at least ptycho_workspace_bytes()
 * bytes, 256-byte aligned, owned by the caller, used exclusively by this
 * plan.  stream: a hipStream_t (NULL = default stream).  The call enqueues
 * the upload of the index tables (the plan keeps their host copies) and the
 * count of unmasked pixels on `stream`, returns the handle in *out, and does
 * not wait for the stream; later calls on the plan's stream see the tables. */
PTYCHO_API int ptycho_plan(const ptycho_desc_t *desc, const int32_t *offsets_host,
                const float *iobs_dev, const uint8_t *mask_dev,
                void *workspace_dev, size_t workspace_bytes,
                void *stream, ptycho_plan_t *out);

/* Build and check a plan's host-side index tables (frame order, object-gather
 * lists) for `desc` and offsets_host without any GPU work; *table_bytes_out
 * receives their size.  Same checks and status codes as ptycho_plan
 * (without the device pointers); for capacity planning and tests (the
 * index tables of the stacks of Section 4 that ptycho_plan builds). */
PTYCHO_API int ptycho_plan_dry_run(const ptycho_desc_t *desc, const int32_t *offsets_host,
                        size_t *table_bytes_out);

/* Near-field geometry (Section 4: near and far-field geometries; operator
 * PropagateNearField of the ptychography-operator table, which the paper
 * names without a formula).  Reading: the paraxial Fresnel transfer
 * function, Q[u][v] = exp(-i (fy u'^2 + fx v'^2)) on the DFT grid with
 * u' = u for u < N/2 else u - N, i.e. exp(-i pi lambda z |q|^2) with the
 * constant phase exp(ikz) dropped: fy = pi lambda z / (N dy)^2 and
 * fx = pi lambda z / (N dx)^2 for pixel sizes dy, dx (a magnified geometry
 * enters through its effective distance).  Every operator of the plan then
 * propagates with D = F^-1 Q F (sample to detector) and its inverse
 * F^-1 conj(Q) F, and takes iobs and mask in natural pixel order.  The plan
 * must have been created with PTYCHO_FLAG_NEAR_FIELD (PTYCHO_E_INVALID
 * otherwise, and for non-finite parameters).  The table Q/N is computed on
 * the host in double precision and uploaded on the plan's stream without
 * waiting; calls may change it between cycles (e.g. another distance). */
PTYCHO_API int ptycho_plan_set_near_field(ptycho_plan_t plan, double fy, double fx);

/* Incoherent background (Section 4: the Ptycho object carries one beside the
 * object and probe estimates): bg_dev float[N][N] in the detector layout of iobs, shared by
 * all frames, caller-owned, NULL = none.  Every operator then models the
 * intensity as I = sum_k |FT(O_j P_k)|^2 + bg: the modulus projection (the
 * background is scaled like one more incoherent mode), LLK, icalc, the ML
 * gradient and line search.  ptycho_ap_cycle with PTYCHO_UPDATE_BACKGROUND
 * refines it in place: bg <- bg * (1/J) sum_j s_j^2, s_j^2 = Iobs / I at
 * frame j (1 at bad pixels), from the projection of that cycle (the
 * augmented projections the paper cites for AP background optimisation). */
PTYCHO_API int ptycho_plan_set_background(ptycho_plan_t plan, float *bg_dev);

/* Position refinement (operator Psi2PosShift, Section 4, after Odstrcil et
 * al. 2018): for every frame j, the shift d of its illumination position
 * that best explains the exit waves psi_dev (complex[J][K][N][N], e.g. the
 * projected ones an AP cycle leaves) against the current views:
 *   chi = Psi_jk - P_k O_j ~ d_y P_k dO/dy + d_x P_k dO/dx,
 * the two components solved together by least squares over the frame's
 * pixels and modes (d = 0 if the 2x2 system is singular), the gradient by
 * centred differences on the object (one-sided on its border).
 * out_dev: double[J][3] device, per frame (d_y, d_x, gradient energy
 * S_yy + S_xx) in pixels, frames in scan order.  The caller moves the
 * positions (the paper's filter leaves frames of low gradient energy in
 * place) and builds a plan from the new offsets.  probe_dev and psi_dev must
 * be 16-byte aligned (PTYCHO_E_INVALID otherwise; torch allocations are). */
PTYCHO_API int ptycho_position_shifts(ptycho_plan_t plan, const float *obj_dev, const float *probe_dev,
                           const float *psi_dev, double *out_dev);

/* Position update of the refinement (Section 4: position optimisation
 * during AP and ML after Odstrcil et al. 2018, with a filter that keeps
 * frames of too little object contrast in place).  For every frame j and
 * axis, with e_j the gradient energy and d_j the shift from
 * ptycho_position_shifts (shifts_dev, double[J][3] device):
 *   keep_j = e_j >= min_grad * median_j(e_j)
 *   p'_j   = pos_j + mult * (keep_j ? d_j : 0)
 *   out_j  = pos0_j + clamp(p'_j - pos0_j, -max_shift, max_shift)
 * (the paper's update_pos_mult and update_pos_max_shift; the median of an
 * even count is the mean of the two middle values; gradient energies must
 * be finite).  pos_dev, pos0_dev (starting positions), pos_out_dev:
 * double[J][2] device, in pixels; pos_out_dev may equal pos_dev.  Enqueued
 * on `stream` (hipStream_t), no plan and no workspace; the caller turns the
 * new positions into offsets (ptycho_offsets_from_positions) and a plan.
 * PTYCHO_E_INVALID for n_frames < 1, null pointers, non-finite parameters or
 * negative max_shift / min_grad. */
PTYCHO_API int ptycho_update_positions(int32_t n_frames, const double *pos_dev, const double *pos0_dev,
                                       const double *shifts_dev, double mult, double max_shift,
                                       double min_grad, double *pos_out_dev, void *stream);

/* Real scan positions of a plan created with PTYCHO_FLAG_POSITIONS (Section 4:
 * position optimisation during AP and ML, after Odstrcil et al. 2018).
 * pos_yx_host: double[J][2] as for ptycho_offsets_from_positions; the plan's
 * offsets must be their windows' integer corners
 * (ptycho_windows_from_positions), else PTYCHO_E_INVALID; every corner must
 * stay inside the object when moved by up to desc->max_shift on each axis,
 * else PTYCHO_E_BOUNDS.  These become the start and the current positions;
 * from then on every operator of the plan views the object through
 * sub-pixel windows (bilinear interpolation, the object sums through its
 * adjoint).  mult and min_grad are the step factor and low-contrast filter
 * of the position updates (see ptycho_update_positions; finite, min_grad
 * >= 0).  The tables are uploaded on the plan's stream without waiting. */
PTYCHO_API int ptycho_plan_set_positions(ptycho_plan_t plan, const double *pos_yx_host, double mult,
                                         double min_grad);

/* Current positions of a PTYCHO_FLAG_POSITIONS plan into pos_yx_dev
 * (double[J][2] device, pixels from the object centre), enqueued. */
PTYCHO_API int ptycho_plan_positions(ptycho_plan_t plan, double *pos_yx_dev);

/* One position-refinement step of a plan with positions set: the shifts of
 * every frame from the exit waves psi_dev (complex[J][K][N][N], e.g. the
 * projected ones an AP cycle leaves) against the plan's current windows, as
 * ptycho_position_shifts, then the update of ptycho_update_positions with
 * the plan's start positions, max_shift, mult and min_grad, and the new
 * windows: all on the device, enqueued.  shifts_dev (nullable,
 * double[J][3]) receives the shifts.  ptycho_ap_cycle and ptycho_ml_cycle
 * do the same every cycle with PTYCHO_UPDATE_POSITIONS.  As for
 * ptycho_position_shifts, probe_dev and psi_dev must be 16-byte aligned
 * (also in those cycles). */
PTYCHO_API int ptycho_refine_positions(ptycho_plan_t plan, const float *obj_dev, const float *probe_dev,
                                       const float *psi_dev, double *shifts_dev);

/* Failure detection: flag_dev (int32[1], device) is set to 1 if any value
 * of the object or probe is NaN or infinite, else 0 (enqueued, so a caller
 * can copy the flag back and read it at its next poll without waiting). */
PTYCHO_API int ptycho_check_finite(ptycho_plan_t plan, const float *obj_dev, const float *probe_dev,
                        int32_t *flag_dev);

/* Change the stream later calls enqueue on (hipStream_t); the paper's
 * asynchronous execution (Section 2) queues every operator on one stream. */
PTYCHO_API int ptycho_plan_set_stream(ptycho_plan_t plan, void *stream);

/* Frames per launch actually used by the plan (the stack size of Section 4). */
PTYCHO_API int ptycho_plan_stack(ptycho_plan_t plan, int32_t *stack_out);

/* Free the host-side plan (the data object of Section 4 whose device arrays
 * belong to the caller).  Device buffers, including the workspace, are
 * untouched; work already enqueued must complete before the caller frees
 * them.  A null plan is accepted. */
PTYCHO_API int ptycho_plan_destroy(ptycho_plan_t plan);

/* n_cycles alternating-projection cycles (operator AP): for every frame and
 * mode Psi = IFT * ApplyAmplitude * FT (O_j P_k); then the overlap update
 * (Psi2ObjProbe) from all frames, object first, then the probe from the new
 * object, each with inertia alpha = delta * max(den):
 *   O <- (sum_jk conj(P_k) Psi_jk + alpha_O O) / (sum_jk |P_k|^2 + alpha_O)
 *   P_k <- (sum_j conj(O_j) Psi_jk + alpha_P P_k) / (sum_j |O_j|^2 + alpha_P)
 * (pixels with a zero denominator keep their value).
 * update: PTYCHO_UPDATE_OBJECT | PTYCHO_UPDATE_PROBE, and
 * PTYCHO_UPDATE_BACKGROUND to refine the background set with
 * ptycho_plan_set_background (the plan must have PTYCHO_FLAG_BACKGROUND;
 * PTYCHO_E_INVALID otherwise), PTYCHO_UPDATE_POSITIONS to refine the
 * positions after each cycle's object and probe update, from the projected
 * exit waves (ptycho_refine_positions; a plan with positions set, and psi
 * needed).  obj, probe: in/out.
 * psi_dev: complex[J][K][N][N] storage for the projected exit waves, needed
 * (PTYCHO_E_INVALID otherwise) when the probe is updated, since the probe
 * update runs after the object update over all frames; may be NULL for an
 * object-only update.  On return it holds the last cycle's exit waves. */
PTYCHO_API int ptycho_ap_cycle(ptycho_plan_t plan, float *obj_dev, float *probe_dev,
                    float *psi_dev, int32_t n_cycles, uint32_t update);

/* n_cycles difference-map cycles (operator DM, beta = 1) on the persistent
 * exit waves psi (in/out, complex[J][K][N][N]):
 *   Psi <- Psi + IFT ApplyAmplitude FT (2 Phi - Psi) - Phi,  Phi = O_j P_k
 * followed by the overlap update of obj / probe as in ptycho_ap_cycle
 * (object, then probe from the new object). */
PTYCHO_API int ptycho_dm_cycle(ptycho_plan_t plan, float *obj_dev, float *probe_dev,
                    float *psi_dev, int32_t n_cycles, uint32_t update);

/* psi <- O_j P_k for every frame and mode: operator ObjProbe2Psi of the
 * ptychography-operator table (the views of Section 4's Psi array), the
 * DM starting point.  psi_dev: complex[J][K][N][N], caller-owned. */
PTYCHO_API int ptycho_psi_init(ptycho_plan_t plan, const float *obj_dev,
                    const float *probe_dev, float *psi_dev);

/* Poisson log-likelihood (operator LLK): llk_dev (double[2], device)
 * receives { sum over unmasked pixels of all frames of
 * I - Iobs + Iobs ln(Iobs / I), number of those pixels }, with
 * I = sum_k |FT(O_j P_k)|^2 floored at icalc_floor, 0 ln 0 = 0. */
PTYCHO_API int ptycho_llk(ptycho_plan_t plan, const float *obj_dev, const float *probe_dev,
               double *llk_dev);

/* Noise models for reporting the likelihood (Section 4 lists Poisson,
 * Gaussian and Euclidian models, after Thibault & Guizar-Sicairos 2012).
 * Each term is the negative log-density difference to a perfect fit. */
typedef enum {
    PTYCHO_LLK_POISSON = 0,     /* I - Iobs + Iobs ln(Iobs / I)                */
    PTYCHO_LLK_GAUSSIAN = 1,    /* (I - Iobs)^2 / (2 (Iobs + 1))               */
    PTYCHO_LLK_EUCLIDEAN = 2    /* 2 (sqrt(I) - sqrt(Iobs))^2 (amplitudes)     */
} ptycho_llk_model_t;

/* As ptycho_llk with the terms of `model` (a ptycho_llk_model_t); an unknown
 * model is PTYCHO_E_INVALID.  llk_dev: double[2] device, as ptycho_llk. */
PTYCHO_API int ptycho_llk_model(ptycho_plan_t plan, const float *obj_dev,
                     const float *probe_dev, int32_t model, double *llk_dev);

/* Gradient of that LLK (maximum-likelihood operator ML):
 * g = dL/dRe + i dL/dIm, i.e. with psi_jk = IFT((1 - Iobs/I) FT(O_j P_k))
 * (zero at bad pixels):
 *   g_obj   = 2 sum_jk S_j^T (conj(P_k) psi_jk)       complex[obj_ny][obj_nx]
 *   g_probe = 2 sum_j conj(O_j) psi_jk                 complex[K][N][N]
 * llk_dev (nullable, double[2]) receives the LLK as ptycho_llk. */
PTYCHO_API int ptycho_ml_grad(ptycho_plan_t plan, const float *obj_dev,
                   const float *probe_dev, float *g_obj_dev,
                   float *g_probe_dev, double *llk_dev);

/* Line-search coefficients along (d_obj, d_probe): coef_dev (double[2],
 * device) receives { L'(0), L''(0) } of L(g) = LLK(O + g dO, P + g dP), with
 * L'' from the quadratic expansion of the intensity in g.  This is the step
 * of operator ML (Section 4 algorithm list and the ptychography-operator
 * table: conjugate gradient on the Poisson likelihood, after Thibault and
 * Guizar-Sicairos 2012), whose quadratic line search it follows. */
PTYCHO_API int ptycho_ml_linesearch(ptycho_plan_t plan, const float *obj_dev,
                         const float *probe_dev, const float *d_obj_dev,
                         const float *d_probe_dev, double *coef_dev);

/* Device state of the conjugate-gradient ML iteration (operator ML, Section
 * 4: search direction, previous gradient and scalars), in bytes, for
 * ptycho_ml_cycle (host only). */
PTYCHO_API int ptycho_ml_state_bytes(ptycho_plan_t plan, size_t *bytes_out);

/* n_cycles Polak-Ribiere conjugate-gradient ML cycles on the Poisson LLK,
 * entirely on the device (no host synchronisation): gradient, preconditioned
 * direction (probe block scaled by max(denO)/max(denP)), quadratic line
 * search, step.  state_dev: ptycho_ml_state_bytes() bytes, 256-byte aligned;
 * reset != 0 starts a new conjugate sequence (beta = 0).  llk_hist_dev
 * (nullable, double[n_cycles]) receives the LLK at the start of each cycle.
 * update may add PTYCHO_UPDATE_POSITIONS (a plan with positions set): each
 * cycle's gradient pass also takes the position shifts, with minus half the
 * back-propagated gradient wave as the exit-wave change (the AP correction
 * to first order near the fit), at the cycle's start point, and the
 * positions move after the step. */
PTYCHO_API int ptycho_ml_cycle(ptycho_plan_t plan, float *obj_dev, float *probe_dev,
                    void *state_dev, int32_t n_cycles, uint32_t update,
                    int32_t reset, double *llk_hist_dev);

/* Allocation-free Poisson LLK, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * allocation): ptycho_llk of one far-field scan without a plan or a
 * workspace.  Its scratch (frame tables, the stack of transformed frames,
 * reduction partials) lives in a static device array of
 * PTYCHO_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until
 * the process ends; the call allocates nothing.  desc: as for ptycho_plan,
 * flags must be 0 (PTYCHO_E_INVALID otherwise); desc->stack is ignored, the
 * stack is as many frames as fit the scratch; a problem whose frame
 * (K*N*N complex) or tables do not fit is PTYCHO_E_WORKSPACE.
 * offsets_dev: int32[J][2] device, top-left window corners; a window
 * outside the object is clamped to it and llk_dev[0] receives NaN.
 * iobs_dev, mask_dev (NULL = none), obj_dev, probe_dev: as for ptycho_plan
 * and ptycho_llk.  llk_dev: double[2] device, { LLK sum, unmasked pixels }.
 * Enqueued on `stream` (hipStream_t).  Every call on one GPU shares that
 * GPU's scratch: calls that overlap on one GPU (different streams, or
 * threads) race and must be serialised by the caller. */
#define PTYCHO_NOALLOC_SCRATCH_BYTES (64u << 20)
PTYCHO_API int ptycho_llk_noalloc(const ptycho_desc_t *desc, const int32_t *offsets_dev, const float *iobs_dev,
                                  const uint8_t *mask_dev, const float *obj_dev, const float *probe_dev,
                                  double *llk_dev, void *stream);

/* Calculated intensity sum_k |FT(O_j P_k)|^2 of every frame into
 * icalc_dev (float[J][N][N], FFT order); the forward model used to simulate
 * data. */
PTYCHO_API int ptycho_icalc(ptycho_plan_t plan, const float *obj_dev,
                 const float *probe_dev, float *icalc_dev);

/* Batched unitary 2D FFT of `count` complex N x N frames in place
 * (direction -1 forward, +1 inverse), exposed for tests and the FFT
 * bandwidth benchmark of the paper's appendix (FFT performance). */
PTYCHO_API int ptycho_fft2(int32_t n, int32_t count, float *data_dev, int32_t direction,
                void *stream);

/* Per-kernel timing for diagnostics and benchmarks: `classes` is a bit mask
 * of kernel classes (bit c for class c: 0 forward row FFTs, 1 column FFT +
 * Fourier-space step, 2 inverse row FFTs, 3 object gather, 4 per-stack probe
 * gather, 5 all-frame probe gather, 6 normalisation, 7 other; 255 = all).
 * With classes != 0 the plan records a HIP event pair on its stream around
 * every later launch of the selected classes (each pair adds a few
 * microseconds to the stream, so time a whole run with few classes);
 * 0 stops recording.  PTYCHO_E_INVALID for bits beyond class 7.
 * ptycho_plan_timing_read waits for the last recorded event and returns the
 * summed milliseconds and the launch count of one class since timing was
 * last enabled. */
PTYCHO_API int ptycho_plan_timing(ptycho_plan_t plan, int32_t classes);
PTYCHO_API int ptycho_plan_timing_read(ptycho_plan_t plan, int32_t cls, double *ms_total,
                            int64_t *launches);

/* Message for the calling thread's last non-OK status ("" if none). */
PTYCHO_API const char *ptycho_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PTYCHO_H */

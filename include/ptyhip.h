/*
 * ptyhip — the data-parallel hot path of gradient-based ptychographic reconstruction
 * (arxiv 2510.20929, "Pty-Chi") on AMD MI355X (gfx950): the batched far-field forward
 * model and its exact adjoint, behind a plain C ABI.
 *
 * What the library computes (Sec. 2.1 forward model; Eq. (1); Eq. (2); Eq. (4)):
 *   for each scan position k and probe mode m
 *     o_k      = bilinear patch of the object at position r_k          (patch extraction)
 *     P_{k,m}  = sum_e w_{k,e} U_{e,m}                                 (scan-point probes, OPR)
 *     psi      = P_{k,m} * o_k, propagated through the slices          (exit wave; multislice)
 *     Psi      = unitary 2D DFT of the last exit wave                  (far-field propagation)
 *     I_k      = sum_m |Psi_{k,m}|^2                                   (incoherent modes)
 *   L = sum_k sum_px l(I_k, I_meas_k) / (K_norm N^2), l = (sqrt(I) - sqrt(I_meas))^2
 *   (Eq. (1)) or l = I - I_meas ln(I + eps) (Poisson), and the gradients of L with
 *   respect to the object, the probe (eigenprobes), the positions and the OPR weights.
 *
 * Conventions (each is a reading of a point the paper leaves open):
 *   - complex arrays are interleaved (re, im) float32 pairs ("complex64"), row-major;
 *   - the DFT is unitary with kernel exp(-2 pi i k.n / N);
 *   - measured and predicted intensities are DC-centred (fftshift layout) in the far field
 *     and in natural pixel order in the near field;
 *   - a position (y, x) is the frame's top-left corner in object pixels; the integer
 *     part is the floor, the fraction drives bilinear interpolation; the window is
 *     N x N, one row/column wider when the fraction is non-zero or position gradients
 *     are requested;
 *   - gradients are g = dL/dRe z + i dL/dIm z (the torch convention; twice Eq. (2));
 *   - multislice: transmit then propagate by exp(-i pi lambda_z (fy^2 + fx^2)), S - 1
 *     propagations, the last exit wave goes to the far field.
 *
 * Memory and ownership: every array argument of a call is a DEVICE pointer owned by
 * the caller; the library never frees or retains it beyond the call. A plan owns its
 * workspace (allocated once in ptyhip_plan_create, freed in ptyhip_plan_destroy);
 * calls allocate nothing. Calls are asynchronous on `stream` (a hipStream_t, or NULL
 * for the default stream). A plan is not re-entrant: one call in flight per plan.
 *
 * Errors: host-detectable problems (NULL pointers, bad shapes, K > max_positions,
 * unsupported sizes) return a status and launch nothing. Problems only the device can
 * see (a scan window leaving the object, non-finite inputs) set bits of a latched flag
 * word in the plan; the offending position contributes nothing. Read it with
 * ptyhip_get_error.
 */
#ifndef PTYHIP_H
#define PTYHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PTYHIP_OK = 0,
  PTYHIP_EINVAL = 1,       /* NULL pointer or invalid argument value */
  PTYHIP_ESHAPE = 2,       /* inconsistent sizes */
  PTYHIP_EBOUNDS = 3,      /* K outside [0, max_positions] */
  PTYHIP_ENONFINITE = 4,   /* non-finite scalar parameter */
  PTYHIP_EHIP = 5,         /* a HIP runtime call failed */
  PTYHIP_ENOMEM = 6,       /* workspace allocation failed */
  PTYHIP_EUNSUPPORTED = 7  /* size or option the library does not support */
} ptyhip_status;

typedef enum {
  PTYHIP_LOSS_AMPLITUDE = 0, /* Gaussian magnitude loss, Eq. (1) */
  PTYHIP_LOSS_POISSON = 1    /* l = I - I_meas ln(I + eps) (the paper names no formula) */
} ptyhip_loss;

/* flags of ptyhip_forward_adjoint / ptyhip_batch_launch */
enum {
  PTYHIP_GRAD_OBJ = 1,      /* object gradient               [S][H][W] complex */
  PTYHIP_GRAD_PROBE = 2,    /* probe / eigenprobe gradient   [E][M][N][N] complex */
  PTYHIP_GRAD_POS = 4,      /* position gradient             [K][2] float */
  PTYHIP_GRAD_WEIGHTS = 8,  /* OPR weight gradient           [K][E] float */
  PTYHIP_ACCUMULATE = 16,   /* add into the outputs (and loss) instead of overwriting */
  PTYHIP_PLAIN = 32,        /* run the per-step kernels instead of the fused kernel */
  PTYHIP_BATCH_PER_CALL = 64, /* batch only: one non-captured fused call per dataset */
  PTYHIP_GRAD_LAMBDA_Z = 128  /* dL/d(lambda z) of the plan's Fresnel propagator, device double[1]:
                                 det_lambda_z (near field) or the slice spacing lambda_z
                                 (several slices); fused form only */
};

/* sub-pixel patch model (Software design, Overview: patch extraction is a shared routine;
 * the paper names no interpolation) */
typedef enum {
  PTYHIP_SUBPIXEL_BILINEAR = 0, /* bilinear taps over the (N+1)^2 window */
  PTYHIP_SUBPIXEL_FOURIER = 1   /* o = F^-1(exp(2 pi i (ky fy + kx fx) / N) F window), window at the
                                   integer corner, periodic within the window */
} ptyhip_subpixel;

/* propagation to the detector */
typedef enum {
  PTYHIP_PROP_FAR = 0, /* far field: unitary 2D DFT, DC-centred detector */
  PTYHIP_PROP_NEAR = 1 /* near field: Fresnel propagation F^-1 H F, natural pixel order */
} ptyhip_propagation;

/* bits of the device error latch */
enum { PTYHIP_FLAG_BOUNDS = 1, PTYHIP_FLAG_NONFINITE = 2 };

/* Problem description. Sizes: N = frame, M = n_modes, E = n_eig, S = n_slices,
 * object H x W per slice. */
typedef struct {
  int32_t frame;        /* N: 16, 32, 64, 128, 256 or 512 */
  int32_t n_modes;      /* M: 1..64 incoherent probe modes (Sec. 2.1) */
  int32_t n_eig;        /* E: 1..16 eigenprobes (OPR, Sec. 2.1); 1 = none */
  int32_t n_slices;     /* S: 1..64 multislice slices (Sec. 2.1); multislice plans of 256^2 and
                           512^2 frames run the per-step form (no PTYHIP_GRAD_LAMBDA_Z there) */
  int32_t obj_h, obj_w; /* object size per slice, >= N each, <= 2^20 each, at most 4e9 pixels
                           over all slices; for N >= 256 also (N + 1) * obj_w * 8 < 2^31
                           (byte span of a patch window); otherwise PTYHIP_ESHAPE */
  int32_t loss;         /* ptyhip_loss */
  float poisson_eps;    /* eps of the Poisson loss, photons (>= 0) */
  float lambda_z;       /* slice spacing times wavelength, px^2 (used when S > 1) */
  double norm_count;    /* K_norm of the 1/(K_norm N^2) normaliser; <= 0: K of the call */
  int32_t propagation;  /* a ptyhip_propagation value: far- or near-field propagation in the
                           forward model (Software design, Overview); near needs S == 1; near
                           fields of 256^2 and 512^2 frames run the per-step form (no
                           PTYHIP_GRAD_LAMBDA_Z there) */
  float det_lambda_z;   /* near field: wavelength times detector distance, px^2; the detector
                           wave is F^-1(exp(-i pi det_lambda_z (fy^2 + fx^2)) F chi) */
  int32_t subpixel;     /* a ptyhip_subpixel value: bilinear interpolation (default) or the
                           Fourier shift of the integer N x N window; Fourier needs S == 1
                           and the far field; Fourier-shift plans of 256^2 and 512^2 frames
                           run the per-step form */
} ptyhip_desc;

/* Optional implementation choices (the autotuner's search space). Zero = default. */
typedef struct {
  int32_t variant;      /* on-chip fused kernel (64^2, 128^2): 0 = 512 threads, patch in scratch;
                           1 = 1024 (128^2) / 256 (64^2) threads; 2 = 512 threads, patch and
                           patch gradient in registers; 3 = as 2 with 1024 / 256 threads;
                           4 = as 3 with the patch gradient in scratch; 128^2 only, one slice,
                           far field, bilinear patch, whole positions (PTYHIP_EUNSUPPORTED
                           otherwise): 5 = 1024 threads with the working frame resident in
                           LDS, patch and running patch gradient in registers, dl/dI in
                           scratch, far fields always recomputed; 6 = as 5 with dl/dI in
                           registers.
                           Four-step fused kernel (256^2, 512^2): 0 = one workgroup of 1024
                           threads per CU; 1 = two per CU (512 / 256 threads, smaller line
                           blocks); other values are PTYHIP_EINVAL */
  int32_t grid;         /* persistent workgroups; 0 = occupancy x compute units */
  int32_t recompute;    /* 1 = recompute (multislice: incident waves; several modes: far fields)
                           instead of keeping them in workgroup scratch */
  int32_t plain_chunk;  /* positions per chunk of the per-step path; 0 = auto */
  int32_t mode_groups;  /* 0 or 1: a workgroup takes whole positions; G > 1 (one slice, far field,
                           bilinear patch, any frame size): the modes of every position are split
                           into at most G groups, each (position, group) a work item of its own, in
                           three passes (partial intensities, loss, adjoint), so that calls with
                           few positions keep more workgroups busy; G is capped at the mode count;
                           forward and forward + adjoint calls only (the linear maps keep whole
                           positions). Other models: PTYHIP_EUNSUPPORTED */
  int32_t probe_stage;  /* 0: probe gradients staged per position only with several eigenprobes (or
                           mode groups), else accumulated in each workgroup's scratch frames;
                           1: always staged (each position writes its probe-wave gradients once,
                           a separate pass adds them), one slice only */
} ptyhip_tune;

typedef struct {
  size_t workspace_bytes;  /* device memory owned by the plan */
  size_t scratch_bytes;    /* of which per-workgroup scratch of the fused kernel */
  size_t window_bytes;     /* of which per-position window gradients of the fused form */
  size_t plain_bytes;      /* of which per-step path buffers */
  int32_t grid;            /* fused kernel workgroups */
  int32_t threads;         /* fused kernel threads per workgroup */
  int32_t fused_on_chip;   /* 1 if the frame stays on chip in the fused kernel */
  int32_t plain_chunk;     /* positions per chunk of the per-step path */
} ptyhip_plan_info;

typedef struct ptyhip_plan_s* ptyhip_plan;
typedef struct ptyhip_batch_s* ptyhip_batch;

const char* ptyhip_status_str(ptyhip_status s);
const char* ptyhip_version(void);

/* Pure host check of a description; no GPU needed. */
ptyhip_status ptyhip_desc_validate(const ptyhip_desc* desc);

/* Create a plan: one problem shape of the image-formation map I = F(o, p, Lambda) of
 * Eq. (4) (frame size, incoherent modes, OPR eigenprobes and slices as in Sec. 2.1,
 * Software design / Overview), for up to max_positions scan positions per call, on the
 * current device. tune may be NULL (defaults). The plan allocates its whole workspace
 * here (twiddle and propagator tables, per-position partial sums, per-workgroup scratch,
 * window-gradient buffer, per-step buffers); it owns that memory until
 * ptyhip_plan_destroy. Errors: EINVAL for a NULL out or a bad tune value, the
 * ptyhip_desc_validate statuses, EBOUNDS for max_positions < 0, EHIP / ENOMEM when a
 * device query or allocation fails. *out is NULL on any failure. */
ptyhip_status ptyhip_plan_create(const ptyhip_desc* desc, int32_t max_positions, ptyhip_plan* out);
ptyhip_status ptyhip_plan_create_ex(const ptyhip_desc* desc, int32_t max_positions, const ptyhip_tune* tune,
                                    ptyhip_plan* out);
void ptyhip_plan_destroy(ptyhip_plan plan);
ptyhip_status ptyhip_plan_get_info(ptyhip_plan plan, ptyhip_plan_info* info);

/* Forward model and loss (Eq. (1) / Poisson) for K positions.
 *   obj       [S][H][W] complex      probe   [E][M][N][N] complex
 *   weights   [K][E] float or NULL (NULL requires E == 1 and means w = 1)
 *   positions [K][2] float (y, x)    I_meas  [K][N][N] float, DC-centred (near field: natural order)
 *   loss      device double[1] (written, or added to with PTYHIP_ACCUMULATE)
 *   I_pred    [K][N][N] float, same layout as I_meas, or NULL */
ptyhip_status ptyhip_forward(ptyhip_plan plan, void* stream, int32_t K, const float* obj, const float* probe,
                             const float* weights, const float* positions, const float* I_meas, double* loss,
                             float* I_pred);

/* Forward model, loss and the gradients selected by `flags` (Eq. (2) extended to every
 * parameter by the chain rule). Gradient outputs not requested may be NULL:
 *   g_obj [S][H][W] complex, g_probe [E][M][N][N] complex, g_pos [K][2], g_weights [K][E].
 * Outputs are overwritten unless PTYHIP_ACCUMULATE is set. I_pred may be NULL. */
ptyhip_status ptyhip_forward_adjoint(ptyhip_plan plan, void* stream, int32_t K, uint32_t flags, const float* obj,
                                     const float* probe, const float* weights, const float* positions,
                                     const float* I_meas, double* loss, float* I_pred, float* g_obj,
                                     float* g_probe, float* g_pos, float* g_weights);

/* As ptyhip_forward_adjoint, plus (PTYHIP_GRAD_LAMBDA_Z) the gradient with respect to the
 * wavelength-distance product of the plan's Fresnel propagator H = exp(-i pi lz (fy^2 +
 * fx^2)), by the chain rule through the propagator, in g_lambda_z (device double[1],
 * overwritten or accumulated like the loss):
 *   - near-field plan: lz = det_lambda_z (Software design, Overview: the near-field
 *     propagation option), dL/dlz = sum_k,m Re sum_f conj(F g_Psi) (-i pi q^2) H F chi;
 *   - multislice plan (S > 1): lz = the slice spacing lambda_z (Sec. 2.1 multislice; the
 *     automatic-differentiation reconstructor refines the slice spacing, Reconstructors),
 *     dL/dlz = sum_k,m sum_{s>0} Re sum_f conj(F g_psi_s) (-i pi q^2) F psi_s, with
 *     psi_s the incident wave of slice s and g_psi_s its gradient.
 * The flag with a single-slice far-field plan, or with a NULL g_lambda_z, is EINVAL;
 * with PTYHIP_PLAIN, or with a near-field plan of frames above 128^2 (which runs the
 * per-step form), it is EUNSUPPORTED (the fused kernels compute it). */
ptyhip_status ptyhip_forward_adjoint_ex(ptyhip_plan plan, void* stream, int32_t K, uint32_t flags, const float* obj,
                                        const float* probe, const float* weights, const float* positions,
                                        const float* I_meas, double* loss, float* I_pred, float* g_obj,
                                        float* g_probe, float* g_pos, float* g_weights, double* g_lambda_z);

/* The linear map (object, probe) -> far-field waves Psi [K][M][N][N] (unshifted):
 * Eq. (4) before the modulus, i.e. the exit waves of Sec. 2.1 (patch extraction, probe
 * times patch, multislice propagation) carried to the far field by the unitary DFT,
 * with the object linear for a fixed probe and the probe linear for a fixed object;
 * and its adjoint (for the identity <A x, y> = <x, A^H y>): apply_AH takes Y [K][M][N][N]
 * and returns, per slice, the adjoint of O_s -> Psi (other slices and probe fixed) in
 * g_obj and the adjoint of U -> Psi (object fixed) in g_probe (either may be NULL). */
ptyhip_status ptyhip_apply_A(ptyhip_plan plan, void* stream, int32_t K, const float* obj, const float* probe,
                             const float* weights, const float* positions, float* Psi);
ptyhip_status ptyhip_apply_AH(ptyhip_plan plan, void* stream, int32_t K, const float* Y, const float* obj,
                              const float* probe, const float* weights, const float* positions, float* g_obj,
                              float* g_probe);

/* Illumination map in the object frame: the probe intensity of every scan position
 * superimposed where it falls, illum[y][x] = sum_k S_k^T (sum_m |P_k,m|^2), with S_k^T
 * the transpose of the bilinear patch extraction (the scatter used for the object
 * gradient) and P_k,m = sum_e w_k,e U_e,m. This is the object preconditioner of the
 * least-squares reconstructor (Introduction: the illumination superimposed in the
 * object frame; Performance benchmarking: the cost of building it).
 *   probe [E][M][N][N] complex, weights [K][E] or NULL (E == 1), positions [K][2]
 *   illum [H][W] float, overwritten, or added to with PTYHIP_ACCUMULATE (the only flag)
 * Positions whose window leaves the object contribute nothing and set the error
 * latch, as in ptyhip_forward_adjoint. */
ptyhip_status ptyhip_illumination(ptyhip_plan plan, void* stream, int32_t K, uint32_t flags, const float* probe,
                                  const float* weights, const float* positions, float* illum);

/* Scale-normalised gradients (Reconstructors: the ePIE-style treatment of the gradient
 * after Eq. (2)): g_obj *= K_norm N^2 / max_{k,p} sum_m |P_k,m(p)|^2 and, read the same
 * way for the probe, g_probe *= K_norm N^2 / max |O|^2 (over every object pixel).
 * K_norm is the plan's norm_count, or K when that is <= 0. Either gradient may be NULL
 * (then it is left alone); K >= 1. The maxima are computed on the device; a zero
 * maximum leaves the gradient unchanged. In place, asynchronous on `stream`. */
ptyhip_status ptyhip_normalize_gradients(ptyhip_plan plan, void* stream, int32_t K, const float* probe,
                                         const float* weights, const float* obj, float* g_obj, float* g_probe);

/* Probe-mode orthogonalisation, one of the parameter routines shared by every
 * reconstructor (Software design, Overview). The modes of eigenprobe 0 are replaced by
 * the eigenmodes of their Gram matrix G_mn = sum_p conj(P_m(p)) P_n(p) = V diag(l) V^H,
 * strongest first: P'_j = sum_m V_mj P_m. The same unitary is applied to every
 * eigenprobe, so sum_m |P_k,m|^2 and the forward model are unchanged. Each column of V
 * has its largest-magnitude entry (the first on ties) made real and positive.
 *   probe, probe_out [E][M][N][N] complex (out of place: the two may not overlap)
 *   powers           device double[M] (l_j = ||P'_j||^2, descending) or NULL
 * Gram sums and the Jacobi eigen-solver run in FP64 on the device. */
ptyhip_status ptyhip_orthogonalize_modes(ptyhip_plan plan, void* stream, const float* probe, float* probe_out,
                                         double* powers);

/* Graph replay of repeated calls (for launch-bound loops of small calls, such as
 * minibatches visited epoch after epoch, Performance benchmarking). When enabled, the
 * first ptyhip_forward / ptyhip_forward_adjoint[_ex] call with a given argument set (every
 * pointer, K and the flags) captures its launch chain (fused kernel, object-gradient
 * gather, reductions) into a hipGraph on a stream of the plan and launches it on `stream`;
 * later calls with the same set replay that graph. The data behind the pointers may change
 * between calls; the buffers must stay allocated while the plan caches graphs that use
 * them (disabling the option, or destroying the plan, releases the graphs). Up to 4096
 * argument sets are kept; beyond that the cache is emptied. With timing enabled, a
 * replayed call is timed as one unit (its whole chain). Disabling synchronises the device. */
ptyhip_status ptyhip_plan_set_graphs(ptyhip_plan plan, int32_t enable);

/* Kernel timing: when enabled, every call records a pair of HIP events on its stream
 * immediately around its main kernel (the fused kernel, or the whole per-step chain).
 * ptyhip_plan_kernel_time waits for those events, returns the summed milliseconds and
 * the number of timed launches since the last read, and resets the tally. Up to 4096
 * launches are recorded between reads. */
ptyhip_status ptyhip_plan_set_timing(ptyhip_plan plan, int32_t enable);
ptyhip_status ptyhip_plan_kernel_time(ptyhip_plan plan, double* total_ms, int32_t* launches);

/* Synchronise `stream` and read the plan's device error latch (PTYHIP_FLAG_*) into the
 * host word *flags. The latch collects, over every call since the last clear, the
 * positions the device had to drop: a patch window that leaves the object (the paper's
 * patch extraction, Sec. 2.1, is silent on borders; this library neither wraps nor
 * clamps) or a non-finite position or loss. Returns EINVAL for NULL arguments and EHIP
 * if the synchronisation or the copy fails. */
ptyhip_status ptyhip_get_error(ptyhip_plan plan, void* stream, uint32_t* flags);
/* Clear the latch (asynchronously on `stream`). */
ptyhip_status ptyhip_clear_error(ptyhip_plan plan, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ptyhip_forward_adjoint without a plan.
 * It runs the same fused on-chip kernels; every buffer beyond the caller's inputs and
 * outputs (twiddles, per-workgroup frames and probe-gradient accumulators, per-position
 * partial sums, window gradients, the error latch) is carved out of one file-scope
 * device array of 128 MiB that each GPU the library runs on holds until the process
 * ends. The call allocates nothing: no hipMalloc, no hipFree, no allocating library
 * routine. Positions are processed in chunks that fit the array, with as many
 * persistent workgroups as fit beside them (at most one per CU, or tune->grid).
 *   desc, tune   problem and implementation choice as for ptyhip_plan_create_ex (tune
 *                may be NULL; its mode_groups and probe_stage fields are ignored: a
 *                workgroup always takes whole positions and accumulates the probe
 *                gradient in its own frames; variant 0-4 only, the LDS-resident 5 and 6 are
 *                PTYHIP_EINVAL here); N <= 128, one slice, far field (bilinear or
 *                Fourier-shift patch), else PTYHIP_EUNSUPPORTED
 *   other args   as ptyhip_forward_adjoint (device pointers owned by the caller);
 *                PTYHIP_PLAIN is EUNSUPPORTED, PTYHIP_GRAD_LAMBDA_Z is EINVAL
 *   err_flags    device uint32[1] or NULL: receives this call's error latch
 *                (PTYHIP_FLAG_*; the latch is cleared at the start of every call)
 * PTYHIP_ENOMEM means that one workgroup's frames plus one position's buffers exceed the
 * array (for example N = 128 with very many modes times eigenprobes). Every call on a GPU
 * shares that GPU's array, which keeps the last call's contents: calls that overlap on
 * one GPU (other streams or threads) race and must be serialised by the caller. */
ptyhip_status ptyhip_forward_adjoint_static(const ptyhip_desc* desc, const ptyhip_tune* tune, void* stream,
                                            int32_t K, uint32_t flags, const float* obj, const float* probe,
                                            const float* weights, const float* positions, const float* I_meas,
                                            double* loss, float* I_pred, float* g_obj, float* g_probe, float* g_pos,
                                            float* g_weights, uint32_t* err_flags);

/* Many independent reconstructions of uneven frame sizes in one persistent launch per
 * frame size (64^2, 128^2, 256^2, 512^2), captured once into a hipGraph and replayed (Sec. 2.1: scan points and modes are
 * processed together). descs[i] / K[i] describe dataset i; tune may be NULL. For a batch,
 * tune->grid is the workgroup total of a launch (0: one per CU) and tune->variant the
 * schedule of the frame-size classes: 0 = one after the other, each launch on the whole
 * GPU; 1 = concurrently, as parallel branches of the graph whose launches split the
 * total in proportion to their classes' work (other values are PTYHIP_EINVAL). */
ptyhip_status ptyhip_batch_create(const ptyhip_desc* descs, const int32_t* K, int32_t n, const ptyhip_tune* tune,
                                  ptyhip_batch* out);
/* Bind dataset i's device arrays (same meaning as in ptyhip_forward_adjoint). Rebinding
 * updates a device descriptor table; a captured graph stays valid. */
ptyhip_status ptyhip_batch_bind(ptyhip_batch b, int32_t i, const float* obj, const float* probe,
                                const float* weights, const float* positions, const float* I_meas, double* loss,
                                float* g_obj, float* g_probe, float* g_pos, float* g_weights);
/* Run every dataset (gradient flags as in ptyhip_forward_adjoint; outputs are
 * overwritten). By default the datasets of each frame-size class run in one persistent
 * launch (one workgroup per CU, or the tuned grid) whose workgroups are split among
 * them in proportion to their work, followed by per-dataset
 * reductions; the first launch with given flags captures this into a hipGraph on
 * `stream` and later launches replay it. PTYHIP_BATCH_PER_CALL runs one non-captured
 * fused call per dataset instead, PTYHIP_PLAIN one per-step call per dataset. Frame
 * sizes 64, 128, 256 and 512, one slice. */
ptyhip_status ptyhip_batch_launch(ptyhip_batch b, void* stream, uint32_t flags);
ptyhip_status ptyhip_batch_get_error(ptyhip_batch b, void* stream, uint32_t* flags);
void ptyhip_batch_destroy(ptyhip_batch b);

#ifdef __cplusplus
}
#endif
#endif /* PTYHIP_H */

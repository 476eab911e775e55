/*
 * smi.h -- C ABI of the MI355X staggered-grid acoustic modelling / RTM / FWI library.
 *
 * The library implements, for one GPU, the hot path of SMIwiz (Yang, "SMIwiz: An
 * integrated toolbox for multidimensional seismic modelling and imaging"):
 *
 *   smi_forward              forward modelling (Sec. 2.1, eq. 1-5; Alg. 2 forward loop):
 *                            seismograms, optional boundary saving (Sec. 4.2)
 *   smi_adjoint_reconstruct  reverse loop of Alg. 2: source-field reconstruction from the
 *                            saved boundaries (Sec. 4.2) while the adjoint field (eq. 8) is
 *                            propagated; accumulates the Vp gradient (eq. 7), the
 *                            cross-correlation image (eq. 10) and the source illumination
 *   smi_rtm_image            forward + reverse with the observed data as adjoint source (Sec. 2.3)
 *   smi_fwi_grad             forward + L2 misfit (eq. 6) + reverse: dJ/dVp with rho fixed
 *
 * Work is restricted to the evolving computing box of Sec. 4.1 when grid.box = 1.
 *
 * Conventions
 *   - Every array is float32 unless stated.  Model arrays have n1*n2*n3 entries with
 *     n1 = z fastest, then x (n2), then y (n3) -- the layout of the paper's binary files
 *     (Sec. 3.5, 3.6).  In 2D set ndim = 2 and n3 = 1.
 *   - Positions are (z, x, y) in metres from interior cell 0, inside the interior extent.
 *     A point within 1e-3 of a spacing of a node acts on that node; any other point acts
 *     through a Kaiser-windowed sinc of half-width order/2 per axis (Sec. 2.1; tensor product,
 *     window parameter 2.94 for order 4 and 6.31 for order 8): sources spread
 *     dt stf / dV w_j over the nodes j, receivers record sum_j w_j p_j, and adjoint sources are
 *     injected with the same weights (the transpose of the sampling).
 *   - "device" pointers are HIP device memory of the context's device; "host" pointers are
 *     ordinary host memory, read during the call only.
 *   - All device work is enqueued on the caller's HIP stream (hip_stream; NULL = the null
 *     stream) and is asynchronous: results are ready once that stream is synchronised.
 *   - The caller owns every device buffer, including the workspace `ws`, whose size is
 *     given by smi_workspace_bytes.  The compute entry points never allocate device memory.
 *   - Errors: argument, stability and capacity checks return synchronously (no work is
 *     enqueued then).  Faults detected on the device (non-finite or out-of-range model
 *     values, non-finite wavefields) are latched in a status word inside the workspace and
 *     reported by smi_poll_status.  smi_last_error gives a human-readable reason.
 *   - A context is not thread-safe; use one per host thread.
 */
#ifndef SMI_H
#define SMI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SMI_OK = 0,
    SMI_E_ARG = -1,          /* invalid argument, shape, position or pointer */
    SMI_E_CFL = -2,          /* eq. (5) violated: dt Vmax sqrt(sum 1/d^2) sum|a_l| > 1 */
    SMI_E_DISPERSION = -3,   /* too few points per wavelength (Sec. 3.8) */
    SMI_E_WORKSPACE = -4,    /* workspace missing or smaller than smi_workspace_bytes */
    SMI_E_HIP = -5,          /* HIP runtime error */
    SMI_E_UNSUPPORTED = -6,  /* order not in {4, 8}, grid too large */
    SMI_E_STATE = -7,        /* state missing, consumed, or saved without boundaries */
    SMI_E_NONFINITE = -8     /* device status: non-finite / non-positive model or field */
} smi_status;

/* What a workspace must hold (smi_workspace_bytes). */
typedef enum {
    SMI_JOB_FORWARD = 0,       /* smi_forward without state */
    SMI_JOB_FORWARD_SAVE = 1,  /* smi_forward with state, then smi_adjoint_reconstruct */
    SMI_JOB_RTM = 2,           /* smi_rtm_image */
    SMI_JOB_GRAD = 3,          /* smi_fwi_grad */
    SMI_JOB_BORN = 4           /* smi_born */
} smi_job;

typedef struct smi_ctx smi_ctx;      /* device, options, last error text */
typedef struct smi_state smi_state;  /* host record of a saved forward pass (views into ws) */

/* Simulation parameters; names follow the paper's keywords (Sec. 3.6, 3.8, 4.1, 4.2). */
typedef struct {
    int ndim;                /* 2 or 3 */
    int n1, n2, n3;          /* interior cells along z, x, y (n3 = 1 in 2D) */
    double d1, d2, d3;       /* spacing [m] */
    int nb;                  /* absorbing (CPML) layers per side, >= order/2 */
    int order;               /* spatial order 2N: 4 or 8 */
    int freesurf;            /* 1: free surface (p = 0) on the first interior row z = 0, by the
                                image method (Sec. 2.1): p odd and v_z even about it, no CPML
                                above; 0: absorbing on all sides */
    int nt;                  /* time steps */
    double dt;               /* time step [s] */
    double fm;               /* wavelet centre frequency [Hz]: CPML alpha, dispersion check */
    int dr;                  /* boundary decimation ratio (Sec. 4.2), 1 = exact */
    int box;                 /* 1: evolving computing box (Sec. 4.1) */
    int box_margin;          /* box margin in cells; < 0: default 2N */
    double vpmin, vpmax;     /* bounds of the model speed; 0, 0: reduced from the model
                                on the device (one blocking read-back) */
} smi_grid;

/* Acquisition (Sec. 3.4): one source per shot; receivers of shot s are
 * rec[rec_off[s] .. rec_off[s+1]).  All host arrays. */
typedef struct {
    int nshot;
    const double *src;       /* [nshot][3] (z, x, y) metres */
    const int *rec_off;      /* [nshot + 1], rec_off[0] = 0, non-decreasing */
    const double *rec;       /* [rec_off[nshot]][3] (z, x, y) metres */
} smi_acq;

/* Options (smi_set_option). */
typedef enum {
    SMI_OPT_KERNEL = 0,      /* 0 (default): register-blocked half-step kernels, every shot of
                                the batch in one launch per half step, 4 cells per lane and
                                the XCD-contiguous order in 2D; in 3D the forward and adjoint
                                half steps of 5 (marching along y, SMI_OPT_CHUNK 432) where
                                they apply, register-blocked kernels with 2 cells per lane
                                elsewhere;
                                1: plain stepper -- one shot per launch, one cell per lane;
                                2: fused 2D step (v and p in one marching kernel,
                                double-buffered levels); 3: register-blocked kernels with
                                SMI_OPT_CHUNK = 2, 4 or 8 cells per lane along the slowest
                                axis and the order of SMI_OPT_TILEMAP; 4: batched one-cell-per-
                                lane sweep kernels in the order of SMI_OPT_TILEMAP; 5: as 0, and
                                in 3D half steps that march along y (SMI_OPT_CHUNK = 100 BX + CY:
                                BX = 4 or 8 x-columns of 64 z cells per wavefront, CY = 16,
                                32 or 64 y-planes per workgroup, 32 at order 4; 0: 432); 6: as 0,
                                and in 2D forward passes the fused marching step (v and p of
                                every shot in one launch, levels in two buffers, SMI_OPT_CHUNK
                                = 100 D + C: runs of C = 32 or 64 columns per wavefront, loads
                                issued D = 1, 2 or 4 columns ahead; 0: D 2, C 32); 7: as 0, and
                                in 2D forward passes the tiled fused step (v and p of every
                                shot in one launch, one workgroup per 64-row x C-column tile
                                with its halos staged in LDS; SMI_OPT_CHUNK = C = 32 or 64,
                                else 32); 8: as 0, and in 3D forward and adjoint half steps
                                on plane tiles marching along y (64 z-rows per workgroup, the
                                y-stencil in registers, the plane's z- and x-halo staged in
                                LDS; SMI_OPT_CHUNK = CY + 1000 F: CY = 16, 32 or 64 y-planes per
                                workgroup, tile form F = 0: 2 x-cells per lane x 8 wavefronts,
                                1: 4 x 8, 2: 2 x 16; 0 selects 32).  With a free surface, 2, 6, 7
                                and 8 give way to the kernels of 0 (the y-marching kernels of 0
                                and 5 write the image rows themselves). */
    SMI_OPT_GRAPH = 1,       /* 1: the time loops of a call run as a HIP graph, captured the
                                first time a plan is seen (same geometry, boxes, kernels and
                                buffers) and replayed on later calls; up to 8 graphs are kept
                                per context (default 0).  Not combined with SMI_OPT_TIMING. */
    SMI_OPT_CHUNK = 2,       /* tuning.  SMI_OPT_KERNEL 3: cells per lane (2, 4, 8; else 4),
                                plus 100 to take the z-neighbours from LDS.
                                SMI_OPT_KERNEL 2: 4 or 8 columns per lane (else 4); plus 100:
                                the tiled variant (64 rows x 4 C columns per workgroup, p and
                                the new v staged in LDS) */
    SMI_OPT_TIMING = 3,      /* S > 0: every S-th forward time step of the batched kernels
                                is launched with device-stamped start / stop events, and every
                                S-th reverse iteration is bracketed by events (read with
                                smi_kernel_timing); 0: off (default).  Setting it clears the
                                samples collected so far.  Reverse loops are not replayed as
                                graphs while it is on. */
    SMI_OPT_TILEMAP = 4,     /* tile order of SMI_OPT_KERNEL 3 and 4: 0 plain (z-block fastest,
                                then x-block); 1 each of the 8 XCDs takes a contiguous range of
                                x-blocks, so tiles that share halos share an L2; 2 (3D, kernel
                                3) each XCD takes a contiguous range of tiles ordered z-block
                                fastest, then x-group, y-strip and shot, so the tiles resident
                                on one XCD are neighbours that read the same halo planes (the
                                order of the default's 3D register-blocked kernels) */
    SMI_OPT_FAMILY = 5,      /* parametrisation of the gradients (Sec. 2.2): 1 (default) (Vp, rho):
                                grad_vp = dJ/dVp at fixed rho, grad_rho = dJ/drho at fixed Vp;
                                2 (Vp, Ip = rho Vp): grad_vp = dJ/dVp at fixed Ip, grad_rho =
                                dJ/dIp at fixed Vp */
    SMI_OPT_REVERSE = 6,     /* 2D reverse step of the default kernels: 0 (default) two launches
                                per step (reconstruction of p with the adjoint v update and the p
                                bands; then reconstruction of v with the adjoint p update and the
                                v bands) when the shots of a reverse loop (SMI_OPT_REV_GROUP)
                                hold up to 8 M padded cells, five launches above; 1 always two;
                                2 always five.  Same results. */
    SMI_OPT_AUTOTUNE = 7,    /* 1: the library picks the kernels per plan shape (geometry, shots,
                                nt, box, dr, job kind) by timing them on the device: the first
                                forward pass of a shape times every forward candidate (kernel
                                family, cells per lane, tile order, the fused 2D step's run width
                                and look-ahead) on 24 steps spread over the schedule, on cleared
                                fields, and runs with the fastest (one blocking wait per shape);
                                the first 2D reverse pass of a shape alternates its two reverse-
                                step forms on every 16th iteration and the next reverse pass
                                keeps the faster.  Every candidate gives the default's results.
                                smi_tuning_report tells the last pick.  0: off (default);
                                2: forget the picks made so far (the switch stays as it was). */
    SMI_OPT_REV_GROUP = 8,   /* 2D reverse passes (Alg. 2 reverse loop) run the loop once per
                                group of consecutive shots: 0 (default) the largest equal groups
                                whose reverse state (source and adjoint fields, CPML variables,
                                accumulators), as their computing boxes touch it on average over
                                the reverse steps, fits 224 MiB, 7/8 of the device's last-level
                                cache, so that each group's launches keep it there; k > 0 at
                                most k shots per group (k >= the shot count: one loop over all
                                shots).  3D passes and the plain stepper run one loop.  Same
                                results for every value. */
    SMI_OPT_FWD_GROUP = 9    /* 2D forward passes of the default (register-blocked) kernels run
                                the time loop once per group of consecutive shots, as
                                SMI_OPT_REV_GROUP does for reverse passes: 0 (default) one
                                loop while the fields (p, v and the CPML variables) under every
                                shot's computing box fit 224 MiB at every step, else the count
                                of equal groups (at most 16) of least modelled time over the
                                schedule of boxes (a fixed cost per launch, and a higher cost
                                per cell at steps where a group's fields exceed 224 MiB);
                                k > 0 at most k shots per group.  The fused steps
                                (SMI_OPT_KERNEL 2, 6, 7), 3D passes and the plain stepper run
                                one loop.  Same results for every value. */
} smi_option;

/* Text of the autotuner's last pick on this context (candidates, their times per step, the
 * pick), or "" before any (never NULL). */
const char *smi_tuning_report(const smi_ctx *ctx);

/* Create a context on HIP device `hip_device`. */
smi_status smi_ctx_create(int hip_device, smi_ctx **out);
void smi_ctx_destroy(smi_ctx *ctx);
/* Text of the last error raised on this context (never NULL). */
const char *smi_last_error(const smi_ctx *ctx);
smi_status smi_set_option(smi_ctx *ctx, int option, int value);

/* Results per group of shots (the sum over shots of Alg. 2 / Sec. 3.2 taken per group instead
 * of over the whole call), for callers that batch the shots of several independent jobs on one
 * model into one call.  shot_off: host [ngroup + 1], shot_off[0] = 0, strictly increasing; group
 * k is the shots [shot_off[k], shot_off[k+1]).  While set, every reduced output of
 * smi_adjoint_reconstruct, smi_rtm_image and smi_fwi_grad (grad_vp, grad_rho, image, illum,
 * image_norm: device [ngroup][n1*n2*n3]; misfit: device double [ngroup]) holds one result per
 * group, each summed over its own shots in order -- bitwise what the group's shots give in a
 * call of their own.  A call whose shot count differs from shot_off[ngroup] fails with
 * SMI_E_ARG.  ngroup = 0 returns to one result per call (the default).  Copied; host only. */
smi_status smi_set_shot_groups(smi_ctx *ctx, int ngroup, const int *shot_off);

/* Host checks run by every entry point (Sec. 3.8): eq. (5) with Vmax = vp_max, and at least
 * 5 (order 4) or 3 (order 8) points per wavelength at the highest frequency 2.5 fm:
 * vp_min / (2.5 fm max(d)) >= ppw.  Returns SMI_OK, SMI_E_CFL, SMI_E_DISPERSION or SMI_E_ARG. */
smi_status smi_check(const smi_ctx *ctx, const smi_grid *grid, double vp_min, double vp_max);

/* Bytes of device workspace that `job` needs for this grid and acquisition. */
smi_status smi_workspace_bytes(const smi_ctx *ctx, const smi_grid *grid, const smi_acq *acq,
                               smi_job job, size_t *bytes);

/* Forward modelling, all shots batched (Sec. 2.1; Alg. 2 forward loop).
 *   vp, rho  device [n1*n2*n3]       model (extended into the CPML layers by edge replication)
 *   stf      device [nshot][nt]      source time function; p[src] += dt stf[it] / (d1 d2 [d3])
 *                                    after the p update of step it
 *   dcal     device                  shot s at dcal + nt*rec_off[s], layout [nt][nrec_s]:
 *                                    dcal[it][r] = p^{it+1} at receiver r
 *   state_out NULL: no boundary saving.  Otherwise the bands of Sec. 4.2 are saved every dr
 *            steps and *state_out receives a host record of the final wavefield and the bands
 *            (inside ws, which must be sized for SMI_JOB_FORWARD_SAVE); free it with
 *            smi_state_destroy.  vp, rho, stf must stay valid until the state is consumed.
 *   snap_it, nsnap, snaps   optional: host list of time levels (0..nt); snaps (device,
 *            [nshot][nsnap][n1*n2*n3]) receives p at those levels (interior).  NULL/0 = none.
 *   ws, ws_bytes  device workspace (>= smi_workspace_bytes). */
smi_status smi_forward(smi_ctx *ctx, const smi_grid *grid, const smi_acq *acq,
                       const float *vp, const float *rho, const float *stf, float *dcal,
                       smi_state **state_out, const int *snap_it, int nsnap, float *snaps,
                       void *ws, size_t ws_bytes, void *hip_stream);

/* Size of the static workspace of smi_forward_static, per device (bytes). */
#define SMI_STATIC_WS_BYTES (64u << 20)

/* smi_forward (no state, no snapshots) for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation.  The workspace
 * is a static device buffer of SMI_STATIC_WS_BYTES that the library keeps on each device from
 * the first context created there until the process ends; the caller passes only inputs and
 * outputs (vp, rho, stf, dcal as in smi_forward).  The call allocates nothing, captures no graph
 * and records no timing events (SMI_OPT_GRAPH and SMI_OPT_TIMING are ignored for it).
 * SMI_E_WORKSPACE, before any device work, when the job's SMI_JOB_FORWARD workspace exceeds
 * SMI_STATIC_WS_BYTES (a 2D order-8 grid of about 1.5 M padded cells per shot fits); SMI_E_HIP
 * when the buffer's device address could not be obtained.  Every call on one device uses that
 * device's one buffer, which keeps the last call's contents (each call clears what it needs):
 * calls that overlap in time on one device, on any streams or contexts, race -- serialise
 * them. */
smi_status smi_forward_static(smi_ctx *ctx, const smi_grid *grid, const smi_acq *acq,
                              const float *vp, const float *rho, const float *stf, float *dcal,
                              void *hip_stream);

/* Reverse loop of Alg. 2 on a saved forward pass (consumes the state).
 *   adj_src  device, layout of dcal: the adjoint source G injected as p~[rec] += kappa G[it]
 *            before reverse step it (eq. 8 in the scaled variable p~ = kappa pbar).
 *            G = dt (dcal - dobs) gives dJ/dVp of eq. (6)-(7); G = dL/d(dcal) gives the
 *            vector-Jacobian product of any loss; G = dt dobs gives the RTM image (Sec. 2.3).
 *   grad_vp  device [n1*n2*n3] or NULL: sum over shots of dL/dVp, rho held fixed:
 *            -(2 dt / Vp) sum_it p~ div v^{it+1/2} (eq. 7 with kappa = rho Vp^2).  Overwritten.
 *            With SMI_OPT_FAMILY 2: dL/dVp at fixed Ip = rho Vp.
 *   grad_rho device [n1*n2*n3] or NULL: dL/drho at fixed Vp (family 1) or dL/dIp at fixed Vp
 *            (family 2).  The density part of eq. (7) in the discrete scheme: every v update
 *            uses beta_a = 2/(rho_i + rho_{i+1}) on the face, so dL/drho at fixed kappa sums
 *            -(dt/2) beta_f v~^{it+1/2}_f (D+_a p^it)_f over the faces of the node (v~ the
 *            adjoint velocity of the same solver); kappa = rho Vp^2 adds Vp^2 dL/dkappa.
 *            Interior nodes only (the edge-replicated values in the absorbing layers are not
 *            differentiated).  Needs a state saved for SMI_JOB_FORWARD_SAVE or
 *            SMI_JOB_GRAD (SMI_E_ARG otherwise).  Overwritten.
 *   image    device [n1*n2*n3] or NULL: sum_s sum_it dt p~^it p^it (eq. 10).  Overwritten.
 *   illum    device [n1*n2*n3] or NULL: sum_s sum_it dt (p^it)^2.  Overwritten.
 *   image_norm device [n1*n2*n3] or NULL: the normalised imaging condition of Sec. 2.3, each
 *            shot's image divided by its own source illumination, summed over shots:
 *            sum_s image_s / (illum_s + 1e-3 max(illum_s)) (the stabiliser is not given by the
 *            paper).  Overwritten.
 *   snap_it, nsnap, snaps   optional: reconstructed source-field p at the listed levels,
 *            device [nshot][nsnap][n1*n2*n3].
 * The state must come from smi_forward on the same context. */
smi_status smi_adjoint_reconstruct(smi_ctx *ctx, smi_state *state, const float *adj_src,
                                   float *grad_vp, float *grad_rho, float *image, float *illum,
                                   float *image_norm, const int *snap_it, int nsnap, float *snaps,
                                   void *hip_stream);

/* RTM (Sec. 2.3): forward with boundary saving, then the reverse loop with G = dt dobs.
 * dobs has the layout of dcal.  image / illum / image_norm as in smi_adjoint_reconstruct (any
 * may be NULL). */
smi_status smi_rtm_image(smi_ctx *ctx, const smi_grid *grid, const smi_acq *acq,
                         const float *vp, const float *rho, const float *stf, const float *dobs,
                         float *image, float *illum, float *image_norm, void *ws, size_t ws_bytes,
                         void *hip_stream);

/* Born (tangent-linear) modelling with respect to kappa = rho Vp^2: the data perturbation
 * of a model perturbation dkappa (the linearisation the paper lists as under development;
 * the derivative of smi_forward's data).  The background field runs the forward step; the
 * perturbation field obeys the same step (CPML included) plus the secondary source
 * -dt dkappa div v^{it+1/2} in its p update, and ddata[it][r] = dp^{it+1} at receiver r.
 *   dkappa  device [n1*n2*n3] (interior; zero in the absorbing layers).  For a velocity
 *           perturbation at fixed rho, dkappa = 2 rho Vp dVp.
 *   ddata   device, layout of dcal.
 *   ws      device workspace of SMI_JOB_BORN. */
smi_status smi_born(smi_ctx *ctx, const smi_grid *grid, const smi_acq *acq, const float *vp,
                    const float *rho, const float *stf, const float *dkappa, float *ddata,
                    void *ws, size_t ws_bytes, void *hip_stream);

/* Laplace filter of an image (Sec. 2.3, against the low-wavenumber artefacts of RTM images):
 * out = sum_a (f[i+1] - 2 f[i] + f[i-1]) / d_a^2 over the grid's axes (second-order central
 * differences), with f = 0 outside the n1*n2[*n3] image.  in, out: device, z fastest, must not
 * alias.  Only ndim, n1..n3 and d1..d3 of the grid are read.  SMI_E_ARG on bad sizes. */
smi_status smi_laplacian(smi_ctx *ctx, const smi_grid *grid, const float *in, float *out,
                         void *hip_stream);

/* FWI gradient (Sec. 2.2): forward with boundary saving, residual r = dcal - dobs,
 * misfit J = 1/2 dt sum r^2 (eq. 6, rectangle rule; device double, may be NULL), G = dt r,
 * reverse loop -> grad_vp and / or grad_rho (device [n1*n2*n3], as in
 * smi_adjoint_reconstruct, at least one).  dcal_out (device, layout of dcal) receives the
 * synthetic data when not NULL. */
smi_status smi_fwi_grad(smi_ctx *ctx, const smi_grid *grid, const smi_acq *acq,
                        const float *vp, const float *rho, const float *stf, const float *dobs,
                        float *grad_vp, float *grad_rho, double *misfit, float *dcal_out,
                        void *ws, size_t ws_bytes, void *hip_stream);

void smi_state_destroy(smi_state *state);

/* Synchronise hip_stream and report the device status word of the last workspace used on
 * this context (SMI_E_NONFINITE when a model value was non-finite or non-positive, or a
 * wavefield became non-finite).  Clears the word. */
smi_status smi_poll_status(smi_ctx *ctx, void *hip_stream);

/* Algorithmic counts of the last compute call on this context (host, after the call):
 * cell updates inside the computing boxes, summed over shots and steps, for the forward
 * field (fwd), the adjoint field (adj) and the reconstructed field (rec). */
smi_status smi_last_counts(const smi_ctx *ctx, double *fwd, double *adj, double *rec);

/* Algorithmic HBM bytes of the last forward loop and the last reverse loop on this context:
 * the FP32 traffic the method itself requires (fields and CPML memory variables read and
 * written once per cell-step inside the boxes, the model once per step, receivers, saved and
 * restored boundary bands, image / gradient accumulators), independent of how the kernels
 * move it.  Used to express throughput as a fraction of the HBM roofline. */
smi_status smi_last_bytes(const smi_ctx *ctx, double *fwd_bytes, double *rev_bytes);

/* Durations of the forward time-step kernels (which 0-2) or of whole reverse iterations
 * (which 3) sampled (SMI_OPT_TIMING) since the option was last set, over every forward or
 * reverse pass run on this context meanwhile.  Waits for the sampled work to finish.
 *   which 0: the whole step (start of the v kernel to the end of the p kernel), with the
 *            algorithmic bytes of the step as the method defines it (fields read and written
 *            once, CPML memory variables, the model once per step for the batch);
 *         1: the v kernel (eq. 3, first row) and its own algorithmic bytes (reads p, reads and
 *            writes v_a, CPML variables of p, dt beta_a);
 *         2: the p kernel (eq. 3, second row, source injection) and its bytes (reads v_a, reads
 *            and writes p, CPML variables of v, dt kappa).
 *         3: a reverse iteration of Alg. 2 (adjoint source, source removal, reconstruction,
 *            adjoint step, accumulators; from its first launch to the end of its last, gaps
 *            between launches included) and its algorithmic bytes (adjoint and reconstructed
 *            fields read and written once, CPML variables, model, restored bands, adjoint
 *            sources, and the accumulators the call computes).
 *   With a fused 2D step (SMI_OPT_KERNEL 2 or 6) the step is one kernel: which 0 and 1 both
 *   report it, with the step's bytes, and which 2 reports nothing (0 ms, 0 bytes).
 *   avg_ms     mean kernel duration over the samples (ms);
 *   avg_bytes  mean algorithmic bytes of the sampled launches;
 *   nsamples   number of samples (0: nothing timed; both means are then 0).
 * Any output pointer may be NULL.  SMI_E_ARG for another `which`. */
smi_status smi_kernel_timing(smi_ctx *ctx, int which, double *avg_ms, double *avg_bytes,
                             int *nsamples);

#ifdef __cplusplus
}
#endif

#endif /* SMI_H */

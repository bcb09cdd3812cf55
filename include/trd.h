/*
 * trd.h -- C ABI of the MI355X TRD tracklet-to-track matcher.
 *
 * Problem (paper, abstract and Sect. 3): given ITS-TPC seed tracks
 * extrapolated to the TRD and the TRD tracklets of the same interaction(s),
 * return for every track the tracklet matched in each of the six layers (at
 * most one per layer) and the track state after the Kalman updates.  Tracks
 * are independent; a track only sees tracklets of its own group (frame or
 * trigger, Sect. 4 of the paper).
 *
 * Conventions
 *   - Units: cm, GeV/c, tesla.  Track state p = (y, z, sin phi, tan lambda,
 *     q/pT) at local x in the frame of sector `sector`, rotated by
 *     alpha = (sector + 1/2) * 20 degrees.  Covariance: upper triangle of the
 *     symmetric 5x5 matrix, row-major, 15 values.
 *   - All array arguments are DEVICE pointers in structure-of-arrays layout,
 *     component-major: element k of track i is at [k * n + i].
 *   - Floating-point arrays of tracks and results are float (TRD_PREC_FP32,
 *     TRD_PREC_FP32_COV64) or double (TRD_PREC_FP64), as set in the config.
 *   - Every call enqueues work on `hip_stream` (a hipStream_t, NULL = default
 *     stream) and returns without waiting.  The caller synchronises.  One
 *     context must not be used from two streams at once; contexts are
 *     independent of each other.
 *   - Calls return an int status (TRD_OK or a negative TRD_E* code) and never
 *     throw across the ABI.  Invalid arguments are reported synchronously
 *     (TRD_EINVAL).  Before it enqueues anything, every stream-ordered call
 *     checks for a HIP error left pending on the calling thread (a failed
 *     launch or call) and for one that work already on its stream ran into
 *     (a fault in an enqueued kernel, seen once the stream has reached it;
 *     not checked while the stream is being captured); it consumes the error
 *     and returns TRD_EDEVICE without enqueuing.  Per-track problems never
 *     fail a call: they are status bits (TRD_TRK_*).
 */
#ifndef TRD_H
#define TRD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRD_N_SECTORS 18
#define TRD_N_STACKS 5
#define TRD_N_LAYERS 6
#define TRD_N_DET 540 /* sector * 30 + stack * 6 + layer */

/* call status */
#define TRD_OK 0
#define TRD_EINVAL (-1)  /* bad config, shape or pointer */
#define TRD_ENOMEM (-2)  /* device allocation failed */
#define TRD_EDEVICE (-3) /* HIP error from enqueued work or the runtime */
#define TRD_ESTATE (-4)  /* trd_match before any trd_load_tracklets */
#define TRD_EBUDGET (-5) /* request exceeds the context's HBM budget */

/* arithmetic of the match kernel */
#define TRD_PREC_FP64 0       /* everything in double */
#define TRD_PREC_FP32 1       /* float state and covariance; tracks whose
                                 covariance stops being positive definite
                                 are re-run with a double covariance */
#define TRD_PREC_FP32_COV64 2 /* float state, double covariance */

/* per-track status bits (trd_results.status) */
#define TRD_TRK_STOP_SNP 1u      /* |sin phi| reached snp_max: track stopped */
#define TRD_TRK_ROT_FAIL 2u      /* sector change impossible: track stopped */
#define TRD_TRK_OUT_OF_Z 4u      /* a layer's search window missed the chambers in z */
#define TRD_TRK_FP64_FALLBACK 8u /* result comes from the double-covariance re-run */
#define TRD_TRK_NOT_PD 16u       /* float covariance lost positive definiteness */
#define TRD_TRK_BAD_INPUT 32u    /* non-finite seed, bad sector/group, |snp| >= snp_max,
                                    or covariance not positive definite; copied through */
#define TRD_TRK_REFIT_FEW 64u    /* trd_refit: fewer than refit_min tracklets; copied */
#define TRD_TRK_REFIT_SKIP 128u  /* trd_refit: a tracklet more than one sector away was skipped */
#define TRD_TRK_STOPPED 256u     /* a layer's energy loss left the particle no kinetic energy */

/* config flags */
#define TRD_CFG_FAIL_ALLOC 1u     /* test hook: trd_create fails with TRD_ENOMEM */
#define TRD_CFG_FORCE_FALLBACK 2u /* test hook (TRD_PREC_FP32): every track takes the
                                     double-covariance re-run */
#define TRD_CFG_INPUT_ORDER 8u    /* match the tracks in the caller's order; by default
                                     the one-lane-per-track and the several-hypotheses
                                     launches first sort them by (group, sector,
                                     |q/pT| class, z, y) of the seed so that neighbouring
                                     lanes read neighbouring cells (results are the same,
                                     bit for bit, and come back in input order) */
#define TRD_CFG_TIME_KERNEL 16u   /* record HIP events on the launch stream around the
                                     main match kernel of every trd_match (read them with
                                     trd_kernel_times) */
#define TRD_CFG_PERSISTENT 4u     /* one-lane-per-track matching as a persistent grid
                                     (resident workgroups pull blocks of tracks from a
                                     work counter); for large multi-frame batches.
                                     Requires search_lanes 0 or 1 (else TRD_EINVAL). */

typedef struct trd_ctx trd_ctx;

/* Plain-value configuration.  Geometry and resolutions follow Sect. 3 of the
 * paper (18 sectors x 5 stacks x 6 layers, tracklets with y, dy over the drift
 * length and a pad row, tilted pads); the numbers the paper leaves open are
 * fields. */
typedef struct trd_config {
    uint32_t struct_size;     /* sizeof(trd_config) */
    int32_t precision;        /* TRD_PREC_* */
    double x_layer[6];        /* radius (local x) of each layer's chamber plane */
    double tilt[6];           /* tan(pad tilt) per layer; y measured = y + tilt*(z - z_row) */
    double z_min;             /* lower z edge of stack 0; chambers span [z_min, -z_min] */
    double pad_len;           /* pad-row length in z */
    int32_t n_rows;           /* pad rows per stack (<= 32) */
    int32_t n_yb;             /* y bins per (chamber, dy bin) in the tracklet cells */
    int32_t n_db;             /* deflection (dy) bins per chamber; 1 = no dy binning */
    uint32_t flags;           /* TRD_CFG_* */
    double y_bin_w;           /* y bin width, a power of two; bins cover
                                 [-n_yb*w/2, n_yb*w/2), outer bins are open */
    double dy_bin_w;          /* dy bin width, a power of two, same layout */
    double drift_len;         /* drift length L: dy = L * (tan phi - tan_psi) */
    double dx_chamber[540];   /* radial offset of each chamber from x_layer (misalignment) */
    double bz;                /* solenoid field */
    double x_over_x0;         /* material per layer, radiation lengths */
    double mass;              /* particle mass for scattering */
    double sigma_y[3];        /* y resolution a0 + a1 s + a2 s^2, s = sin phi */
    double sigma_dy[3];       /* dy resolution, same polynomial form */
    double tan_psi;           /* tangent of the Lorentz angle */
    double chi2_max;          /* chi2 cut of a candidate (2 dof) */
    double n_sigma_dy;        /* dy exclusion gate, in sigma (paper: 4) */
    double n_sigma_road;      /* road half widths n * sqrt(S_yy), n * sqrt(S_zz) */
    double snp_max;           /* stop when |sin phi| reaches this */
    uint64_t hbm_budget_bytes;/* cap on the context's device memory, 0 = none */
    int32_t block_size;       /* match workgroup size: 64, 128, 192 or 256; 0 = 256 */
    int32_t search_lanes;     /* float paths: lanes that share one track's road (each
                                 scans whole cell ranges): 1 (one lane per track),
                                 4, 8, 16, 32 or 64; 0 = 1 */
    int32_t n_hyp;            /* hypotheses kept per layer (Sect. 3, Fig. 2: the best
                                 N_candidates hypotheses of a layer seed the next):
                                 0 = the single best candidate per layer; 1, 2, 4 or 8 =
                                 that many paths, each costing the chi2 of its tracklets
                                 plus chi2_penalty per layer without one; the answer is
                                 the cheapest path after the last layer.  Requires
                                 search_lanes 0 or 1 and no TRD_CFG_PERSISTENT. */
    double chi2_penalty;      /* cost of a layer without a tracklet (n_hyp >= 1);
                                 >= chi2_max makes n_hyp = 1 the single best rule */
    double refit_cov[5];      /* trd_refit: starting covariance, diagonal (y, z, sin phi,
                                 tan lambda, q/pT); each > 0 */
    int32_t refit_min;        /* trd_refit: tracks with fewer tracklets are copied (>= 1) */
    double tpc_x_in, tpc_x_out; /* residual maps: pad row r sits at x_out - r (x_out - x_in)
                                 / (tpc_n_rows - 1), in the sector frame */
    int32_t tpc_n_rows;       /* >= 2, <= 65535 */
    int32_t vox_nx, vox_ny, vox_nz; /* voxels per sector in x, y/x (over +-tan 10 deg),
                                 z/x (over +-1); 18 * nx * ny * nz <= 2048 */
    int32_t vox_min;          /* fewest clusters for a voxel's distortion vector */
    /* Realistic detector model (Sect. 3: the extrapolation to a chamber
       accounts for energy loss; the detector equips 522 of its 540 slots). */
    double eloss_xrho;        /* material of one layer crossed at normal incidence, g/cm^2;
                                 0 = no energy loss.  After each layer's scattering the mean
                                 loss (Bethe formula without density or shell terms, rate at
                                 the momentum before the loss) times the path through the
                                 slab lowers the energy (matching) or restores it (trd_refit,
                                 inward); q/pT scales by p/p' and its covariance row by
                                 (p/p')^3 E'/E.  A particle left with E <= m stops
                                 (TRD_TRK_STOPPED). */
    double eloss_za;          /* Z/A of that material (> 0 when eloss_xrho > 0) */
    double eloss_i;           /* its mean excitation energy, GeV (> 0 when eloss_xrho > 0) */
    uint8_t chamber_absent[540]; /* nonzero: no chamber in this slot (sector * 30 + stack * 6
                                 + layer).  Its tracklets are dropped at load; with n_hyp >= 1
                                 a layer whose predicted point lies in such a slot costs no
                                 chi2_penalty. */
    /* Field inhomogeneity (Sect. 3: the precise extrapolation to a chamber
       accounts for the field).  Bz(r, z) = bz (1 + field_br (r / 370 cm)^2 +
       field_bz (z / 360 cm)^2), r the distance from the beam axis; both 0 =
       uniform field (closed-form helix steps).  Otherwise every propagation
       of the matching and the refit integrates y' = tan(phi), z' =
       tan(lambda)/cos(phi), sin(phi)' = -kappa Bz q/pT over local x with the
       classical 4th-order Runge-Kutta method in equal steps of at most
       field_step, and transports the covariance with the exact helix
       Jacobian over the whole step in the field the integration saw (the mean
       of the Runge-Kutta weighted field samples).  The residual maps keep the
       uniform-field step. */
    double field_br, field_bz; /* |.| < 1 */
    double field_step;        /* cm, in (0, 20]; used with a field map */
} trd_config;

/* Tracklets of one or more groups (device arrays of length n). */
typedef struct trd_tracklets {
    const float *y;          /* offset at the chamber radius */
    const float *z;          /* pad-row centre */
    const float *dy;         /* deflection over the drift length */
    const uint32_t *det_row; /* (det << 5) | pad row within the stack */
    const int32_t *group;    /* group id in [0, n_groups), or NULL: all 0 */
} trd_tracklets;

/* Seed tracks (device arrays, float or double per precision). */
typedef struct trd_tracks {
    const void *p;         /* [5][n] */
    const void *cov;       /* [15][n] */
    const void *x;         /* [n] local x of the state */
    const int32_t *sector; /* [n] */
    const int32_t *group;  /* [n] or NULL: all 0 */
} trd_tracks;

/* Results (device arrays allocated by the caller). */
typedef struct trd_results {
    int32_t *idx;      /* [6][n] input-order tracklet index per layer, -1 if none */
    void *p;           /* [5][n] state after the last layer reached */
    void *cov;         /* [15][n] */
    void *x;           /* [n] */
    int32_t *sector;   /* [n] sector frame of the output state */
    void *chi2;        /* [n] sum of the matched candidates' chi2 */
    void *chi2_layer;  /* [6][n] chi2 per layer (0 if none), or NULL */
    int32_t *n_match;  /* [n] number of matched layers */
    uint32_t *status;  /* [n] TRD_TRK_* bits */
} trd_results;

/* Read-only view of the context's sorted tracklets. */
typedef struct trd_binning_view {
    const uint32_t *offsets; /* [n_cells + 1]: first sorted position of each cell;
                                offsets[n_cells] = number of valid tracklets */
    const float *sorted;     /* [n_valid][4]: y, dy, z, input index (int32 bits),
                                ordered by (cell, input index) */
    int64_t n_cells;         /* n_groups * 540 * n_rows * n_db * n_yb */
    int64_t n_tracklets;     /* tracklets passed to the last load */
} trd_binning_view;

/* Sets up the detector of Sect. 3 of the paper (18 sectors x 5 stacks x 6
 * layers of chambers with pad rows, tilted pads, resolutions as polynomials
 * in sin phi, the chi2 and dy cuts of the search) from the plain values of
 * `cfg`: validates them, selects `device` and uploads the geometry.  Owns no
 * tracklets yet.  Synchronous.  Errors: TRD_EINVAL (bad config: a field out
 * of range, a bin width that is not a power of two, pad rows that do not tile
 * [z_min, -z_min]), TRD_ENOMEM, TRD_EDEVICE (no such device, upload failed).
 * On success *out owns the context until trd_destroy; on failure *out is
 * NULL and nothing is held. */
int trd_create(const trd_config *cfg, int device, trd_ctx **out);

/* Reserves device buffers for up to `max_tracklets` tracklets, `max_groups`
 * groups and `max_tracks` tracks, so that later loads and matches of that
 * size allocate nothing (needed under stream capture).  Synchronous.
 * Errors: TRD_EINVAL, TRD_ENOMEM, TRD_EBUDGET. */
int trd_reserve(trd_ctx *ctx, int64_t max_tracklets, int32_t max_groups, int64_t max_tracks);

/* Prepares the search of Sect. 3 of the paper (every tracklet within a road
 * sized from the track and tracklet covariances, and from the track's own
 * interaction only, Sect. 4): bins the tracklets into (group, chamber, dy bin,
 * y bin, pad row) cells (pad rows innermost, so the cells of one (dy bin,
 * y bin) that overlap a road are contiguous): exact cell keys, a stable sort
 * by (cell, input index) into ctx-owned sorted storage, which replaces the
 * previous load's.  Stream-ordered.  The caller may reuse `t`'s buffers once the stream has
 * passed this call.  Tracklets with a det >= 540, a row >= n_rows, a group
 * outside [0, n_groups) or a non-finite value are dropped.
 * Errors: TRD_EINVAL (n < 0, n_groups < 1, NULL pointers with n > 0,
 * too many cells), TRD_ENOMEM, TRD_EBUDGET, TRD_EDEVICE. */
int trd_load_tracklets(trd_ctx *ctx, const trd_tracklets *t, int64_t n, int32_t n_groups,
                       void *hip_stream);

/* Matches n tracks against the tracklets of the last load (Sect. 3 of the
 * paper: propagation to each layer, sector rotation, multiple scattering,
 * covariance road, dy exclusion, chi2 from y and z, best candidate, precise
 * propagation and Kalman update).  Errors: TRD_EINVAL, TRD_ESTATE,
 * TRD_ENOMEM, TRD_EBUDGET, TRD_EDEVICE. */
int trd_match(trd_ctx *ctx, const trd_tracks *in, int64_t n, trd_results *out, void *hip_stream);

/* trd_match for callers that cannot allocate device memory: code under
 * stream (graph) capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same kernels and results as trd_match, bit for bit, with the
 * tracks matched in the caller's order; it calls no allocating routine.  Its
 * scratch (the float path's re-run queue and the kernels' counters) is one
 * library-owned device array per GPU of 4 * (64 + 2^21) bytes (8 MB), held
 * from the first trd_create on that GPU until the process ends; the counters
 * are cleared by a fill kernel at the start of every call.  The caller still
 * passes inputs and outputs, and the context must have been created (and its
 * tracklets loaded, which allocates unless trd_reserve sized it) beforehand.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on the same GPU (other streams or threads, other contexts) race and give
 * wrong results; serialise them.  Errors: as trd_match, and TRD_EINVAL for
 * n > 2^21 tracks or a device ordinal >= 64. */
int trd_match_noalloc(trd_ctx *ctx, const trd_tracks *in, int64_t n, trd_results *out, void *hip_stream);

/* Matched tracks for trd_refit (device arrays of the state type, as written
 * by trd_match). */
typedef struct trd_refit_in {
    const void *p;          /* [5][n] state after matching */
    const void *x;          /* [n] its radius */
    const int32_t *sector;  /* [n] its sector */
    const int32_t *idx;     /* [6][n] matched tracklet per layer (input index), -1 if none */
} trd_refit_in;

/* Refit results (device arrays the caller owns). */
typedef struct trd_refit_out {
    void *p;           /* [5][n] state at layer 0 (the innermost layer reached) */
    void *cov;         /* [15][n] its covariance, packed upper triangle */
    void *x;           /* [n] */
    int32_t *sector;   /* [n] */
    void *chi2;        /* [n] sum of the predicted chi2 of the updates */
    int32_t *n_used;   /* [n] tracklets used */
    uint32_t *status;  /* [n] TRD_TRK_* bits of the refit */
} trd_refit_out;

/* trd_load_tracklets followed by trd_match on the same stream (the search
 * of Sect. 3 over one batch of tracklets and seeds), with the same results,
 * but the seeds' processing order is computed on a stream of the context
 * while the tracklets are binned (the two are independent), joined before
 * the match.  Both inputs must be ready on hip_stream when it is called.
 * Arguments and errors as of the two calls (checked before anything is
 * enqueued); capturable into a graph like them (the fork is joined back
 * into hip_stream). */
int trd_load_and_match(trd_ctx *ctx, const trd_tracklets *t, int64_t n_tkl, int32_t n_groups,
                       const trd_tracks *in, int64_t n, trd_results *out, void *hip_stream);

/* TRD-only refit of matched tracks (Sect. 2, step 3: a refit from the outer
 * detectors in which the TPC information is ignored).  For each track: the
 * state of trd_match with its covariance replaced by diag(refit_cov), then
 * inward over layers 5..0: propagation to the layer plane (sector hops as in
 * the matching), for a matched tracklet a turn into its sector if that is a
 * neighbour (else REFIT_SKIP), the step to its radius and the Kalman update,
 * then the layer's scattering (not below layer 0).  The covariance is kept in
 * double in every precision.  tkl: the tracklets the indices refer to (y, z,
 * det_row of the trd_match input, n_tkl of them; group unused).  An index
 * counts only if it lies in [0, n_tkl) and names a tracklet of that layer's
 * chamber (det < 540, det mod 6 = layer); others count as -1.  Tracks with
 * fewer than refit_min usable indices are copied with REFIT_FEW, rejected
 * states with BAD_INPUT.  Stream-ordered.  Errors: TRD_EINVAL, TRD_EDEVICE. */
int trd_refit(trd_ctx *ctx, const trd_refit_in *in, const trd_tracklets *tkl, int64_t n_tkl, int64_t n,
              trd_refit_out *out, void *hip_stream);

/* Reference tracks for the residual maps (device arrays of the state type,
 * e.g. a trd_refit_out): state, radius, sector, status (tracks with any
 * status bit are left out). */
typedef struct trd_reference {
    const void *p;           /* [5][n] */
    const void *x;           /* [n] */
    const int32_t *sector;   /* [n] */
    const uint32_t *status;  /* [n] */
} trd_reference;

/* TPC clusters of the reference tracks (device arrays). */
typedef struct trd_tpc_clusters {
    const float *y, *z;        /* [n_cl] cluster position at its pad row, sector frame */
    const uint32_t *row_sec;   /* [n_cl] (sector << 16) | pad row */
    const int64_t *first;      /* [n + 1] clusters of track i: first[i] .. first[i+1]-1,
                                  outermost row first */
} trd_tpc_clusters;

/* Residual maps (Sect. 2, steps 4-5): each reference track is carried along
 * its helix to its clusters' pad rows (turning into a neighbouring sector
 * when the cluster lies there; clusters further away are left out), and the
 * residuals r_y = y_cl - y, r_z = z_cl - z with the track angles
 * t_y = tan(phi), t_z = tan(lambda)/cos(phi) are summed per voxel
 * (sector, x, y/x, z/x of the track point) as n, sum t_y, sum t_z,
 * sum (t_y^2 + t_z^2), sum r_y, sum r_z, sum (t_y r_y + t_z r_z),
 * sum (r_y^2 + r_z^2).  sums: device [n_vox][8] doubles, ADDED to (zero them
 * before the first batch of a map; several batches accumulate), n_vox =
 * 18 * vox_nx * vox_ny * vox_nz.  Stream-ordered; the summation order is not
 * fixed, so results vary in the last bits.  Errors: TRD_EINVAL, TRD_EDEVICE. */
int trd_residual_sums(trd_ctx *ctx, const trd_reference *ref, const trd_tpc_clusters *cl, int64_t n,
                      int64_t n_cl, double *sums, void *hip_stream);

/* Per voxel distortion vector from the sums: dist[v] = (dX, dY, dZ, n), the
 * least-squares solution of r_y = dY - dX t_y, r_z = dZ - dX t_z (a cluster
 * seen at row x was created at x - dX and displaced by dY, dZ); NaN for voxels
 * with fewer than vox_min clusters.  dist: device [n_vox][4] floats.
 * Stream-ordered.  Errors: TRD_EINVAL, TRD_EDEVICE. */
int trd_voxel_solve(trd_ctx *ctx, const double *sums, float *dist, void *hip_stream);

/* Fills *out with the context's sorted tracklets (valid until the next load
 * or destroy; read them on the load's stream).  Errors: TRD_EINVAL, TRD_ESTATE. */
int trd_get_binning(trd_ctx *ctx, trd_binning_view *out);

/* Copies the context's sorted tracklets into caller device buffers:
 * offsets_out[n_cells + 1] and sorted_out[4 * n_valid] (layout as in
 * trd_binning_view), stream-ordered after the last load.  n_valid is
 * offsets[n_cells]; pass capacity max_valid >= it (use n_tracklets).
 * Errors: TRD_EINVAL, TRD_ESTATE, TRD_EDEVICE. */
int trd_copy_binning(trd_ctx *ctx, uint32_t *offsets_out, float *sorted_out, int64_t max_valid,
                     void *hip_stream);

/* Device memory currently held by the context, in bytes. */
int64_t trd_device_bytes(const trd_ctx *ctx);

/* Durations (ms, from HIP events on the launch stream) of the main match
 * kernel of the last min(calls, 64, max_n) trd_match calls since the
 * previous read, oldest first, into ms[]; waits for them to finish and
 * starts a new count.  Returns how many were written (>= 0), or TRD_ESTATE
 * without TRD_CFG_TIME_KERNEL, TRD_EINVAL, TRD_EDEVICE.  Not for calls
 * captured into a graph. */
int trd_kernel_times(trd_ctx *ctx, float *ms, int32_t max_n);

/* Ends the context of trd_create: frees every device buffer it owns (the
 * sorted tracklets of the last load included, so views from
 * trd_get_binning become invalid) and its events.  Waits for the device to
 * finish its work first.  NULL is a no-op.  Never fails. */
void trd_destroy(trd_ctx *ctx);

/* Static text for a call status code (TRD_OK, TRD_E*): the name of the
 * failure, for logs; "unknown status" for any other value.  The pointer is
 * owned by the library and valid for its lifetime.  Needs no device. */
const char *trd_status_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* TRD_H */

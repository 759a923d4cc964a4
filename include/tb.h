/*
 * tb.h — C ABI of the MI355X (gfx950) temporal-blocking wave-propagation
 * library.
 *
 * The library implements the method of "Temporal blocking of
 * finite-difference stencil operators with sparse off-the-grid sources"
 * (Bisbas et al., arXiv 2010.10248): explicit finite-difference wave
 * propagators whose sparse off-the-grid source injection and receiver
 * interpolation are precomputed by an inspector (Section II-A) into
 * grid-aligned per-point wavelets, so that wave-front temporal blocking
 * (Section II-B) can advance several time steps per pass over memory.
 *
 * Conventions
 *  - Every call returns a tb_status (TB_OK == 0, errors < 0); no C++
 *    exception crosses this boundary. tb_last_error() returns a thread-local
 *    text for the last failure on the calling thread.
 *  - Grids are C-order [nx][ny][nz] float32 with z fastest. "Device" pointers
 *    are HIP device memory on the current device; "host" pointers are
 *    ordinary host memory, read during the call and not retained.
 *  - Streams are passed as void* (a hipStream_t; NULL = the null stream).
 *    Work is enqueued asynchronously; execution errors surface at the
 *    caller's synchronisation.
 *  - Handles are immutable after creation apart from internal caches that
 *    are built under a lock; a handle may be used from several streams.
 */
#ifndef TB_H
#define TB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tb_status;

#define TB_OK 0
#define TB_EINVAL (-1)       /* malformed argument                           */
#define TB_EUNSUPPORTED (-2) /* physics / space order / option not built     */
#define TB_EUNSTABLE (-3)    /* dt exceeds the discrete stability bound      */
#define TB_ERANGE (-4)       /* a sparse coordinate lies outside the grid    */
#define TB_ENOMEM (-5)       /* device or host allocation failed             */
#define TB_EHIP (-6)         /* a HIP runtime call or kernel launch failed   */
#define TB_EWORKSPACE (-7)   /* caller workspace / buffer too small          */

#define TB_ACOUSTIC 0 /* isotropic acoustic, Section III-A                  */
#define TB_TTI 1      /* pseudo-acoustic TTI, Section III-B                 */
#define TB_ELASTIC 2  /* isotropic elastic velocity-stress, Section III-C  */

#define TB_SCHED_SB 0 /* spatial blocking: one time step per pass (Fig. 4a) */
#define TB_SCHED_TB 1 /* wave-front temporal blocking (Fig. 4b, Fig. 7)    */

typedef struct tb_model tb_model;
typedef struct tb_sparse tb_sparse;

/*
 * Model description (equation (acou) of Section III-A, the TTI system of
 * Section III-B, the elastic system of Section III-C; Section IV-B).
 *  shape       grid nodes per axis; the absorbing layers lie inside it.
 *  spacing     h per axis in metres; origin in metres.
 *  space_order 4, 8 or 12 (centred Taylor weights, radius space_order/2).
 *  nbl         absorbing-layer width in nodes (0 = no damping).
 *  dt, nt      time step (s) and number of updates of a forward run.
 *  damp_vmax   velocity used by the damping profile (<= 0: max(vp)).
 *  vp          device float32 [nx][ny][nz] P velocity (m/s); read during the
 *              call only (the library derives its own coefficient arrays).
 *              NULL when slowness2 is given.
 *  epsilon, delta, theta, phi   TTI only (device float32 [nx][ny][nz]):
 *              Thomsen parameters (delta is clipped to epsilon) and the tilt
 *              from vertical / azimuth (radians) of the symmetry axis.
 *  vs, rho     elastic only (device float32 [nx][ny][nz]): S velocity (m/s)
 *              and density (kg/m^3).
 *  slowness2   acoustic only, in place of vp (device float32 [nx][ny][nz]):
 *              the squared slowness m = 1/vp^2 (s^2/m^2) of equation (acou),
 *              the variable tb_gradient differentiates by. The coefficient
 *              is then c = dt^2/m (FP64, rounded once); vp NULL.
 * All parameter arrays are read during the call only.
 */
typedef struct {
    int32_t physics;
    int32_t shape[3];
    double spacing[3];
    double origin[3];
    int32_t space_order;
    int32_t nbl;
    double dt;
    int32_t nt;
    double damp_vmax;
    const float *vp;
    const float *epsilon;
    const float *delta;
    const float *theta;
    const float *phi;
    const float *vs;
    const float *rho;
    const float *slowness2;
} tb_model_desc;

/*
 * Schedule of the time loop (Section II-B; the wave-front loop nest of the
 * last listing). mode TB_SCHED_SB runs one step per pass; TB_SCHED_TB runs
 * time_tile steps per pass with a wave-front along x and overlapped y-z
 * halos. time_tile is 1..4 at space order 4 (4 with tile_y 16 only) and
 * 1..2 at space orders 8 and 12.
 *  tile_y   y rows one workgroup holds: 16 or 32 (16 lanes x 4 z per row),
 *           or 0 for 32 where that shape fits the depth, else 16.
 *  chunk_x  x planes one work segment streams (at most 1024 are used).
 *           Below nx: each (chunk, tile) pair is one segment; one workgroup
 *           per compute unit streams the segments of a slab of neighbouring
 *           tiles, chunk by chunk, with the slabs spread over the XCDs.
 *           nx or more (up to 1024): whole x per tile; with fewer tiles than
 *           compute units, each tile streams a head [0, s) on its own
 *           workgroup and the spare workgroups stream the tails [s, nx), s
 *           chosen to balance the two. 0 splits the tile-x space evenly
 *           over two workgroups per compute unit. A segment whose injection
 *           list exceeds the staged capacity is streamed as consecutive
 *           pieces.
 * TTI and elastic (Section II-B applied to the systems of Sections III-B
 * and III-C): TB_SCHED_TB runs passes of time_tile (1..4) steps over
 * overlapped x-slabs of chunk_x owned planes (0: 32), each step's range
 * shrinking by the skew 2 * radius (the two chained first-derivative stages
 * of a step) from the first to the last step of a pass; tile_y is ignored.
 * TB_SCHED_SB is one step per pass over all of x.
 * Every schedule gives bit-identical results. Passing NULL where a schedule
 * is accepted selects the tuned choice for the model if tb_autotune cached
 * one, else: acoustic TB with time_tile 3 at space order 4, 2 at space order
 * 8 and SB (time_tile 1) at space order 12, tile_y 32, with whole x when nx
 * <= 1024 and the tiles fill at least half the compute units but not all of
 * them, else chunk_x 64 when nx >= 256, else 0; TTI and elastic SB.
 */
typedef struct {
    int32_t mode;
    int32_t time_tile;
    int32_t tile_y;
    int32_t chunk_x;
} tb_schedule;

/* Workspace operations for tb_workspace_size. */
#define TB_OP_FORWARD 0
#define TB_OP_ADJOINT 1
#define TB_OP_GRADIENT 2

/*
 * Create a model: validates the description, computes c = dt^2 vp^2 (or
 * dt^2/m; FP64, rounded once to FP32) and the damping profile into
 * library-owned device memory on the current device. Errors: TB_EINVAL,
 * TB_EUNSUPPORTED (physics, space order; nx above 65535: the sparse-list keys
 * hold x in 16 bits; a padded y-z plane of 2 GiB or more, ny * nzp * 4 >=
 * 2^31 with nzp = nz rounded up to a multiple of 4: the wave-front kernel
 * addresses a plane with 32-bit offsets), TB_EUNSTABLE (vp_max dt exceeds
 * the leapfrog bound of the chosen weights), TB_ENOMEM, TB_EHIP. *out is
 * NULL on failure.
 */
tb_status tb_create_model(const tb_model_desc *desc, tb_model **out);
void tb_destroy_model(tb_model *m);

/*
 * Inspector (Section II-A; the empty-grid injection, mask/ID and
 * decomposition listings). Host inputs: nsrc source coordinates
 * src_xyz[nsrc][3] (m), their wavelets src_wavelet[nt][nsrc] (the value
 * injected at t_n = n dt), and nrec receiver coordinates rec_xyz[nrec][3].
 * Builds the unique affected-point set with ascending IDs, the decomposed
 * per-point wavelets src_dcmp[nt][npts] (summed in FP64, rounded once to
 * FP32) and the receiver mirror, and uploads them. Per-schedule tile lists
 * are built lazily and cached in the handle. Errors: TB_ERANGE (a point
 * outside [origin, origin + (n-1) h]), TB_EINVAL, TB_ENOMEM, TB_EHIP.
 * nsrc or nrec may be 0 (the pointer may then be NULL).
 */
tb_status tb_inspect_sparse(const tb_model *m, int32_t nsrc, const double *src_xyz,
                            const double *src_wavelet, int32_t nrec, const double *rec_xyz,
                            tb_sparse **out);
void tb_destroy_sparse(tb_sparse *s);

/* Sizes of the inspector's products: unique source points, unique receiver
 * points. */
tb_status tb_sparse_counts(const tb_sparse *s, int32_t *npts, int32_t *nrid);

/*
 * Host-only inspector (no device memory touched), for checking the
 * decomposition on a machine without a GPU. vp_host is float32
 * [nx][ny][nz]. On input *npts holds the capacity of nodes[cap][3] and
 * dcmp[nt][cap]; on return it holds the number of unique affected points
 * (TB_EWORKSPACE if it exceeds the capacity; nothing else written then).
 * nodes are listed in ascending raster order (their IDs); dcmp[n][id] =
 * sum_s sum_corner W c(node) q_s(t_n) with c = dt^2 vp^2.
 */
tb_status tb_inspect_host(const int32_t shape[3], const double spacing[3], const double origin[3],
                          double dt, int32_t nt, const float *vp_host, int32_t nsrc,
                          const double *src_xyz, const double *src_wavelet, int32_t *npts,
                          int32_t *nodes, float *dcmp);

/*
 * Host-only view of how an acoustic schedule splits the wave-front loop nest
 * of Section II-B into work (no device memory touched): for a grid `shape`
 * at `space_order` (4, 8 or 12), the schedule `s` (not NULL; mode SB means
 * time_tile 1) and `wgs` resident workgroups (the device launches one per
 * compute unit for chunk_x > 0, two for chunk_x 0). tile[4] receives the
 * tile's rows, its z width, and the rows and z columns it owns (the rest is
 * the overlapped halo). On input *nseg holds the capacity of seg[cap][5]; on
 * return the number of work segments (TB_EWORKSPACE if it exceeds the
 * capacity; seg is then not written). Segment k, in launch order, is
 * seg[k] = {workgroup, tile index along y, tile index along z, xs, xe}: that
 * workgroup streams planes [xs, xe) of that tile (with its x halo). The
 * pieces into which the inspector splits segments with dense injection lists
 * depend on the sparse set and are not shown. Errors: TB_EINVAL (NULL
 * pointer, wgs < 1, shape below 1), TB_EUNSUPPORTED (space order, or no
 * kernel of that shape).
 */
tb_status tb_schedule_segments_host(const int32_t shape[3], int32_t space_order,
                                    const tb_schedule *s, int32_t wgs, int32_t tile[4],
                                    int32_t *nseg, int32_t *seg);

/* Bytes of caller workspace needed by an operation (TB_OP_*). */
tb_status tb_workspace_size(const tb_model *m, const tb_sparse *s, const tb_schedule *sched,
                            int32_t op, size_t *bytes);

/*
 * Forward propagation from zero initial conditions over nt steps
 * (naive-order semantics of the first listing, computed in the order of the
 * chosen schedule). Outputs (device, caller-owned, any may be NULL):
 *  acoustic  rec_out[nt][nrec] with d^n = P_r u^n (so d^0 = 0),
 *            field_out = u^{nt}, field_prev_out = u^{nt-1};
 *  TTI       the same for the field p (the source enters p and r);
 *  elastic   rec_out[2][nt][nrec]: vz^{n-1/2} (interpolated on the vz grid)
 *            then P^n = (txx + tyy + tzz)^n / 3; field_out = vz^{nt-1/2},
 *            field_prev_out = tzz^{nt}.
 * Fields are [nx][ny][nz]. ws must hold tb_workspace_size(TB_OP_FORWARD)
 * bytes of device memory for the same schedule. Every schedule of every
 * physics gives the same bits.
 * Errors: TB_EINVAL, TB_EWORKSPACE, TB_EUNSUPPORTED, TB_EHIP.
 */
tb_status tb_forward(const tb_model *m, const tb_sparse *s, const tb_schedule *sched, void *ws,
                     size_t ws_bytes, float *rec_out, float *field_out, float *field_prev_out,
                     void *stream);

/*
 * tb_forward for callers that cannot allocate (code under stream capture,
 * serving loops or harnesses that forbid device allocation): the same plan
 * and kernels, with the workspace in a fixed 64 MiB device array of the
 * library (one per device it runs on, held until the process ends) instead
 * of caller memory. Outputs as tb_forward. It calls no allocating routine;
 * host bookkeeping only. Limits and errors: TB_EWORKSPACE when the run needs
 * more than 64 MiB (tb_workspace_size(TB_OP_FORWARD); acoustic grids up to
 * about 145^3); TB_EINVAL when the model is not on the current device, when
 * per-launch timing (tb_kernel_timing) is on, or when the schedule's tile
 * lists are not built yet (the first tb_forward of a sparse handle with that
 * schedule builds and uploads them). Every call on a device shares that
 * device's array, and each call clears what it needs: calls that overlap on
 * one device (other streams, other threads) race and must be serialised by
 * the caller.
 */
tb_status tb_forward_noalloc(const tb_model *m, const tb_sparse *s, const tb_schedule *sched,
                             float *rec_out, float *field_out, float *field_prev_out,
                             void *stream);

/*
 * Exact discrete adjoint of the linear map q -> d of tb_forward, driven by
 * rec_in[nt][nrec] at the receiver points; output src_out[nt][nsrc] (device).
 * Used for the dot-product test and for imaging. Acoustic: the forward update
 * run backward in time in the scaled multiplier c lambda / alpha (any
 * schedule). TTI (spatially blocked): the multiplier recursion with the
 * transposed coupling, lambda^k = H D (c/alpha) lambda^{k+1} + (2/alpha)
 * lambda^{k+1} - (beta/alpha) lambda^{k+2} + (P_r^T rec_in^k, 0), H =
 * diag(H0, Hz), D = [[1+2 eps, s], [s, 1]] (the forward couples through D H),
 * and src_out^n = P_s (c (lambda_p + lambda_r)^{n+1}). Elastic (spatially
 * blocked; rec_in is [2][nt][nrec], the vz block then the P block): the two
 * passes of each step reversed with transposed staggered operators (D^T =
 * -E, E^T = -D for the divergence D and strain E with zero outside the
 * grid), and src_out^n = dt P_s (tr of the stress multiplier)^{n+1}.
 */
tb_status tb_adjoint(const tb_model *m, const tb_sparse *s, const tb_schedule *sched, void *ws,
                     size_t ws_bytes, const float *rec_in, float *src_out, void *stream);

/*
 * Gradient of J = 1/2 sum_{n<nt} |P_r u^n - d_obs^n|^2 with respect to the
 * squared slowness m = 1/vp^2, the damping profile held fixed (the exact
 * discrete adjoint of the update of equation (acou); the paper names
 * full-waveform inversion as the use of the adjoint, Section I, and leaves
 * its form open). With nu the adjoint wavefield,
 *   dJ/dm = -(1/dt^2) sum_{k=1}^{nt-1} nu^k (c L u^{k-1} + alpha s^{k-1}),
 * s^{k-1} the injected increment of step k-1 (which carries the dt^2/m
 * source scaling). The call runs the forward pass keeping (u^{jK}, u^{jK-1})
 * every K = checkpoint_every steps (0 = ceil(sqrt(nt)); rounded up to a
 * multiple of the schedule's time_tile), then for each segment in reverse
 * recomputes its levels from the checkpoint and runs the adjoint through it,
 * imaging every level (FP64 accumulation). The recomputed levels are
 * bit-identical to the forward ones, so K does not change the result.
 * d_obs[nt][nrec] device; grad_m [nx][ny][nz] device FP32 (overwritten);
 * loss_out host (may be NULL; when given, the call synchronises the stream to
 * write it). ws must hold tb_gradient_workspace_size(checkpoint_every) bytes
 * (tb_workspace_size(TB_OP_GRADIENT) is the size for checkpoint_every = 0).
 * TTI (spatially blocked; J on the traces of p): with y^k = (c/alpha)
 * lambda^k, lambda the multiplier of tb_adjoint driven by the residual,
 *   dJ/dm = -(1/dt^2) sum_{k=1}^{nt-1} sum_{f=p,r} y_f^k (c (A w^{k-1})_f
 *           + alpha s^{k-1}),  A = D H the coupled operator,
 * eps, delta and the axis held fixed; checkpoints of (p, r, w_p, w_r) every K
 * levels (0 = ceil(sqrt(nt))). Elastic (spatially blocked): J on both
 * trace blocks (d_obs [2][nt][nrec], vz then P), gradient with respect to
 * lambda, mu and b = 1/rho at the nodes into grad_m [3][nx][ny][nz], the
 * stress-pass terms (dt tr(s) tr(e), 2 dt s_ii e_ii, and dt s_c e_c at each
 * shear point shared 1/4 by the four nodes of its mean of mu) and the
 * velocity-pass terms (dt vh_a (div t)_a / alpha at each velocity point,
 * shared 1/2 by the two nodes of its mean of b), s the stress multiplier over
 * alpha and e the strain of the forward velocities; checkpoints of the nine
 * fields every K steps.
 * Errors: TB_EINVAL, TB_EWORKSPACE, TB_EUNSUPPORTED, TB_EHIP.
 */
tb_status tb_gradient(const tb_model *m, const tb_sparse *s, const tb_schedule *sched, void *ws,
                      size_t ws_bytes, const float *d_obs, float *grad_m, double *loss_out,
                      int32_t checkpoint_every, void *stream);

/* Bytes of workspace tb_gradient needs for a given checkpoint interval. */
tb_status tb_gradient_workspace_size(const tb_model *m, const tb_sparse *s,
                                     const tb_schedule *sched, int32_t checkpoint_every,
                                     size_t *bytes);

/*
 * Autotuner (the paper sweeps tile and block sizes per kernel and platform,
 * Section IV-C / Table 1, and leaves the time-tile depth open). Times every
 * valid schedule on the device for `steps` updates of this model and sparse
 * set (zero initial state; no output is written) — acoustic: time_tile,
 * tile_y, chunk_x and, for chunk_x 0, one to three resident workgroups per
 * compute unit (a choice tb_schedule does not express; a NULL schedule
 * gets it); TTI and elastic: time_tile 1..3 and slab widths 16, 32, 64 —
 * caches the fastest per (physics, space order, grid shape) for the process,
 * and returns it. Afterwards a NULL schedule on any model of that key
 * resolves to the tuned choice. Allocates a temporary workspace.
 * Errors: TB_EINVAL, TB_ENOMEM, TB_EHIP.
 */
tb_status tb_autotune(const tb_model *m, const tb_sparse *s, int32_t steps, void *stream,
                      tb_schedule *best, double *ms_per_step);
/* Forget every tuned schedule. */
tb_status tb_autotune_clear(void);

/*
 * Serving runtime (continuous batching of shots on one device).
 *
 * A request is a forward run (traces) or a checkpointed gradient (the
 * forward, residual, adjoint and imaging of tb_gradient) on a caller-created
 * model and sparse set, which must stay alive until the request completes.
 * Requests queue in submission order; the head is admitted when fewer than
 * max_active requests run and its workspace fits in the server's device
 * arena of arena_bytes (allocated once by tb_server_create). Each
 * tb_server_step runs the pending side actions of every admitted request and
 * then an epoch of up to 8 rounds in which every admitted request advances by
 * one propagation pass, the passes of one round that share a kernel shape
 * forming one batched launch (TB_SERVE_GRAPHS: each epoch structure is
 * captured once as a hipGraph and replayed). A request's results are
 * bit-identical to running it alone with tb_forward / tb_gradient and the
 * same schedule. All work runs on the server's own stream; the call blocks
 * at most until the epoch before last has started executing. Completed
 * requests are reported by tb_server_poll (ids and, for gradients, J).
 * A server is not thread-safe; use one per host thread.
 */
typedef struct tb_server tb_server;
typedef struct {
    int32_t op;                /* TB_OP_FORWARD or TB_OP_GRADIENT                   */
    const tb_model *model;
    const tb_sparse *sparse;
    const tb_schedule *sched;  /* read at submission; NULL: tuned, else default    */
    const float *d_obs;        /* gradient: device [nt][nrec]                       */
    float *rec_out;            /* forward: device [nt][nrec] traces, or NULL        */
    float *grad_out;           /* gradient: device [nx][ny][nz] dJ/dm               */
    int32_t checkpoint_every;  /* gradient: as in tb_gradient                       */
} tb_request;

#define TB_SERVE_GRAPHS 1

tb_status tb_server_create(size_t arena_bytes, int32_t max_active, int32_t flags,
                           tb_server **out);
/* Queue a request; *id identifies it in tb_server_poll. TB_EWORKSPACE if its
 * workspace exceeds the arena. */
tb_status tb_server_submit(tb_server *sv, const tb_request *rq, int64_t *id);
/* Admit, run side actions, enqueue one epoch; report running / queued. */
tb_status tb_server_step(tb_server *sv, int32_t *n_active, int32_t *n_queued);
/* Up to cap completed requests (device work finished): ids and losses. */
tb_status tb_server_poll(tb_server *sv, int32_t cap, int64_t *ids, double *losses,
                         int32_t *n_done);
/* Counters: epochs, rounds, batched launches, passes batched, graph captures,
 * graph replays, side actions, completed requests (first n of these 8). */
tb_status tb_server_stats(const tb_server *sv, int64_t *stats, int32_t n);
/* Waits for the server's stream, then frees everything it owns. */
void tb_server_destroy(tb_server *sv);

/*
 * Kernel timing for measurement. While enabled, every propagation kernel
 * launch made by this library (from any thread) is bracketed by HIP events on
 * the stream it is launched on. tb_kernel_timing_read synchronises those
 * events and returns the number of timed launches and their summed device
 * time in milliseconds since the last enable, then keeps counting.
 * Enabling resets the counters; disabling releases the events.
 */
tb_status tb_kernel_timing(int32_t enable);
tb_status tb_kernel_timing_read(int32_t *launches, double *total_ms);

/* Text of the last error on this thread ("" if none). */
const char *tb_last_error(void);

/* Library version string. */
const char *tb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TB_H */

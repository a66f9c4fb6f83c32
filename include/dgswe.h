/*
 * dgswe.h - C ABI of the MI355X (gfx950) nodal discontinuous Galerkin solver
 * for the 2D nonlinear shallow water equations on triangles.
 *
 * Method (Gandham, Medina & Warburton, "GPU accelerated discontinuous
 * Galerkin methods for shallow water equations"):
 *   - conservative SWE with bathymetry source            Section 2, Eq. 2.1-2.3
 *   - nodal DG on Warp & Blend nodes, strong form with
 *     the well-balanced local Lax-Friedrichs flux          Section 3, Eq. 3.2-3.3;
 *                                                          Section 5.1, Eq. 5.1-5.2
 *   - multi-rate Adams-Bashforth 3 over levels that step
 *     with 2^(l-1) dt_min                                  Section 4, Eq. 4.1, Algorithm 4.1
 *   - positivity limiter, then positivity-modified TVB
 *     limiter after every update                           Algorithms 5.1, 5.2; Eq. 5.3
 *
 * Conventions for every call:
 *   - Return value: DG_OK (0) or a negative DG_E* code; the message of the
 *     last failure on the calling thread is returned by dg_last_error().
 *   - Host arrays are owned by the caller and are only read or written during
 *     the call; nothing keeps a pointer to them.
 *   - Device memory is owned by the caller: dg_query_sizes() says how many
 *     bytes the solver needs, the caller allocates one device buffer of at
 *     least that size (256-byte aligned) and hands it over with dg_bind().
 *     The library never frees it.  The solver handle is owned by the caller
 *     and released with dg_destroy().
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     dg_advance() only enqueues work; dg_get_* calls that return device
 *     data synchronise the stream before returning.
 *   - Element order: arrays indexed by element use the caller's element
 *     order of the instance (the library reorders internally).  Nodal arrays
 *     are [K][Np] row-major, node order as returned by dg_node_coords().
 *   - A handle is not thread-safe; calls on one handle must be serialised.
 */
#ifndef DGSWE_H
#define DGSWE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define DG_OK          0
#define DG_EINVAL     -1  /* bad argument (null pointer, out-of-range value)       */
#define DG_EMESH      -2  /* malformed mesh: clockwise/degenerate element, face    */
                          /* shared by more than two elements, inconsistent faces  */
#define DG_ENOMEM     -3  /* host allocation failed or bound buffer too small      */
#define DG_EDEVICE    -4  /* a HIP runtime call failed                             */
#define DG_ENOTBOUND  -5  /* device buffer not bound, or state not set             */
#define DG_ENUMERIC   -6  /* non-finite value in input or state                    */
#define DG_ESTATE     -7  /* call not valid in the current state                   */

/* contraction / kernel path (dg_params.precision) */
#define DG_PLAIN_FP32     0  /* separate RHS, update and limiter kernels, FP32 VALU  */
#define DG_FUSED_FP32     1  /* fused RHS+AB3+positivity kernel, FP32 VALU matvecs   */
#define DG_FUSED_MFMA32   2  /* fused kernel, [Dr Ds LIFT] contraction on FP32 MFMA  */
                             /* (N <= 5)                                           */
#define DG_FUSED_BF16X3   3  /* fused kernel, BF16 MFMA, operands split in 2 parts,  */
                             /* 3 products, FP32 accumulate (N <= 5)               */
#define DG_FUSED_BF16X6   4  /* fused kernel, BF16 MFMA, operands split in 3 parts,  */
                             /* 6 products, FP32 accumulate (N <= 5)               */

/* limiter switches (dg_params.limiter_mask) */
#define DG_LIMIT_PP   1      /* positivity limiter, Algorithm 5.2         */
#define DG_LIMIT_TVB  2      /* TVB limiter with Eq. 5.3                  */

/* per-element flag byte: bits 0-1 positivity code, bits 2-3 TVB code */
#define DG_PP_KEEP     0     /* min nodal depth above eps: untouched      */
#define DG_PP_SCALED   1     /* P1 projection scaled about the mean       */
#define DG_PP_DRY      2     /* mean depth below h0: element set dry      */
#define DG_TVB_SKIPPED 0     /* dry element or neighbour of a dry element */
#define DG_TVB_KEPT    1     /* no characteristic component limited       */
#define DG_TVB_LIMITED 2     /* limited to P1                             */
#define DG_TVB_POSITIVE 3    /* limited, depth increments rescaled by Eq. 5.3 */

typedef struct dg_solver dg_solver;

/* One triangulated instance.  vx, vy: n_vertices coordinates.  etov:
 * n_elements x 3 vertex indices, counter-clockwise.  Faces not shared with a
 * second element are reflective walls.  Face f of an element joins its
 * vertices f and f+1 (mod 3). */
typedef struct dg_mesh_desc {
    int32_t n_vertices;
    const double* vx;
    const double* vy;
    int32_t n_elements;
    const int32_t* etov;
    /* optional per-face boundary tags, K x 3 in the order of etov's faces
     * (face f joins vertices f and f+1): 0 = interior where another element
     * shares the face, wall otherwise; 1 = reflective wall even where the
     * face is shared (both sides become walls: an internal barrier).  NULL
     * = all 0.  Any other value is DG_EMESH.  Copied during dg_create. */
    const int8_t* bc;
} dg_mesh_desc;

typedef struct dg_params {
    int32_t N;              /* polynomial degree, 1..6                                */
    double g;               /* gravity                                                */
    double cfl;             /* dt_k = cfl * r_k / ((N+1)^2 a_max), Eq. 4.1             */
    double h0;              /* dry threshold of Algorithm 5.2 and Eq. 5.3 (> 0)        */
    double eps;             /* positivity trigger: limit when min nodal h <= eps      */
    double hvel;            /* velocity u = 2 h hu / (h^2 + max(h^2, hvel^2)): hu/h   */
                            /* for h >= hvel, continuous to 0 at h = 0 (> 0)          */
    double tvb_M;           /* TVB constant M (minmod bypass when |a| <= M d_K^2)      */
    double tvb_nu;          /* TVB factor on the neighbour difference (>= 1)          */
    int32_t limiter_mask;   /* DG_LIMIT_* bits                                        */
    int32_t max_levels;     /* multi-rate levels (1 = single rate AB3), 1..6          */
    int32_t precision;      /* DG_PLAIN_FP32 .. DG_FUSED_BF16X6                        */
    int32_t dry_literal;    /* 1: dry element gets h = h0 (Algorithm 5.2 as printed); */
                            /* 0: h = max(mean, 0), which conserves mass              */
    int32_t use_graph;      /* 1: replay dg_advance steps from a captured hipGraph    */
    int32_t elems_per_block;/* 0 = default for N and path; matrix-core paths: 1, 2, 4 */
                            /* or 8 waves of 64/lanes elements (N = 1, 2, 4: 4, 8,    */
                            /* 16, 32; N = 3: 5, 10, 20, 40; N = 5: 3, 6, 12, 24),    */
                            /* default 8 waves at N = 3, 5, else 4; VALU paths:       */
                            /* floor(256 / Np); anything else is DG_EINVAL            */
    double thin_cut;        /* >= 0; > 0: after the limiters, momentum is set to zero */
                            /* at nodes whose depth is below thin_cut (thin films at  */
                            /* shorelines; the paper is silent there).  0 = off       */
    int32_t overint;        /* 0: nodal collocation (strong form, Dr/Ds and LIFT on   */
                            /* the nodes); 1: the weak form of Eq. 3.2 with volume    */
                            /* integrals by cubature and face integrals by Gauss      */
                            /* quadrature, both exact to degree 3N (Section 3 and the */
                            /* Volume/Surface kernels of Section 7): N <= 5, on        */
                            /* DG_PLAIN_FP32, DG_FUSED_FP32 (vector ALU) or            */
                            /* DG_FUSED_MFMA32 (matrix cores); other paths DG_EINVAL   */
    int32_t regroup_every;  /* multi-rate only (max_levels >= 2): 0 = levels fixed    */
                            /* from the mesh (Section 4); >= 3 = levels from every    */
                            /* element's own wave speed (Eq. 4.1 per element, its     */
                            /* nodes and face neighbours), at dg_prepare and again    */
                            /* every regroup_every coarse steps (the option named     */
                            /* after Algorithm 4.1).  At a regroup each element's AB  */
                            /* history is re-sampled at its new step from the         */
                            /* quadratic through it; graph replay is off.  1, 2 or    */
                            /* < 0 is DG_EINVAL                                        */
} dg_params;

/* Fill *p with the defaults: g 9.81, cfl 0.5, h0 = eps = 1e-5, hvel 1e-3, M 10, nu 1.5,
 * both limiters, single rate, DG_FUSED_FP32, mass-conserving dry branch,
 * graphs on, no thin-film momentum cut. */
int32_t dg_default_params(int32_t N, dg_params* p);

/* Validate and set up n_inst instances (n_inst > 1: an ensemble advanced
 * together, each with its own dt; 1 <= n_inst <= 2^23): the reference element
 * on Warp & Blend nodes with Dr, Ds and LIFT, the face connectivity and the
 * affine geometric factors (Section 3), the multi-rate levels from the element
 * sizes (Section 4, Eq. 4.1) and the TVB stencil of every edge (Section 5.3).
 * meshes[n_inst] and p are read during the call only.  Host only; no device
 * work.  Errors: DG_EINVAL (null/size, parameter out of range), DG_EMESH (see
 * above), DG_ENOMEM. */
int32_t dg_create(const dg_mesh_desc* meshes, int32_t n_inst, const dg_params* p,
                  dg_solver** out);

/* Release the handle (not the caller's device buffer).  NULL is a no-op.
 * Waits first for the work the solver queued on its own stream (graph
 * replays of dg_advance), so that the caller may free or reuse the device
 * buffer as soon as this returns; work queued on the caller's stream is
 * ordered by that stream as usual. */
void dg_destroy(dg_solver* h);

/* Message of the last failed call on this thread ("" if none). */
const char* dg_last_error(void);

/* Sizes: total elements, Np, Nfp, and the device bytes dg_bind needs (any
 * pointer may be NULL).  Errors: DG_EINVAL (null handle). */
int32_t dg_query_sizes(const dg_solver* h, int64_t* total_elements, int32_t* Np,
                       int32_t* Nfp, int64_t* workspace_bytes);

/* Bind caller-owned device memory (>= workspace_bytes, 256-byte aligned) on
 * the current HIP device, and upload the static setup data on `stream`.
 * Errors: DG_EINVAL (null/misaligned), DG_ENOMEM (too small), DG_EDEVICE. */
int32_t dg_bind(dg_solver* h, void* device_workspace, int64_t bytes, void* stream);

/* Number of elements of instance `inst`. */
int32_t dg_instance_elements(const dg_solver* h, int32_t inst, int32_t* K);

/* Physical node coordinates of instance `inst`, [K][Np] each (host): the
 * Warp & Blend nodes of the reference triangle mapped affinely onto each
 * element (Section 3).  Errors: DG_EINVAL. */
int32_t dg_node_coords(const dg_solver* h, int32_t inst, double* x, double* y);

/* Reference nodes r, s (Np each) and operators of Section 3 (Eq. 3.3; the
 * over-integrated ones of the weak form, Eq. 3.2, as the Volume and Surface
 * kernels of Section 7 apply them), row-major, FP64, host arrays:
 * which = 0: Dr (Np x Np), 1: Ds (Np x Np), 2: LIFT (Np x 3Nfp),
 * 3: mass matrix (Np x Np), 4: cell-integral weights w (Np),
 * 5: face node indices (3 x Nfp, as doubles).
 * Over-integrated weak form (any solver; q = (3N+2)/2, Ncub = q^2, NG = q):
 * 6: cubature nodes and weights (3 x Ncub: r, s, w), 7: basis at the
 * cubature nodes Ic (Ncub x Np), 8: Pr, 9: Ps, 10: P (Np x Ncub each),
 * 11: Gauss points and weights on [-1, 1] (2 x NG), 12: face-node basis at the
 * Gauss points I1 (NG x Nfp), 13: L^g (Np x 3NG).  DG_EINVAL for other ids. */
int32_t dg_reference(const dg_solver* h, int32_t which, double* out);
int32_t dg_reference_nodes(const dg_solver* h, double* r, double* s);

/* Bed elevation B at the nodes of instance `inst` ([K][Np], host, FP64): the
 * bathymetry of the source term of Eq. 2.3 and of the face reconstruction of
 * Eq. 5.1.  Must come before dg_set_state of the instance.  Errors: DG_EINVAL,
 * DG_ENUMERIC (non-finite value). */
int32_t dg_set_bathymetry(dg_solver* h, int32_t inst, const double* B);

/* Initial depth and momenta of instance `inst` ([K][Np] each, host, FP64).
 * The time step of the instance is set from the wave speed
 * max |u| + sqrt(g h) of this data (Eq. 4.1).  Once every instance has its
 * state (and bathymetry), the first dg_advance applies Q0 = TVB(PP(Q0))
 * (Algorithm 5.1, first line); setting any state resets the time stepping.
 * Errors: DG_ENOTBOUND (no buffer bound), DG_ESTATE (bathymetry of the
 * instance not set yet), DG_ENUMERIC (non-finite or negative depth),
 * DG_EINVAL. */
int32_t dg_set_state(dg_solver* h, int32_t inst, const double* hh, const double* hu,
                     const double* hv, void* stream);

/* Apply the initial limiting Q0 = TVB(PP(Q0)) of Algorithm 5.1 now, on
 * `stream` (otherwise done by the first dg_advance); with regrouping, also
 * the initial levels from the staged state's wave speeds (Section 4, after
 * Algorithm 4.1).  Errors: DG_ENOTBOUND (no buffer, or an instance without
 * state or bathymetry), DG_EDEVICE. */
int32_t dg_prepare(dg_solver* h, void* stream);

/* Enqueue n_steps steps on `stream`: single-rate AB3 steps, or with
 * max_levels > 1 coarse steps of multi-rate AB3 (2^(L-1) ticks of dt_min,
 * Algorithm 4.1).  Each step: the right-hand side of Eq. 3.3 with the flux of
 * Eq. 5.1-5.2, the Adams-Bashforth update, the positivity limiter of
 * Algorithm 5.2 and the TVB limiter with Eq. 5.3 (Algorithm 5.1).  Returns
 * once the work is queued.  Errors: DG_ENOTBOUND (state not set), DG_EINVAL
 * (n_steps < 0), DG_EDEVICE. */
int32_t dg_advance(dg_solver* h, int32_t n_steps, void* stream);

/* Autotuner (launch shape of the step kernel; the paper tunes the number of
 * elements per work-group by hand, Section 7.4).  Times the step kernel of
 * the next tick `reps` times for each elements-per-block candidate of the
 * path (matrix-core paths: 1, 2, 4 and 8 waves, see elems_per_block; the VALU
 * paths have one shape) and
 * keeps the fastest in the solver's parameters.  The state, history, flags
 * and counters are left as they were.  Writes min(max_out, candidates) pairs (elements per
 * block, average microseconds) to epb/us and the candidate count to *n_out.
 * Synchronises `stream`.  Needs a prepared state (dg_prepare or an earlier
 * dg_advance).  Errors: DG_EINVAL, DG_ENOTBOUND, DG_EDEVICE. */
int32_t dg_autotune(dg_solver* h, int32_t reps, int32_t max_out, int32_t* n_out, int32_t* epb,
                    double* us, void* stream);

/* Current state of instance `inst` as FP64 depth and momenta ([K][Np],
 * host): the conserved variables h, hu, hv of Eq. 2.1 at the nodes.  On the
 * device the surface level is an FP32 pair hi + lo (relative to a
 * per-instance datum) and the momenta are FP32.  Synchronises `stream`.
 * Errors: DG_EINVAL, DG_ENOTBOUND (no state on the device), DG_EDEVICE. */
int32_t dg_get_state(dg_solver* h, int32_t inst, double* hh, double* hu, double* hv,
                     void* stream);

/* Face connectivity of instance `inst` in its own element numbering
 * (Section 3: the exterior trace of face f comes from face etof of element
 * etoe, its nodes in reverse order): etoe[K][3] (the element itself for a wall
 * face), etof[K][3].  Host only.  Errors: DG_EINVAL. */
int32_t dg_get_connectivity(const dg_solver* h, int32_t inst, int32_t* etoe, int8_t* etof);

/* Multi-rate level (1 = finest) of every element of instance `inst`, and the
 * instance's dt_min (0 before its state is set), as Section 4 and Eq. 4.1
 * assign them; with regrouping, the current levels and step (from dg_prepare
 * on).  Either pointer may be NULL.  Host only.  Errors: DG_EINVAL. */
int32_t dg_get_levels(const dg_solver* h, int32_t inst, int8_t* level, double* dt_min);

/* TVB stencil of instance `inst`: pair[K][3][2] face indices used for edge i,
 * alpha[K][3][2] coefficients (Section 5.3).  Host only.  Errors: DG_EINVAL. */
int32_t dg_get_tvb_stencil(const dg_solver* h, int32_t inst, int8_t* pair, double* alpha);

/* Per-element flag bytes (see DG_PP_* / DG_TVB_*) from the last limiter pass
 * (Algorithm 5.2 and Section 5.3), flags[K] in the instance's element order.
 * Synchronises `stream`.  Errors: DG_EINVAL, DG_ENOTBOUND, DG_EDEVICE. */
int32_t dg_get_flags(dg_solver* h, int32_t inst, uint8_t* flags, void* stream);

typedef struct dg_diag {
    double mass;            /* sum_k J_k w.h_k (FP64)                        */
    double min_depth;       /* min nodal h                                    */
    double time;            /* simulated time of the instance                 */
    int64_t steps;          /* steps (coarse steps) taken since set_state     */
    int64_t negative_means; /* positivity-limiter passes that met mean h < 0  */
    int64_t pp_counts[3];   /* elements per DG_PP_* code, last limiter pass   */
    int64_t tvb_counts[4];  /* elements per DG_TVB_* code, last limiter pass  */
} dg_diag;

/* Deterministic FP64 reductions over instance `inst` (the mass that the
 * positivity limiter conserves, Section 5.2; the minimum depth; the limiter
 * branch counts), in a fixed order so that repeated calls agree bit for bit.
 * Synchronises `stream`.  Errors: DG_EINVAL, DG_ENOTBOUND, DG_EDEVICE. */
int32_t dg_get_diagnostics(dg_solver* h, int32_t inst, dg_diag* d, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops): the reductions of dg_get_diagnostics, enqueued on `stream`
 * without allocating, synchronising or copying to the host.  Writes 9 doubles
 * to device memory `out_device` (8-byte aligned, caller-owned): mass,
 * min_depth, pp_counts[3], tvb_counts[4] (counts as doubles), equal to the
 * fields of dg_get_diagnostics for the same state.  The per-block partial
 * sums go to a fixed device array of the library (256 x 16 doubles, 32 KiB,
 * held on each device it runs on until the process ends); their count does
 * not depend on the element count, so every solver size fits.  Calls that
 * overlap on one device share that array and race.  The state buffers are the
 * ones the schedule points to when the call is made.  Errors: DG_EINVAL (bad
 * argument, misaligned out_device), DG_ENOTBOUND (no state yet), DG_EDEVICE
 * (launch or symbol lookup failed). */
int32_t dg_get_diagnostics_noalloc(dg_solver* h, int32_t inst, double* out_device, void* stream);

/* Checkpoint: the full time-stepping state (states, RHS history, half-step
 * traces, counters) as an opaque byte blob; dg_checkpoint_bytes gives the
 * size: a 256-byte header (solver shape, the multi-rate schedule state, the
 * step and finest-level tick counts), one 48-byte record per instance (the
 * vertical datum its stored levels are relative to, its time step, its
 * initial wave-speed bound, a hash of its FP64 bathymetry, and its time
 * origin at the last regroup), every element's multi-rate level, then the
 * device state; any number of instances.  Restoring onto a solver created
 * with the same meshes, params and bathymetry continues bit-identically,
 * single-rate, multi-rate or regrouping, whatever state dg_set_state staged on
 * it: the restore takes the datum, time step and levels of every instance
 * from the blob (rebuilding the shifted bed and, for regrouped levels, the
 * element order on the device).  A later dg_prepare returns to the staged
 * state.  Both synchronise `stream`.  Errors: DG_EINVAL for a buffer shorter
 * than dg_checkpoint_bytes, a blob of another solver shape (K, Np, levels,
 * instances) or bathymetry, or a corrupt blob (schedule state outside its
 * ranges, negative counts, a non-finite or non-positive instance record, a
 * level out of range), each detected before anything is copied;
 * dg_get_checkpoint DG_ENOTBOUND before any state is on the device;
 * dg_set_checkpoint DG_ESTATE before dg_prepare or dg_advance. */
int32_t dg_checkpoint_bytes(const dg_solver* h, int64_t* bytes);
int32_t dg_get_checkpoint(dg_solver* h, void* blob, int64_t bytes, void* stream);
int32_t dg_set_checkpoint(dg_solver* h, const void* blob, int64_t bytes, void* stream);

/* Device timing of the step and TVB kernels.  dg_set_profiling(h, 1) starts
 * a timed region (and resets it): every later tick of dg_advance runs eagerly
 * with start/stop events stamped by the dispatch of its step kernel and of
 * its TVB kernel, on the stream they run on.  dg_kernel_timing(h, which, ...)
 * returns, for which = 0 (step kernel) or 1 (TVB kernel), the average
 * duration in microseconds and the number of timed launches, and the average
 * number of elements per timed launch (all elements single rate; the active
 * levels of each tick with multi-rate stepping; the TVB kernel of a tick
 * covers the same range).  Synchronises on the recorded events.  Errors:
 * DG_EINVAL (null handle, unknown kernel id), DG_EDEVICE. */
int32_t dg_set_profiling(dg_solver* h, int32_t on);
int32_t dg_kernel_timing(const dg_solver* h, int32_t which, double* avg_us, int64_t* launches,
                         int64_t* elements_per_launch);

/* Capture the replay graph of dg_advance now, from the current schedule
 * state, without running any step: the next six coarse steps (the period of
 * the RHS ring and the state ping-pong) are recorded on the library's stream
 * and instantiated, so that a later dg_advance of six or more steps from the
 * same schedule position replays them without paying for capture.  Needs the
 * Adams-Bashforth start-up to be over (two steps advanced since dg_prepare)
 * and use_graph = 1.  Synchronises `stream`.  Errors: DG_EINVAL (null
 * handle), DG_ESTATE (start-up not over, graphs off), DG_EDEVICE. */
int32_t dg_capture_graph(dg_solver* h, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DGSWE_H */

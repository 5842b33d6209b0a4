/*
 * alp.h -- C ABI of libalp, an MI355X (gfx950) implementation of the
 * actuator-line coupling operator of Taran, Bali, Tukovic, Pakrashi and
 * Cardiff, "Two-way actuator-line coupling of a geometrically exact
 * finite-volume beam with incompressible and free-surface flow"
 * (arXiv 2609.39443), Section 3.2.
 *
 * Per coupling step the operator
 *   1. samples the Eulerian velocity upstream of every actuator point
 *      (eq. 16-18, Sec. 3.2.2),
 *   2. evaluates the quasi-steady Morison drag on the relative velocity and
 *      relaxes it (eq. 19-20, Sec. 3.2.3),
 *   3. projects the equal and opposite force onto the mesh through the
 *      truncated Gaussian of eq. (22), normalised per actuator node so that the
 *      transferred resultant force is conserved exactly (eq. 21-23, Sec. 3.2.4).
 *
 * Conventions (all entry points)
 *   - Every array argument is DEVICE memory unless marked HOST, contiguous,
 *     row-major, little-endian, owned by the caller.  [n][3] means n rows of
 *     (x, y, z) doubles.  Indices are 0-based.  An array of zero rows may be
 *     NULL (a case without beams needs no per-point array; its step writes a
 *     zero source).
 *   - The library owns contexts, meshes and workspace.  It keeps no pointer to
 *     caller arrays beyond a call, except where a captured graph replays
 *     (alp_step_batched with ALP_USE_GRAPH): then the arrays named in the cases
 *     must stay valid until alp_invalidate or alp_destroy.
 *   - All calls are asynchronous on the context's stream except alp_create,
 *     alp_bin_cells, alp_get_diag, alp_destroy and alp_mesh_destroy, which
 *     synchronise it.  Calls on one context must not overlap.
 *   - Errors the host can detect return a negative alp_status and launch
 *     nothing; alp_last_error() then describes the problem.  Conditions for
 *     which the method defines a behaviour are not errors: a point outside the
 *     fluid domain carries no load (Sec. 3.2.5), an ill-conditioned upstream
 *     direction falls back to the prescribed one (Sec. 3.2.2), a node that
 *     catches no cell gets no load (Sec. 3.2.4).  They are counted in alp_diag.
 *   - Units are SI.  S is a force per unit volume on the fluid (N/m^3) that
 *     integrates as sum_j S_j V_j; f is the force per unit length on the beam.
 *   - Readings of the paper used throughout: f = +1/2 rho d |U_r| (Cdn U_n +
 *     Cdt U_t) acts on the beam (the printed minus sign of eq. 19 contradicts
 *     eq. 6, eq. 23 and the conservation statement of Sec. 3.2.4); Delta s_k is
 *     the CV length L_k; c(x) is the nearest cell centre (ties: smaller
 *     (x, y, z), then smaller index); the cutoff is inclusive; eps is given per
 *     actuator point and interpolated with the linear weights of Sec. 3.2.4;
 *     beams are normalised independently and their sources add.
 */
#ifndef ALP_H
#define ALP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct alp_context alp_context; /* opaque: stream, workspace, graphs, diagnostics */
typedef struct alp_mesh alp_mesh;       /* opaque: binned copy of a static mesh */

typedef enum {
  ALP_OK = 0,
  ALP_ERR_INVALID_ARG = -1, /* NULL required pointer, bad size, bad enum, eps <= 0, ... */
  ALP_ERR_HIP = -2,         /* HIP runtime failure (details in alp_last_error) */
  ALP_ERR_OOM = -3,         /* device allocation failed */
  ALP_ERR_CAPTURE = -4,     /* call not allowed while the stream is capturing */
  ALP_ERR_SHAPE = -5,       /* shapes changed after graph capture without alp_invalidate */
  ALP_ERR_CAPACITY = -6     /* a per-step work list overflowed; results of that step are invalid */
} alp_status;

typedef enum {
  ALP_PREC_FP64 = 0,      /* everything in FP64 */
  ALP_PREC_FP32_SPLIT = 1 /* kernel weights eta and linear weights omega in FP32; every
                             geometric decision, sum and normalisation in FP64 */
} alp_precision;

typedef enum {
  ALP_DRAG_FULLMAG = 0,      /* eq. (19): 1/2 rho d |U_r| (Cdn U_n + Cdt U_t) */
  ALP_DRAG_COMPONENTWISE = 1 /* eq. (6):  1/2 rho d (Cdn |U_n| U_n + Cdt |U_t| U_t) */
} alp_drag_form;

typedef enum {
  ALP_SAMPLE_CELL = 0,  /* eq. (18): the value of the cell holding P_s */
  ALP_SAMPLE_KERNEL = 1 /* volume average about P_s with the profile of eq. (22):
                           U_s = sum_j g_j V_j U_j / sum_j g_j V_j over the cells with
                           |C_j - P_s| <= 3 eps_k, g_j = exp(-|C_j - P_s|^2 / eps_k^2)
                           (the volume-average sampling named as future work in
                           Sec. 8); with no cell in reach the eq. (18) value is used
                           and counted in alp_diag.n_sample_empty */
} alp_sample_mode;

typedef enum {
  ALP_PROJ_NEAREST = 0,   /* eq. (21)-(23): each (cell, beam) pair takes the closest segment's
                             foot, the 2D Gaussian of eq. (22) at the radial distance and the
                             linear weights (1 - s, s) */
  ALP_PROJ_INTEGRATED = 1 /* the segment-integrated kernel proposed in Sec. 8 to remove the
                             seams of the nearest-segment rule: a cell takes a contribution
                             from EVERY segment i whose closed segment lies within 3 eps_seg of
                             it (inclusive, on the squared distance of eq. 21's clamped foot),
                             eps_seg = (eps_i + eps_i+1)/2, with the 3D Gaussian
                             exp(-|x|^2/eps^2)/(pi^1.5 eps^3) integrated along the segment
                             against the linear weights: a_i = int (1 - u/l) g du,
                             a_i+1 = int (u/l) g du.  Along a straight line the sum over
                             segments is eq. (22).  Zero-length segments contribute nothing;
                             single-CV beams keep the point kernel.  The normalisation of
                             Sec. 3.2.4 and eq. (23) are unchanged (exact balance). */
} alp_proj_mode;

/* The beam set (Sec. 3.2.2): one actuator point per beam control volume.
   Beams are a CSR over points: beam b owns points offsets[b] .. offsets[b+1]-1,
   ordered along the centreline.  All pointers are DEVICE pointers. */
typedef struct {
  int32_t n_beams;
  int32_t reserved0;
  int64_t n_points;
  const int64_t *offsets; /* [n_beams+1], offsets[0] = 0, non-decreasing, last = n_points */
  const double *P;        /* [n_points][3] actuator points P_a (eq. 15) used for sampling */
  const double *P_spread; /* [n_points][3] positions for the projection (Algorithm 1, the
                             projection step uses the updated positions), or NULL = P */
  const double *e_t;      /* [n_points][3] centreline tangents, normalised internally; a zero
                             tangent is an error */
  const double *Pdot;     /* [n_points][3] actuator-point velocities (eq. 13) */
  const double *d;        /* [n_points] drag reference length (diameter) */
  const double *L;        /* [n_points] CV length L_k = Delta s_k */
  const double *eps;      /* [n_points] kernel width eps > 0 (eq. 22) */
  const double *Cdn;      /* [n_beams] normal drag coefficient */
  const double *Cdt;      /* [n_beams] tangential drag coefficient */
  const double *ls;       /* [n_beams] sampling distance l_s (eq. 17) */
  const double *n_p;      /* [n_beams][3] plane normal of eq. (17), unit, or zero = none */
  const double *e_up;     /* [n_beams][3] fallback upstream direction (Sec. 3.2.2) */
  /* Optional Morison inertia, eq. (8), evaluated by alp_step_batched when A and
     the case's fluid acceleration dUdt are both given:
       f_a = rho A (CMt a_rt + CMn a_rn + a_f),  a_r = a_f - a_b
     (relative acceleration fluid minus beam, as U_r in eq. 16 and 19; the
     printed a_b - a_f would make the added-mass reaction push a beam along its
     own acceleration), a_f = dUdt sampled at P_s like U_s, added to the drag
     before the relaxation of eq. (20).  All NULL: drag only, as in the paper. */
  const double *A;        /* [n_points] cross-section area, or NULL (no inertia) */
  const double *CMn;      /* [n_beams] normal added-mass coefficient (required with A) */
  const double *CMt;      /* [n_beams] tangential added-mass coefficient (required with A) */
  const double *a_b;      /* [n_points][3] beam acceleration, or NULL = 0 */
} alp_beams;

typedef struct {
  double rho;      /* fluid density > 0 */
  double alpha_f;  /* relaxation factor of eq. (20) in (0, 1]; used only when f_prev != NULL */
  double tau;      /* fallback threshold on |u0_n| [m/s] (Sec. 3.2.2), >= 0: the fallback
                      direction is used where |u0_n| < tau, and always where u0_n is
                      exactly zero (eq. 17 has no direction there); with tau = 0 only
                      the latter */
  int32_t prec;    /* alp_precision */
  int32_t drag_form; /* alp_drag_form */
  int32_t sample_mode; /* alp_sample_mode */
  int32_t proj_mode;   /* alp_proj_mode */
} alp_params;

/* Diagnostics of the last step of a case (written on the device, read by
   alp_get_diag). */
typedef struct {
  int64_t n_outside;             /* points whose actuator or sampling point left the domain */
  int64_t n_fallback;            /* points that used the fallback direction */
  int64_t n_fallback_degenerate; /* fallback direction parallel to the tangent: e_s = 0 */
  int64_t n_zero_weight;         /* nodes with w_k = 0 (no load transferred) */
  int64_t n_band_cells;          /* cells that received a source */
  int64_t n_pairs;               /* pairs inside the 3 eps cutoff: (cell, beam) pairs, or
                                    (cell, segment) pairs under ALP_PROJ_INTEGRATED */
  int64_t n_overflow;            /* work-list overflow flags (non-zero: results invalid) */
  int64_t n_invalid;             /* points with eps <= 0, a zero tangent or non-finite data */
  double F_beam[3];   /* sum_k f_k L_k  (force on the beam, eq. 14) */
  double F_fluid[3];  /* sum_j S_j V_j  (force on the fluid, eq. 14) */
  double cons_rel_err; /* |F_fluid + F_beam| / sum_k |f_k L_k| */
  int64_t n_sample_empty; /* ALP_SAMPLE_KERNEL points with no cell within 3 eps of P_s */
  int64_t n_guard_fp64;   /* (cell, beam) candidates whose closest segment the FP32 ranking
                             could not single out within its proven error bound, so that more
                             than one segment was evaluated in FP64 (nearest-segment rule) */
} alp_diag;

/* Create a context on HIP device `device` that launches on `hip_stream`
   (a hipStream_t, or NULL for the null stream).  Synchronous. */
alp_status alp_create(int device, void *hip_stream, alp_context **out);
/* Free the context, its workspace and captured graphs.  Synchronous. */
alp_status alp_destroy(alp_context *ctx);
/* Text of the last error on this context ("" if none).  Valid until the next call. */
const char *alp_last_error(const alp_context *ctx);

/* Bin a static mesh once (the paper builds its search structure once at the
   start of the run, Sec. 3.2.5): a uniform spatial hash of the cell centres,
   the cell ids sorted by (tile, bin) with a stable LDS radix sort (a bin's
   cells in caller order), bin CSR, sorted FP64 centres and volumes, and the
   permutation back to the caller's order.  The sorted layout is checked on
   the device against the keys and the CSR; a failed check returns
   ALP_ERR_HIP.
     n_cells     >= 1, < 2^31
     C           DEVICE [n_cells][3] cell centres
     V           DEVICE [n_cells] cell volumes (> 0)
     domain_box  HOST [6] (lo x,y,z, hi x,y,z) or NULL = AABB of the centres
                 inflated by half the largest V^(1/3); points outside it carry no load
     bin_size    > 0, or <= 0 for the cube root of the mean cell volume
     tile_bins   bins per tile edge (1..8), or 0 for the default (4)
   The mesh keeps its own copies; C and V may be freed afterwards.  Synchronous. */
alp_status alp_bin_cells(alp_context *ctx, int64_t n_cells, const double *C, const double *V,
                         const double *domain_box, double bin_size, int32_t tile_bins,
                         alp_mesh **out);
alp_status alp_mesh_destroy(alp_mesh *mesh);

/* Eq. (16)-(18): locate each actuator point, build the upstream sampling point,
   locate it and sample the velocity of that single cell.
     U       DEVICE [n_cells][3] velocity in the caller's cell order
     U_s     DEVICE out [n_points][3] sampled velocity (0 for points outside)
     P_s     DEVICE out [n_points][3] sampling points, or NULL
     cell_a  DEVICE out [n_points] cell of P_a (caller's order, -1 outside), or NULL
     cell_s  DEVICE out [n_points] cell of P_s (-1 outside), or NULL  */
alp_status alp_sample(alp_context *ctx, const alp_mesh *mesh, const double *U,
                      const alp_beams *beams, const alp_params *params, double *U_s,
                      double *P_s, int64_t *cell_a, int64_t *cell_s);

/* Eq. (19) (or eq. 6) and eq. (20): line force on the beam from the sampled
   velocity.  cell_s (nullable) marks points without a sample (< 0): they carry
   no load.  f_prev (nullable) enables relaxation with params->alpha_f.
     f  DEVICE out [n_points][3]  */
alp_status alp_drag(alp_context *ctx, const alp_beams *beams, const alp_params *params,
                    const double *U_s, const int64_t *cell_s, const double *f_prev, double *f);

/* Eq. (21)-(23) and Sec. 3.2.4: nodal weights, normalised forces and the
   momentum source, using beams->P_spread (or P).
     f     DEVICE [n_points][3] line force on the beam
     S     DEVICE out [n_cells][3] source in the caller's order; every cell is
           written (zero outside the 3 eps band)
     w     DEVICE out [n_points] nodal weights w_k, or NULL
     fhat  DEVICE out [n_points][3] normalised nodal forces f_k L_k / w_k, or NULL  */
alp_status alp_spread(alp_context *ctx, const alp_mesh *mesh, const alp_beams *beams,
                      const alp_params *params, const double *f, double *S, double *w,
                      double *fhat);

/* One independent coupling case of a batch.  Outputs other than f and S are
   nullable. */
typedef struct {
  const alp_mesh *mesh;
  const double *U;      /* DEVICE [n_cells][3] */
  alp_beams beams;
  alp_params params;
  const double *f_prev; /* DEVICE [n_points][3] or NULL (no relaxation) */
  double *f;            /* DEVICE out [n_points][3] */
  double *S;            /* DEVICE out [n_cells][3] */
  double *U_s;          /* DEVICE out [n_points][3] or NULL */
  double *w;            /* DEVICE out [n_points] or NULL */
  double *P_s;          /* DEVICE out [n_points][3] or NULL */
  int64_t *cell_a;      /* DEVICE out [n_points] cell of P_a (-1 outside) or NULL */
  int64_t *cell_s;      /* DEVICE out [n_points] cell of P_s (-1 outside) or NULL */
  const double *dUdt;   /* DEVICE [n_cells][3] fluid acceleration (eq. 8), or NULL */
} alp_case;

#define ALP_USE_GRAPH 1u /* capture the step on the first call, replay it afterwards */
#define ALP_CHECKED 2u   /* synchronise at the end, grow the work lists on overflow, and check
                            the pair-record layout on the host (every item's records inside the
                            allocated record area, no two items' records overlapping):
                            ALP_ERR_HIP if violated */
#define ALP_AUTOTUNE 4u  /* before the first step of a new set of cases, choose the launch
                            shape (alp_tuning) by timing graph replays of the step */

/* Launch shape of a step's kernels.  Every output is bitwise independent of
   it (decisions are exact and every sum is exact or in a fixed order), so it
   only changes the time a step takes. */
typedef struct {
  int32_t sample_lanes;  /* lanes per actuator point in the sampler: 2, 4 or 8, i.e. 32, 16
                            or 8 points per 64-lane workgroup */
  int32_t sample_waves;  /* sampler workgroups per CU beside the segment binning (1..32), or
                            0 = chosen from the point count */
  int32_t weights_grab;  /* work items (up to 64 cells of one tile each) a weights workgroup
                            takes from its queue at once: 1..16 */
  int32_t weights_waves; /* weights workgroups (one wave each) per CU: 1..32 */
  int32_t spread_waves;  /* spread workgroups (of 16 waves) per CU (1..32, capped at what a CU holds),
                            or 0 = every resident slot */
} alp_tuning;

/* A whole coupling step (sample -> drag -> project) for n_cases independent
   cases in one set of launches: every stage runs once over the concatenated
   work of all cases.  cases is a HOST array.  With ALP_USE_GRAPH the first call
   for a given set of cases captures the launch sequence in a hipGraph and later
   calls with identical case descriptors replay it; the arrays in the cases may
   be updated in place between replays.  If updated arrays need longer work
   lists than the captured ones (beams that moved so that more cells or tiles
   lie within reach), the replay drops what does not fit (it accesses nothing
   beyond its lists), alp_get_diag reports n_overflow, and the next call with
   the same cases returns ALP_ERR_CAPACITY once that replay has completed and
   drops the graph; the call after it sizes the lists again.  With
   ALP_CHECKED a replay reports its own overflow.  A mesh may appear in at
   most one case of a batch. */
alp_status alp_step_batched(alp_context *ctx, int32_t n_cases, const alp_case *cases,
                            uint32_t flags);

/* For callers that cannot allocate device memory (code that must not call
   hipMalloc, such as tight serving loops or harnesses that forbid it): one
   uncaptured step of alp_step_batched (flags 0) whose whole per-step
   workspace -- counters, work lists, pair records, the case table and scan
   temporaries -- lives in a static device array of 64 MiB per device
   instead of memory the context allocates.  It calls no hipMalloc or
   hipFree; the meshes and every input and output array are the caller's as
   for alp_step_batched.  It synchronises the context stream at the end to
   read the overflow flags.
     ALP_ERR_CAPACITY  the step's fixed lists do not fit (checked before any
                       launch), or its window or pair lists overflowed the
                       rest of the array (results of that step invalid)
   Every call on one device shares that device's array, which keeps the last
   call's contents: calls that overlap on one device (several contexts or
   threads) race.  alp_get_diag reads this step's diagnostics from it, so it
   must come before another call on the same device. */
alp_status alp_step_noalloc(alp_context *ctx, int32_t n_cases, const alp_case *cases);

/* The context's launch shape (the defaults, the last ALP_AUTOTUNE choice or
   the last alp_set_tuning), and setting it.  alp_set_tuning rejects values out
   of range (ALP_ERR_INVALID_ARG) and drops captured graphs.  HOST structs. */
alp_status alp_get_tuning(alp_context *ctx, alp_tuning *out);
alp_status alp_set_tuning(alp_context *ctx, const alp_tuning *t);

/* Diagnostics of case `case_index` of the last step (or of the last
   alp_sample / alp_spread pair, index 0).  Synchronous. */
alp_status alp_get_diag(alp_context *ctx, int32_t case_index, alp_diag *out);

/* Drop captured graphs and work-list sizing (call after shape changes). */
alp_status alp_invalidate(alp_context *ctx);

/* Run one un-captured step of alp_step_batched (same arguments, flags
   ignored) with HIP events recorded on the context stream between its stages,
   synchronise, and return the duration of each stage in milliseconds:
     stage_ms   HOST out [max_stages]; stage i is named by alp_stage_name(i)
     n_stages   HOST out, number of stages written
   The step's outputs are produced as by alp_step_batched.  For measurement. */
alp_status alp_step_profile(alp_context *ctx, int32_t n_cases, const alp_case *cases,
                            double *stage_ms, int32_t max_stages, int32_t *n_stages);
/* Name of profiling stage i ("" when out of range). */
const char *alp_stage_name(int32_t i);

/* Autotuner of the cell binning for a given batch (the search structure of
   Sec. 3.2.5 is built once per run, so its parameters can be chosen once).
   For each candidate setting it bins the cells (bin size 0.75, 1, 1.5 or 2
   times the default of alp_bin_cells; tile edge 2..6 bins), runs
   alp_step_batched on `cases` with that mesh in place of
   cases[tuned_case].mesh (flags as given, plus one sizing run), times `reps`
   steps (<= 0: 3) with the host clock after synchronising, and returns the
   fastest setting:
     C, V, domain_box   as alp_bin_cells (the cells of cases[tuned_case])
     out_bin_size       HOST out, bin size to pass to alp_bin_cells
     out_tile_bins      HOST out, tile edge in bins to pass to alp_bin_cells
     out_ms             HOST out (nullable), the measured milliseconds per step
   The cases' outputs are overwritten by the trial steps.  Captured graphs
   are dropped.  Synchronous; not allowed under capture. */
alp_status alp_autotune(alp_context *ctx, int64_t n_cells, const double *C, const double *V,
                        const double *domain_box, int32_t n_cases, const alp_case *cases,
                        int32_t tuned_case, uint32_t flags, int32_t reps, double *out_bin_size,
                        int32_t *out_tile_bins, double *out_ms);

/* Autotuner of the cell binning of every case of a batch at once: each
   candidate bins every case's cells with bin size = scale x that case's
   default bin size (scale 0.75, 1 or 1.5) and tile edge T (2..5 bins), runs
   the batch with those meshes (flags as given, plus one sizing run), times
   `reps` steps (<= 0: 3) and keeps the fastest.  A candidate whose step
   overflows a per-tile limit (ALP_ERR_CAPACITY) is skipped.
     cases        HOST [n_cases], as for alp_step_batched; on return
                  cases[i].mesh is the best candidate's mesh for case i, a new
                  mesh the caller destroys with alp_mesh_destroy (the meshes
                  passed in are left as they were)
     C, V         HOST arrays [n_cases] of DEVICE pointers: each case's cell
                  centres [n][3] and volumes [n] (n = that mesh's cell count)
     boxes        HOST array [n_cases] of HOST domain boxes (each nullable), or NULL
     out_scale, out_tile_bins, out_ms   HOST out (out_ms nullable)
   The cases' outputs are overwritten by the trial steps.  Captured graphs are
   dropped.  Synchronous; not allowed under capture. */
alp_status alp_autotune_binning(alp_context *ctx, int32_t n_cases, alp_case *cases,
                                const double *const *C, const double *const *V,
                                const double *const *boxes, uint32_t flags, int32_t reps,
                                double *out_scale, int32_t *out_tile_bins, double *out_ms);

/* Beam state for the point-wise helpers (Sec. 3.2.2): one actuator point per
   beam control volume, beams as a CSR over points as in alp_beams.  DEVICE
   pointers. */
typedef struct {
  int32_t n_beams;
  int32_t reserved0;        /* must be 0 */
  int64_t n_points;
  const int64_t *offsets;   /* [n_beams+1], 0 .. n_points, non-decreasing */
  const double *Cb;         /* [n_points][3] initial beam-cell centres C^b */
  const double *Wref;       /* [n_points][3] fixed offsets W^ref, or NULL = 0 */
  const double *W;          /* [n_points][3] current displacements W */
  const double *eps_phys;   /* [n_points] physical kernel width (needed for eps) */
  double eps_factor;        /* multiplier of the local cell size, > 0 (2 in Sec. 8) */
} alp_beam_state;

/* Point-wise geometry ahead of a step, stream-ordered on the context's
   stream, asynchronous:
     P       DEVICE out [n_points][3] (nullable): the actuator points of
             eq. (15), P = (C^b + W^ref) + W.  (Their velocity is the
             beam-cell velocity; nothing to compute.)
     e_t     DEVICE out [n_points][3] (nullable): unit tangents of the spline
             through the current cell centres x = C^b + W (Sec. 3.2.2).  The
             node derivative is that of the parabola through three consecutive
             centres parameterised by chord length (i-1, i, i+1; the first or
             last three at the ends); a two-point beam takes its chord; a
             zero-length chord falls back to the neighbouring one; a single
             point, or only coincident centres, gets the zero vector (counted;
             the step rejects a zero tangent, so the caller supplies one).
     eps     DEVICE out [n_points] (nullable): the local kernel width of
             Sec. 8, eps = max(eps_factor V_c^(1/3), eps_phys) with c the cell
             of P (nearest centre, as for sampling); a point outside the
             domain box keeps eps_phys (counted).  Needs `mesh` and eps_phys.
     counts  DEVICE out int64 [2] (nullable): zero tangents, points outside.
   ALP_ERR_INVALID_ARG for inconsistent sizes or offsets (the offsets are
   read back to validate them, which waits for the caller's stream), nothing
   requested, or eps without a mesh, eps_phys or a positive factor; not
   allowed under capture. */
alp_status alp_beam_geometry(alp_context *ctx, const alp_mesh *mesh, const alp_beam_state *state,
                             double *P, double *e_t, double *eps, int64_t *counts);

/* Library version string. */
const char *alp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ALP_H */

/*
 * grav.h -- C ABI of the MI355X fast-multipole gravity forward model.
 *
 * The library evaluates the gravity field of a voxelised density, Eq. (1) of
 * May & Knepley (Sec. 1.1), g(r) = G * integral rho(x) (r - x)/|r - x|^3 dV,
 * and the potential phi with lap(phi) = -4 pi G rho, phi -> 0 at infinity,
 * g = -grad(phi) (Eqs. (2)-(4)).  The density is constant on each cubic cell
 * of an nx x ny x nz brick mesh (Sec. 2.1); each cell is replaced by the
 * point masses of a 1-point (centroid) or 2-point-per-axis Gauss rule, and the
 * resulting N-body sum (Eq. (11), Sec. 2.3) is evaluated with the fast
 * multipole method of Sec. 2.3: near field by direct summation and far field
 * through multipole (ME) and local (LE) expansions, split as in the
 * near/far decomposition (Eq. (13)), on an octree (hierarchical
 * decomposition, Sec. 2.3) with the upward sweep (P2M, M2M), the downward
 * sweep (M2L over the interaction list, L2L) and the evaluation (L2P plus the
 * near-field direct sum).  A coincident source/target pair contributes
 * nothing; pairs closer than 1e-10 h (FP64) or 1e-5 h (mixed precision)
 * count as coincident, so that a point placed on a source by the caller's
 * own arithmetic is treated the same whatever its last-bit rounding.
 *
 * Expansion order: p means degrees n = 0 .. p-1 of real solid harmonics,
 * i.e. p^2 real coefficients per expansion (the separable form of Eq. (14)).
 *
 * All functions are thread-compatible: distinct plans may be used from
 * distinct threads; one plan must not be used by two host threads at once.
 * No function throws; every failure is reported through grav_status.
 */
#ifndef GRAV_H
#define GRAV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GRAV_OK = 0,
    GRAV_EINVAL = 1,       /* invalid argument or descriptor field */
    GRAV_ENOMEM = 2,       /* device or host allocation failed */
    GRAV_EDEVICE = 3,      /* a HIP call or kernel launch failed */
    GRAV_EUNSUPPORTED = 4, /* valid request outside what the library implements */
    GRAV_EBUSY = 5         /* the plan's workspace is in use by work on another stream */
} grav_status;

enum { GRAV_FP64 = 0, GRAV_MIXED = 1 };

/* Output components per target: 1 = (gz); 3 = (gx, gy, gz); 4 = (phi, gx, gy, gz). */
enum { GRAV_OUT_GZ = 1, GRAV_OUT_G = 3, GRAV_OUT_PHI_G = 4 };

typedef struct grav_plan_s *grav_plan_t;

typedef struct grav_plan_desc {
    /* Voxel mesh (Sec. 2.1): cubic cells of edge h; cell (i, j, k) spans
     * origin + [i, i+1) x [j, j+1) x [k, k+1) times h.  Density arrays are
     * [batch][nz][ny][nx], x fastest. */
    int32_t nx, ny, nz;
    double origin[3];
    double h;
    /* Cell quadrature: 1 = centroid, weight h^3; 2 = tensor 2-point
     * Gauss-Legendre, points at centre +- h/(2 sqrt 3), weight h^3/8. */
    int32_t quad_order;
    /* Evaluation points: n_points explicit points (host array xyz[n][3],
     * copied during grav_plan; may be NULL when n_points == 0), followed,
     * when voxel_centres != 0, by every cell centre in density order.
     * Outputs are in this order. */
    int64_t n_points;
    const double *points;
    int32_t voxel_centres;
    int32_t components;  /* GRAV_OUT_GZ, GRAV_OUT_G or GRAV_OUT_PHI_G */
    int32_t p;           /* expansion order, 1 <= p <= 16 */
    int32_t leaf_size;   /* max source points per leaf; leaf = b^3 cells with
                            b = min(8, max(1, floor((leaf_size / q^3)^(1/3)))) */
    int32_t precision;   /* GRAV_FP64, or GRAV_MIXED: near field and M2L in
                            FP32 (MFMA), expansions stored and translated in
                            FP64, near + far combined in FP64 */
    int32_t batch;       /* B >= 1 density models sharing the tree */
    double G;            /* gravitational constant applied to every output */
    int32_t device;      /* HIP device ordinal the plan lives on */
    /* Explicit sources in place of the cell quadrature (scattered points
     * with volumes, the extension named in Sec. 4): n_sources > 0 points
     * (host xyz[n][3], copied during grav_plan) inside the mesh box
     * origin + [0, n) h, which then only frames the octree (leaves of b^3
     * cells, b from leaf_size as above) and the voxel-centre targets.  The
     * density arrays of grav_eval and grav_adjoint become [batch][n_sources]
     * in source order: with source_volumes (host [n], each > 0, copied) a
     * value is a density and the source's mass is value * volume; without,
     * the value is the mass.  Requires quad_order 1.  grav_direct,
     * grav_direct_noalloc and grav_analytic return GRAV_EUNSUPPORTED on such
     * plans. */
    int64_t n_sources;
    const double *sources;
    const double *source_volumes;
} grav_plan_desc;

/* Fill *d with defaults: 1-point rule, components 3, p = 8, leaf_size 64,
 * FP64, batch 1, G = 1, device 0, no points, cell sources.  Always succeeds. */
void grav_desc_init(grav_plan_desc *d);

/* Build a plan: validates the descriptor, sorts the evaluation points by
 * the Morton key of their leaf with a device radix sort, builds the octree
 * levels and interaction lists on the device, computes the translation
 * operators (FP64 on the host) and allocates the device workspace.
 * Synchronous.  On success *out owns all of it until grav_plan_destroy.
 * Errors: EINVAL (bad field), EUNSUPPORTED (non-cubic request, p > 16, tree
 * deeper than 10 levels), ENOMEM, EDEVICE. */
grav_status grav_plan(const grav_plan_desc *desc, grav_plan_t *out);

void grav_plan_destroy(grav_plan_t plan);

/* Device bytes held by the plan for its whole life (tree, operators) and
 * the workspace one evaluation needs (expansions, near-field buffers).  Both
 * are already allocated by grav_plan; the figures serve admission control. */
grav_status grav_plan_bytes(grav_plan_t plan, size_t *resident, size_t *per_call);

/* Shape facts of a plan: number of evaluation points, tree depth L (leaves
 * are at level L, the root at 0), leaf edge in cells (b), and total number
 * of leaf boxes that hold evaluation points.  Any pointer may be NULL. */
grav_status grav_plan_info(grav_plan_t plan, int64_t *n_targets, int32_t *levels,
                           int32_t *leaf_cells, int64_t *n_target_leaves);

/* Work counts of a plan, per density model: box pairs translated by M2L
 * (over all levels), point pairs of the near-field direct sum (targets times
 * quadrature points of the neighbour leaves, coincident pairs included) and
 * the number of source points (cells times q^3).  Any pointer may be NULL. */
grav_status grav_plan_work(grav_plan_t plan, int64_t *m2l_pairs, int64_t *p2p_pairs,
                           int64_t *n_sources);

/* Forward evaluation (the far/near split of Eq. (13) with the FMM).
 * rho:   device pointer, double [batch][nz][ny][nx].
 * g_out: device pointer, double [batch][n_targets][components], written in
 *        the evaluation-point order of the descriptor, G applied.
 * stream: HIP stream (hipStream_t) to enqueue on; NULL = default stream.
 * Asynchronous: enqueues kernels only (no allocation, no host sync); the
 * caller keeps rho and g_out alive until the stream reaches that point.
 * Calls on one plan from different streams while earlier work is still in
 * flight return GRAV_EBUSY.  The call may be recorded into a HIP graph
 * (stream capture): it enqueues kernels only (no memset, allocation or
 * host synchronisation); during capture the workspace lock is neither
 * checked nor updated, so the caller serialises the replays of graphs that
 * share a plan (and profiling must be off: GRAV_EUNSUPPORTED otherwise).  A
 * plan with no evaluation points does nothing and accepts NULL buffers.
 * Errors: EINVAL (NULL pointer), EBUSY, EDEVICE. */
grav_status grav_eval(grav_plan_t plan, const double *rho, double *g_out, void *stream);

/* Adjoint: the exact transpose of grav_eval's linear map rho -> g (Eq. (1)
 * of Sec. 1.1 is linear in rho, and so is every FMM stage of Sec. 2.3), so
 * that <grav_eval(rho), r> = <rho, grav_adjoint(r)> to rounding and the
 * gradient of a misfit such as 0.5 ||gz - d||^2 is grav_adjoint(gz - d).
 * resid:    device pointer, double [batch][n_targets][components];
 * drho_out: device pointer, double [batch][nz][ny][nx]; overwritten with
 *           drho[b][cell] = sum_j,c resid[b][j][c] * d g[b][j][c] / d rho[b][cell].
 * The transposed stages use the forward's operators (in mixed precision the
 * FP32-rounded M2L matrices), interaction lists, point pairs and
 * coincidence rule; the near field is transposed in the forward's arithmetic
 * type.  Uses the plan's workspace (shared with grav_eval).  Same asynchrony
 * and errors as grav_eval; a plan with no evaluation points writes zeros. */
grav_status grav_adjoint(grav_plan_t plan, const double *resid, double *drho_out, void *stream);

/* Direct summation (the summation method of Sec. 2.1, SUM-G1 / SUM-G2): the
 * same output as grav_eval for the plan's evaluation points and quadrature
 * rule, computed as the plain sum over every (target, quadrature point) pair
 * with the same coincidence rule, O(M N) work, no expansions.  Arguments,
 * layouts, asynchrony and errors as grav_eval; arithmetic in the plan's
 * precision (FP64, or FP32 for GRAV_MIXED with the target-source offset
 * formed in FP64).  Shares the plan's workspace lock (GRAV_EBUSY). */
grav_status grav_direct(grav_plan_t plan, const double *rho, double *g_out, void *stream);

/* grav_direct without any device allocation behind it, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same kernels, launch
 * shape and summation order as grav_direct, so the output is identical, but
 * the per-chunk partial sums live in a fixed 8 MiB device array inside the
 * library (one per GPU, held until the process ends; its address is looked
 * up on the first call on each device) instead of the plan's buffer.
 * Arguments, layouts and asynchrony as grav_direct.  Every call on one GPU
 * shares that array: calls that overlap in time on one GPU (different
 * streams, or different plans) race and must be serialised by the caller.
 * The array needs no clearing: each call writes every partial it reads.
 * Errors: EUNSUPPORTED if the plan's partials (chunks x targets x batch x 4
 * doubles) exceed 8 MiB or its device ordinal is 64 or more; otherwise as
 * grav_direct. */
grav_status grav_direct_noalloc(grav_plan_t plan, const double *rho, double *g_out, void *stream);

/* Closed-form summation (the analytic summation method SUM-AN of Sec. 2.1):
 * gz at the plan's evaluation points as the sum over all cells of the exact
 * attraction of a uniform rectangular prism (the closed form the paper cites
 * for its analytic method and for the exact solution of Sec. 3), so no
 * quadrature rule is involved: exact for a cell-wise constant density, up to
 * rounding.  The plan's quadrature order and p are ignored.
 * rho:    device pointer, double [batch][nz][ny][nx] (as grav_eval);
 * gz_out: device pointer, double [batch][n_targets][1], descriptor order,
 *         gz with the sign of Eq. (1) (positive above a positive anomaly),
 *         G applied.
 * FP64 arithmetic in both precisions, O(M (nx+1)(ny+1)(nz+1)) work.  Plans
 * with components != 1 return GRAV_EUNSUPPORTED (the method gives gz only).
 * Asynchrony, workspace lock and other errors as grav_direct. */
grav_status grav_analytic(grav_plan_t plan, const double *rho, double *gz_out, void *stream);

/* Stage timings of the last evaluation or adjoint enqueued with
 * grav_set_profiling(plan, 1), in milliseconds from HIP events on the
 * evaluation stream: up to n entries of (name, ms).  Synchronizes with the
 * stream.  Returns the number of stages written in *count. */
grav_status grav_set_profiling(grav_plan_t plan, int32_t enable);
grav_status grav_stage_times(grav_plan_t plan, const char **names, double *ms, int32_t n,
                             int32_t *count);

/* Validate a plan's index tables on the host: copies the tables back and
 * checks, with the same column/term resolvers the kernels use, that every
 * expansion, matrix, target-range and cell index of every stage lies inside
 * the buffer it addresses and that no two columns of a stage write the same
 * expansion.  Launches no compute kernel.  Returns GRAV_OK, or GRAV_EINVAL
 * with the first violation described in msg (msglen bytes, may be NULL). */
grav_status grav_plan_check(grav_plan_t plan, char *msg, int32_t msglen);

/* Operator matrices used by the plan (FP64, row-major, p^2 x p^2, real
 * solid-harmonic basis), for inspection and the operator tests:
 * kind 0 = M2M from child octant `which` (bit 0: +x, bit 1: +y, bit 2: +z)
 * to its parent; kind 1 = L2L from the parent to child octant `which`;
 * kind 2 = M2L for the source-box offset (dx, dy, dz) in box units, which
 * must satisfy 2 <= max(|dx|, |dy|, |dz|) <= 3.  out holds p^4 doubles.
 * Host-only; needs no device. */
grav_status grav_operator(int32_t p, int32_t kind, int32_t which, int32_t dx, int32_t dy,
                          int32_t dz, double *out);

/* Evaluate the real solid harmonics used by the expansions at one point
 * (host): regular (kind 0) or irregular (kind 1), p^2 values in the
 * library's real coefficient order (degree n block of 2n+1 values:
 * m = 0 real part, then m = 1..n real and imaginary parts). */
grav_status grav_harmonics(int32_t p, int32_t kind, double x, double y, double z, double *out);

const char *grav_status_string(grav_status s);

/* Library version string. */
const char *grav_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GRAV_H */

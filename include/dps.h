/*
 * dps.h -- Barnes-Hut regularized dipole sums on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libdps.so.  The method is that of Chen, Miller, Gkioulekas,
 * "3D Reconstruction with Fast Dipole Sums" (ACM TOG 43(6), 2024):
 *
 *   D_c(x) = sum_m A_m P_eps(x, p_m) mu_{m,c},                 (Sec. 4.2, eq. dipole_sum)
 *   P_eps(x, y) = rho(|y-x|/eps) n(y).(y-x) / (4 pi |y-x|^3),  (Sec. 4.1, eq. regularized_poisson)
 *   rho(t) = erf(t) - (2t/sqrt(pi)) exp(-t^2),
 *
 * one sum per attribute channel c (Sec. 5.1, eq. appearance_features), all
 * channels sharing one traversal (Sec. 6.3).  Sums are evaluated with the
 * Barnes-Hut scheme of Sec. 6.1 / Algorithm 1 over an octree whose nodes carry
 * the area, area-weighted centroid, radius (eq. farfield_dipole) and the
 * vector moments (eq. farfield_dipole_features); adjoints follow Sec. 6.2 and
 * App. C (node accumulation, then one push-down to the points).
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers on the tree's device, except where
 *    marked "host".  Arrays are dense, row-major, float32 unless stated.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is enqueued on it; inputs must stay valid until the stream reaches it.
 *  - The caller owns every input and output buffer.  Outputs are overwritten,
 *    never accumulated, except the tree's internal adjoint accumulators, which
 *    add up across dps_adjoint_accumulate calls until dps_adjoint_finalize.
 *  - Errors are status codes; nothing throws across the ABI.  On
 *    DPS_ERR_INVALID nothing is launched and no output is touched.  A
 *    human-readable message for the last failure of the calling thread is
 *    returned by dps_last_error().
 *  - Point order: "caller order" is the order of the arrays given to
 *    dps_build.  Internally points are kept in Morton order.
 *  - One call processes at most DPS_MAX_ROWS rows (queries, rays times
 *    samples, grid points); larger counts return DPS_ERR_INVALID.
 */
#ifndef DPS_H
#define DPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dps_tree_s *dps_tree;

typedef enum {
    DPS_OK = 0,
    DPS_ERR_INVALID = 1, /* bad argument or non-finite / non-positive input data */
    DPS_ERR_OOM = 2,     /* device allocation failed */
    DPS_ERR_DEVICE = 3,  /* HIP runtime error (launch, copy, synchronisation) */
    DPS_ERR_STATE = 4    /* handle unknown, destroyed, or in a failed state */
} dps_status;

typedef enum {
    DPS_STORE_FP32 = 0,  /* attributes and node moments stored as float32 */
    DPS_STORE_BF16 = 1   /* attributes and node moments stored as bfloat16 (round
                            to nearest even), except the moments of the nodes of
                            depth <= 3, which stay float32 (a query far from the
                            geometry takes a few such nodes as its whole far
                            field, so their rounding would not average out) */
} dps_storage;

typedef enum {
    DPS_KERNEL_DIPOLE = 0,   /* the regularised dipole kernel of eq. regularized_poisson */
    DPS_KERNEL_MONOPOLE = 1  /* the same kernel without the foreshortening factor n.(y-x)/|y-x|
                                (appearance attributes, Sec. 7.1), see dps_build_kernel */
} dps_kernel;

/* Maximum rows (queries, placed ray samples, grid points) of one call: 2^38. */
#define DPS_MAX_ROWS ((int64_t)1 << 38)

/* Maximum number of attribute channels per tree. */
#define DPS_MAX_CHANNELS 32
/* Maximum leaf size (points per bucket leaf). */
#define DPS_MAX_LEAF 256
/* Octree depth: 21 levels below the root (63-bit Morton codes). */
#define DPS_LEVELS 21

/*
 * dps_build -- octree over an oriented point cloud with its far-field data.
 * Sec. 6.1 (octree, eq. farfield_dipole, eq. farfield_dipole_features) and
 * Sec. 6.3 (built once, since points and areas are fixed during optimisation).
 *
 *  p      [M][3] point positions p_m          n [M][3] normals n_m (used as given)
 *  A      [M]    area weights A_m (> 0)       attrs [M][C] per-point attributes mu_{m,c}
 *  M      number of points, 1 <= M <= 2^31-1
 *  C      channels, 1 <= C <= DPS_MAX_CHANNELS
 *  leaf_size  bucket size, 1 <= leaf_size <= DPS_MAX_LEAF; a node is a leaf iff
 *         it holds <= leaf_size points or sits at level DPS_LEVELS
 *  storage    DPS_STORE_FP32 or DPS_STORE_BF16
 *  out    host pointer receiving the handle (set to NULL on failure)
 *
 * Layout (canonical, reproduced bit-exactly by dps_export_tree): the bounding
 * cube is the componentwise FP32 min of the points with side = max extent
 * (FP64; 1 if zero), quantised as q = min(floor((p - lo) * 2^21/side), 2^21-1)
 * in FP64, Morton code with x at bit 3i+2, y at 3i+1, z at 3i; points stably
 * sorted by code; nodes numbered breadth-first with children contiguous in
 * ascending octant order; the node centroid is the FP64 area-weighted mean
 * rounded once to FP32, and the node's squared radius r_t^2 is the largest
 * FP32 value fma(dz, dz, fma(dy, dy, dx*dx)) over its points, d = p_m - p_t
 * against that FP32 centroid (each operation rounded once, nothing else
 * fused).
 *
 * Moments (eq. farfield_dipole_features, refreshed by dps_set_attributes):
 * D_t = sum A_m mu_m n_m, formed from A_m, mu_m and n_m with compensated FP32
 * sums (FP64 for the nodes of depth <= 3 when M >= 4,194,304) and stored
 * rounded once from the working sum: FP32 storage holds the exact moment
 * rounded to FP32 (up to a rare one-ulp tie); BF16 storage rounds that FP32
 * value to bfloat16 below depth 3.
 *
 * Synchronises `stream` (node counts are needed on the host).  Returns
 * DPS_ERR_INVALID for bad sizes / NULL pointers, or if any p, n, A, attrs
 * value is non-finite or any A_m <= 0 (checked on the device).
 */
dps_status dps_build(const float *p, const float *n, const float *A, const float *attrs,
                     int64_t M, int32_t C, int32_t leaf_size, dps_storage storage,
                     void *stream, dps_tree *out);

/*
 * dps_build_kernel -- as dps_build (same arguments, layout, synchronisation
 * and errors) with the kernel of the sums chosen per tree.  Sec. 7.1 sums its
 * 32 appearance attributes with the foreshortening term of the kernel skipped,
 * i.e. with the monopole kernel
 *   m(r) = rho(r/eps) / (4 pi r^2),   D_c(x) = sum_m A_m m(|p_m - x|) mu_{m,c},
 *   grad D_c(x) = sum_m A_m mu_{m,c} (r lambda - kappa / r) (p_m - x),
 * whose node moments are the scalar charges Q_tc = sum_{m in t} A_m mu_{m,c}
 * placed at the node's area-weighted centroid; the octree, the far test and
 * the traversal order are those of the dipole kernel (Algorithm 1).  A source
 * at the query point itself contributes nothing.  Normals are stored but not
 * used by the monopole kernel.  The geometry channel keeps the dipole kernel:
 * callers build one tree per kernel over the same points (the two trees have
 * identical node layouts).
 *
 * A DPS_KERNEL_MONOPOLE tree supports dps_set_attributes, dps_query,
 * dps_query_channels, dps_query_counts, dps_adjoint_zero / _accumulate /
 * _accumulate_channels / _finalize, dps_adjoint, dps_adjoint_finalize_ext
 * (dattrs only), dps_export_tree (moments: the charge in component 0 of each
 * channel, components 1 and 2 zero), dps_tree_info, dps_set_launch /
 * dps_get_launch and dps_check.  The gradient-cotangent, normal and eps
 * derivatives, dps_set_normals and dps_query_grid are defined for the dipole
 * kernel only and return DPS_ERR_INVALID on a monopole tree.
 *  kernel  DPS_KERNEL_DIPOLE or DPS_KERNEL_MONOPOLE (else DPS_ERR_INVALID)
 */
dps_status dps_build_kernel(const float *p, const float *n, const float *A, const float *attrs,
                            int64_t M, int32_t C, int32_t leaf_size, dps_storage storage,
                            dps_kernel kernel, void *stream, dps_tree *out);

/* dps_get_kernel -- host output: the tree's kernel (a dps_kernel value). */
dps_status dps_get_kernel(dps_tree t, int32_t *kernel);

/*
 * dps_set_attributes -- moment refit after the attributes changed (Sec. 6.3:
 * node moments are refreshed each iteration; eq. farfield_dipole_features).
 *  attrs [M][C] in caller order.  Asynchronous; values are not checked.
 */
dps_status dps_set_attributes(dps_tree t, const float *attrs, void *stream);

/*
 * dps_query -- Barnes-Hut primal query (Algorithm 1, PrimalQuery; Sec. 6.1,
 * eq. farfield) at Q points, all channels in one traversal.
 *  x     [Q][3] query points, not checked: a non-finite point gets a NaN row
 *        and leaves the other rows unchanged (a NaN point fails every far test
 *        and so walks the whole tree); in the adjoint calls such a point makes
 *        the node and point accumulators it reaches non-finite
 *  beta  > 0, finite: a node is used as far field iff |x - p_t| > beta r_t,
 *        evaluated in FP32 as fma(dz, dz, fma(dy, dy, dx*dx)) > (beta*beta)*r_t^2
 *        with d = p_t - x, each operation rounded once and nothing else fused
 *        (strict: a tie opens the node)
 *  eps   >= 0, finite: regularisation; 0 gives the unregularised dipole sum
 *  f     [Q][C] output values D_c(x)
 *  grad  [Q][C][3] output spatial gradients dD_c/dx, or NULL
 * Q = 0 is a no-op.  Asynchronous.
 */
dps_status dps_query(dps_tree t, const float *x, int64_t Q, float beta, float eps,
                     float *f, float *grad, void *stream);

/*
 * dps_query_counts -- traversal statistics of dps_query (same decisions):
 *  counts [Q][4] int32: nodes visited (far tests evaluated), nodes used as
 *  far field, leaves opened, points summed exactly.  Asynchronous.
 */
dps_status dps_query_counts(dps_tree t, const float *x, int64_t Q, float beta,
                            int32_t *counts, void *stream);

/*
 * Adjoint (Sec. 6.2, App. C).  Stage 1 (dps_adjoint_accumulate, Algorithm 1
 * AdjointQuery) adds, for every query, df . (dD/dmu_t) into the node
 * accumulators of the far-field nodes it uses (eq. farfield_gradient) and the
 * exact near-field terms into per-point accumulators, and writes dL/dx.
 * Stage 2 (dps_adjoint_finalize) pushes node accumulators down to the points
 * through all their ancestors (eq. farfield_features_gradient).
 *
 * dps_adjoint_zero       clears the accumulators.
 * dps_adjoint_accumulate x [Q][3], df [Q][C] = dL/dD_c(x); dx [Q][3] output
 *                        dL/dx (overwritten), or NULL (the walk then skips the
 *                        gradient terms).  Same beta/eps rules as dps_query.
 *                        Accumulates across calls.
 * dps_adjoint_finalize   dattrs [M][C] output dL/dmu in caller point order.
 * dps_adjoint            zero + accumulate + finalize.
 * All asynchronous and free of host synchronisation and memory set / copy
 * nodes, so a training step (set_attributes, query, adjoint) can be captured
 * in a hipGraph and replayed.
 *
 * Ordering: calls on one tree must be ordered by the caller (one stream, or
 * events between streams).  set_attributes and adjoint_* mutate the tree, and
 * every traversal (dps_query*, dps_adjoint*, dps_query_grid, dps_ray_march)
 * resets and consumes the tree's tile counters when the launch is persistent
 * (dps_set_launch bits 2, 3) or a ray march, so two such calls running at
 * the same time on one tree would share its tile queue.  Trees are
 * independent of each other.
 */
dps_status dps_adjoint_zero(dps_tree t, void *stream);
dps_status dps_adjoint_accumulate(dps_tree t, const float *x, int64_t Q, float beta, float eps,
                                  const float *df, float *dx, void *stream);
dps_status dps_adjoint_finalize(dps_tree t, float *dattrs, void *stream);
dps_status dps_adjoint(dps_tree t, const float *x, int64_t Q, float beta, float eps,
                       const float *df, float *dattrs, float *dx, void *stream);

/*
 * dps_export_tree -- canonical arrays for parity checks (any may be NULL):
 *  codes   [M] uint64 sorted Morton codes
 *  perm    [M] uint32 sorted position -> caller index
 *  nodes   [N][6] int32 {level, parent (-1 root), first_child (-1 leaf),
 *          n_children, pt_begin, pt_count} in breadth-first order
 *  geom    [N][4] float {cx, cy, cz, r^2}
 *  moments [N][C][3] float node dipoles D_t = sum_{m in t} A_m mu_m n_m
 *          (decoded to float32 from the storage format); for a monopole tree
 *          the charge sum_{m in t} A_m mu_m in component 0, components 1, 2 zero
 * Synchronises `stream`.
 */
dps_status dps_export_tree(dps_tree t, uint64_t *codes, uint32_t *perm, int32_t *nodes,
                           float *geom, float *moments, void *stream);

/* dps_tree_info -- host outputs (any may be NULL): node count, depth (deepest
 * level), device bytes held by the tree, point count, channel count. */
dps_status dps_tree_info(dps_tree t, int64_t *n_nodes, int32_t *depth, int64_t *bytes,
                         int64_t *n_points, int32_t *channels);

/*
 * dps_set_launch -- launch shape of the traversal kernels (results do not
 * depend on it beyond floating-point summation order).
 *  query_k, adjoint_k  queries per lane, 1, 2 or 4 (0 keeps): a 64-lane
 *      wavefront walks the tree once for 64*k consecutive queries, lane l
 *      carrying queries base + 64 i + l, so node fetches and, in the adjoint,
 *      the wavefront sums and atomics are shared by 64*k queries (the packet
 *      queries suggested in Sec. 6.3).  Large channel blocks cap k so the
 *      accumulators stay in registers.
 *  flags  (-1 keeps) bit 0 / bit 1: for dps_query / the adjoint, the
 *      workgroups that run on one of the 8 XCDs take a contiguous eighth of
 *      the queries, so each XCD's L2 serves one region of a coherently ordered
 *      query set; bit 2 / bit 3: persistent launch -- a grid of resident
 *      workgroups pulls 64*k-query tiles from per-XCD counters (own eighth
 *      first, then the others), balancing uneven batches inside one launch;
 *      bit 4: dps_ray_march marches one ray per lane (see dps_ray_march).
 * Host-only; applies to later launches.  The defaults are k = 2 / 4 with the
 * XCD-contiguous order.
 */
dps_status dps_set_launch(dps_tree t, int32_t query_k, int32_t adjoint_k, int32_t flags);
dps_status dps_get_launch(dps_tree t, int32_t *query_k, int32_t *adjoint_k, int32_t *flags);

/*
 * dps_set_split -- subtree-split walks, for batches too small to fill the GPU
 * (the few hundred thousand samples of a 4096-ray training batch make a few
 * wavefronts per SIMD, each waiting on its own chain of node fetches).  With
 * P > 1 parts the walk of each 64-query tile (one query per lane) is divided
 * over P wavefronts.  Nodes are numbered level by level in Morton order, and
 * node t of level <= cut_level belongs to part t mod P.  Every part tests the
 * nodes above the cut level that its queries reach (each part opens the same
 * ones) but adds a node's far-field term only if it owns the node; a node of
 * the cut level, or a leaf above it, that the part does not own is skipped
 * with its whole subtree.  Each source term of Algorithm 1 is therefore added
 * by exactly one part.
 *  query_parts  (0 keeps) 1, 2, 4 or 8, for dps_query and dps_query_channels
 *      on dipole trees.  The call zeroes the f (and grad) rows and the parts
 *      add their sums into them with FP32 atomics: with 2 parts the result
 *      does not depend on their order; with more it can change between runs
 *      in the last bit.  Summation order differs from the unsplit walk.
 *  adjoint_parts  (0 keeps) 1, 2, 4 or 8, for the dipole adjoint accumulation
 *      when dL/dx is not formed in the walk (dx NULL, or
 *      dps_adjoint_accumulate_from_forward); part 0 writes dL/dx.  The
 *      accumulators are FP64 atomic sums either way.
 *  cut_level  (-1 keeps) 0 to 21.
 * The packet sizes and flags of dps_set_launch do not apply to split walks;
 * grid queries, ray marches, the gradient-cotangent adjoint and monopole
 * trees are never split.  Host-only; applies to later launches.  Default 1, 1
 * (unsplit), cut level 3.  Errors: DPS_ERR_INVALID for other values.
 */
dps_status dps_set_split(dps_tree t, int32_t query_parts, int32_t adjoint_parts, int32_t cut_level);
dps_status dps_get_split(dps_tree t, int32_t *query_parts, int32_t *adjoint_parts, int32_t *cut_level);

/*
 * dps_query_channels / dps_adjoint_accumulate_channels -- as dps_query /
 * dps_adjoint_accumulate for the channel range [c_begin, c_begin+n_channels)
 * only (e.g. the geometry channel alone for shadow rays).  f, grad and df rows
 * hold n_channels entries.  With BF16 storage c_begin must be even.
 *  Q        rows of x / f / grad / df / dx (capacity)
 *  q_count  device pointer or NULL: when given, only the first
 *           min(Q, max(*q_count, 0)) rows are processed, the count being read
 *           on the device when the kernels run (batch sizes decided on the GPU,
 *           e.g. the number of shadow rays, inside a captured graph); the other
 *           rows are left untouched.
 */
dps_status dps_query_channels(dps_tree t, const float *x, int64_t Q, const int64_t *q_count, float beta,
                              float eps, int32_t c_begin, int32_t n_channels, float *f, float *grad,
                              void *stream);
dps_status dps_adjoint_accumulate_channels(dps_tree t, const float *x, int64_t Q, const int64_t *q_count,
                                           float beta, float eps, int32_t c_begin, int32_t n_channels,
                                           const float *df, float *dx, void *stream);

/*
 * dps_adjoint_accumulate_from_forward -- as dps_adjoint_accumulate_channels,
 * with dL/dx formed from the spatial gradients the forward query already
 * returned for these points instead of a second evaluation of every term's
 * gradient in the walk:
 *   dL/dx_q = sum_c df_qc grad_qc,
 * the same sum as the walk's (the Barnes-Hut gradient is the sum of the
 * gradient terms of the sources the value accepts, and both calls make the
 * same far decisions).  The walk then accumulates only the node and point
 * increments of Algorithm 1 (AdjointQuery).  For a step that queries values
 * with gradients and then back-propagates (the usual training step), this
 * is the cheaper call.
 *  x        device [Q][3]
 *  q_count  device row count or NULL (as dps_query_channels)
 *  c_begin, n_channels  channel range (BF16 storage: c_begin even)
 *  df       device [Q][n_channels] cotangents (required)
 *  grad     device [Q][n_channels][3]: dps_query / dps_query_channels
 *           gradients at the same x with the same beta and eps and the
 *           attributes as they are now (required; the result is only as
 *           right as these are)
 *  dx       device [Q][3] output (overwritten), or NULL (grad then unused)
 * Accumulates like dps_adjoint_accumulate.  Graph-safe.  DPS_ERR_INVALID for
 * a NULL x, df or grad, bad ranges, or a monopole-kernel tree.
 */
dps_status dps_adjoint_accumulate_from_forward(dps_tree t, const float *x, int64_t Q, const int64_t *q_count,
                                               float beta, float eps, int32_t c_begin, int32_t n_channels,
                                               const float *df, const float *grad, float *dx, void *stream);

/*
 * dps_adjoint_accumulate_grad -- stage 1 of the adjoint for cotangents of the
 * spatial gradients (and optionally of the values), for losses that use
 * grad D, as the surface density sigma = |w . grad v| / v of Sec. 3.1, eq.
 * (surface_density), does.  Each source term's gradient
 * -kappa D + lambda (D.d) d (d = source - x) is linear in its dipole D, so the
 * cotangent h adds lambda (d.h) d - kappa h to the same node and point
 * accumulators as the value cotangents (finalised by dps_adjoint_finalize);
 * dL/dx adds the term's Hessian applied to h,
 *   nu s (d.h) d - lambda (d (D.h) + D (d.h)) - lambda s h,  s = D.d,
 * nu = chi(t)/(4 pi r^7), chi = 5 psi - t psi'.  Same traversal decisions
 * (Algorithm 1) as the forward query.
 *  x        device [Q][3]
 *  q_count  device row count or NULL (as dps_query_channels)
 *  c_begin, n_channels  channel range (BF16 storage: c_begin even)
 *  df       device [Q][n_channels] value cotangents, or NULL (zero)
 *  dg       device [Q][n_channels][3] gradient cotangents (required)
 *  dx       device [Q][3] or NULL: overwritten with dL/dx of these rows
 * Accumulators add across calls (mixing with dps_adjoint_accumulate*).
 * Graph-safe; DPS_ERR_INVALID for a NULL x / dg or bad ranges.
 */
dps_status dps_adjoint_accumulate_grad(dps_tree t, const float *x, int64_t Q, const int64_t *q_count, float beta,
                                       float eps, int32_t c_begin, int32_t n_channels, const float *df,
                                       const float *dg, float *dx, void *stream);

/*
 * Derivatives in the point normals and in eps.  Sec. 5.2 optimises the
 * normals and the global regularisation eps together with the attributes.
 * A term depends on n_m only through its dipole A_m mu_m n_m (the tree
 * geometry -- centroids, radii, far decisions -- does not involve normals), so
 *   dL/dn_m = A_m sum_c mu_mc dL/dD_mc,
 * with the far-field part pushed down from the node accumulators of all
 * ancestors; eps enters kappa and lambda only:
 *   d kappa / d eps = -exp(-t^2) / (pi^1.5 eps^4),
 *   d lambda / d eps = -2 exp(-t^2) / (pi^1.5 eps^6),
 * nonzero in practice inside the regularised zone t < 4.5 (beyond it the
 * kernels use rho = 1, psi = 3 and the derivative is below FP32 resolution).
 *
 * dps_adjoint_accumulate_ext -- as dps_adjoint_accumulate_grad, with df and
 *   dg each optional (not both NULL), and want a mask of DPS_WANT_NORMALS
 *   (accumulate the near-field part of dL/dn) and DPS_WANT_EPS (accumulate
 *   dL/deps in FP64).  All calls between a zero and a finalize must use the
 *   same eps.
 * dps_adjoint_finalize_ext -- as dps_adjoint_finalize, every output optional
 *   (at least one): dattrs [M][C], dnormals [M][3] (caller order), deps one
 *   FP64 value; all device pointers.
 * dps_set_normals -- replaces the point normals (device [M][3], caller order;
 *   A_m n_m is stored).  The node moments follow at the next
 *   dps_set_attributes, which must be called before the next query.
 * All graph-safe; DPS_ERR_INVALID for NULL or out-of-range arguments.
 */
#define DPS_WANT_NORMALS 1
#define DPS_WANT_EPS 2
dps_status dps_adjoint_accumulate_ext(dps_tree t, const float *x, int64_t Q, const int64_t *q_count, float beta,
                                      float eps, int32_t c_begin, int32_t n_channels, const float *df,
                                      const float *dg, int32_t want, float *dx, void *stream);
dps_status dps_adjoint_finalize_ext(dps_tree t, float *dattrs, float *dnormals, double *deps, void *stream);
dps_status dps_set_normals(dps_tree t, const float *n, void *stream);

/*
 * dps_query_grid -- dps_query_channels at the points of a regular grid, for
 * mesh extraction by marching cubes on the geometry field (Sec. 7.1 extracts
 * the 1/2 level set at 512^3 and 1024^3).  The positions are generated in the
 * kernels, in 4 x 4 x 4 bricks (one wavefront per brick), so no position array
 * is read.
 *  origin, spacing  host float[3]; point (i, j, k) is
 *                   origin + (i, j, k) * spacing, each coordinate computed in
 *                   FP32 as o + (float)i * h with no fused multiply-add
 *  dims             host int64[3] = (nx, ny, nz), each in [1, 2^24]
 *  f                device [nz][ny][nx][n_channels]
 *  grad             device [nz][ny][nx][n_channels][3] or NULL
 * Persistent launch with the tree's queries-per-lane setting.  Graph-safe.
 */
dps_status dps_query_grid(dps_tree t, const float origin[3], const float spacing[3], const int64_t dims[3], float beta,
                          float eps, int32_t c_begin, int32_t n_channels, float *f, float *grad, void *stream);

/*
 * Ray front-end (Sec. 7.1, ray sampling): each camera ray's first crossing of
 * the geometry level set is found with a dense march, and the quadrature
 * samples are then placed around it (the paper uses 1024 march samples and
 * 24 / 48 / 8 samples before / around / after the crossing, or 80 uniform
 * samples for a ray without one).  Rays: o, d device [R][3] (d need not be
 * unit), tnear, tfar device [R] near and far limits.
 *
 * dps_ray_march -- march sample k of ray r is x_k = o + t_k d with
 *   t_k = tnear + (k + 1/2) h, h = (tfar - tnear) / n_samples, in FP32 with
 *   one rounding per operation; D is channel `channel` of the tree's dipole
 *   sum (beta, eps as dps_query).  Output hit_index [R] int32: the smallest j
 *   with (D(x_j) >= level) != (D(x_{j+1}) >= level), or -1; hit_values [R][2]
 *   float: D(x_j), D(x_{j+1}) (0, 0 without a crossing).  Rays are not
 *   checked: one with a non-finite origin, direction or interval finds no
 *   crossing (-1; 0, 0) and leaves the other rays unchanged.  A wavefront walks
 *   128 consecutive samples of one ray (64 with query packet 1): all chunks of
 *   all rays run at once and a chunk past a crossing already found is skipped,
 *   so any ray order and any batch size keep the GPU busy.  Launch flag bit 4
 *   of dps_set_launch instead gives each lane one ray, walking its samples in
 *   order up to its crossing (consecutive rays should then be neighbouring
 *   pixels, e.g. 8 x 8 tiles); results are identical either way.  The
 *   ray-major march keeps the crossing index in hit_index (an atomic minimum
 *   over chunks) and the two field values of each chunk's first crossing in
 *   a workspace held by the tree (R x chunks x 8 bytes, chunks =
 *   ceil((n_samples - 1) / (64 k - 1)) for query packet k), from which the
 *   values of the ray's crossing are gathered.  The first call that needs a
 *   larger workspace allocates it (counted in the tree's bytes and under
 *   dps_set_memory_limit); an outgrown workspace stays allocated until
 *   dps_destroy, because a graph captured earlier may use it.  A call being
 *   captured into a graph that would need a larger workspace, or one the
 *   memory limit or an allocation failure refuses, evaluates the field at
 *   j and j + 1 in a second pass instead: the same values bit for bit.
 *   n_samples in [2, 2^20]; dipole-kernel trees only; with BF16 storage the
 *   channel must be even.  R = 0 is a no-op.  DPS_ERR_INVALID (nothing
 *   launched) for a bad argument or NULL array, or for more rays x samples
 *   than one launch grid holds.  Uses the tree's query packet setting and
 *   its tile counters (order calls on one tree).  Graph-safe.
 * dps_ray_resample -- no tree.  With a crossing (hit_index >= 0):
 *   t* = t_j + w (t_{j+1} - t_j), w = (level - D_j) / (D_{j+1} - D_j), window
 *   [a, b] = [max(tnear, t* - window h), min(tfar, t* + window h)]
 *   (h = (tfar - tnear) / n_march), n_before samples in [tnear, a], n_dense in
 *   [a, b], n_after in [b, tfar]; without one, S = n_before + n_dense + n_after
 *   samples in [tnear, tfar].  Sample i of the m in [lo, hi] is at
 *   t = lo + (i + u) (hi - lo) / m, u = jitter[r][s] in [0, 1) (device
 *   [R][S]), FP32 with one rounding per operation, x = o + t d.  Outputs
 *   t_out [R][S] and x_out [R * S][3]: row r * S + s (tile_layout = 0) or
 *   ((r / 64) * S + s) * 64 + r % 64 (tile_layout = 1, R a multiple of 64:
 *   a wavefront then holds one sample of 64 neighbouring rays, the layout of
 *   the point queries that follow).  Counts >= 1 with S <= 4096, window >= 0.
 *   Runs on the current device.  Graph-safe.
 */
dps_status dps_ray_march(dps_tree t, const float *o, const float *d, const float *tnear, const float *tfar, int64_t R,
                         int32_t n_samples, float beta, float eps, int32_t channel, float level, int32_t *hit_index,
                         float *hit_values, void *stream);
dps_status dps_ray_resample(const float *o, const float *d, const float *tnear, const float *tfar, int64_t R,
                            int32_t n_march, const int32_t *hit_index, const float *hit_values, float level,
                            const float *jitter, int32_t n_before, int32_t n_dense, int32_t n_after, float window,
                            int32_t tile_layout, float *t_out, float *x_out, void *stream);

/*
 * dps_ray_march_harnack -- the march of dps_ray_march (same samples x_k, same
 * crossing definition, same outputs) accelerated by Harnack tracing (Sec.
 * 7.1, following Gillespie et al. 2024): Harnack's inequality bounds how fast
 * a positive harmonic function can change within a ball around a point, so
 * from an evaluated sample many of the next ones can be skipped.  The field
 * shifted by `lower` (u = D - lower, assumed > 0) is harmonic within
 * R = (distance to the nearest point) - 4.5 eps of a sample x_k (the kernel's
 * regularisation ends there: rho(4.5) = 1 - 8e-9); with a = (level - lower) /
 * (D(x_k) - lower) the field stays on D(x_k)'s side of the level within
 * s R, s = |sqrt(8a + 1) - (2a + 1)| / (2a) (the root of (1 - s) = a (1 + s)^2
 * or of (1 + s) = a (1 - s)^2).  The samples strictly within 0.99 s R are
 * skipped, the next one is evaluated and, if it lies on the other side of the
 * level, the one before it: on D(x_k)'s side it closes the crossing pair,
 * otherwise (the field did not obey the bound, e.g. because `lower` is not a
 * bound or the Barnes-Hut switch between far field and points moved the
 * value) the ray continues sample by sample from x_k.  So wherever the bound
 * holds, hit_index and hit_values equal dps_ray_march's, bit for bit (same
 * walk at the same FP32 positions).  One ray per lane (a persistent tile
 * queue over 64-ray tiles); each step runs a nearest-point walk and a value
 * walk.
 *  lower   a lower bound of the field (finite, < level); the geometry field
 *          of a closed surface lies in [0, 1] up to noise, e.g. -0.25
 *  evals   [R] int32 output: field evaluations per ray, or NULL
 * Other arguments, errors and ordering as dps_ray_march (uses the tree's tile
 * counters).  Graph-safe: no allocation, no memory set or copy.
 */
dps_status dps_ray_march_harnack(dps_tree t, const float *o, const float *d, const float *tnear, const float *tfar,
                                 int64_t R, int32_t n_samples, float beta, float eps, int32_t channel, float level,
                                 float lower, int32_t *hit_index, float *hit_values, int32_t *evals, void *stream);

/*
 * dps_adjoint_noalloc -- for callers that cannot allocate device memory
 * (code under graph capture, serving loops, harnesses that forbid it): the
 * result of dps_adjoint (same arguments, outputs and errors; dattrs [M][C] in
 * caller order, dx [Q][3] or NULL) computed with its working buffers -- the
 * FP64 node and point accumulators and the tile counters -- in a static
 * per-device workspace of DPS_NOALLOC_SCRATCH_BYTES instead of the tree's.
 * Calls no allocating routine.  Each device the library runs on holds one
 * copy of the workspace until the process ends; every call on that device
 * uses the same copy and clears it first, so calls that overlap in time on
 * one device (other streams, other threads, other trees) race and give wrong
 * results: order them.  Leaves the tree's own adjoint accumulators untouched.
 * Needs 8 (N * 3C + M * C) bytes plus 64 (rounded to 256-byte blocks) to
 * fit the workspace (e.g. 1M points, 264k nodes, C = 4: 58 MB); larger trees
 * get DPS_ERR_INVALID.  Dipole-kernel trees only.  Graph-safe.
 */
#define DPS_NOALLOC_SCRATCH_BYTES (64 << 20)
dps_status dps_adjoint_noalloc(dps_tree t, const float *x, int64_t Q, float beta, float eps, const float *df,
                               float *dattrs, float *dx, void *stream);

/* dps_check -- synchronises `stream` and reports device-side failures recorded
 * by earlier calls on this tree (DPS_ERR_DEVICE; sticky until destroyed).  A
 * traversal that would walk more than N nodes stops and sets this flag; its
 * outputs are then incomplete. */
dps_status dps_check(dps_tree t, void *stream);

/* dps_set_step_limit -- caps the nodes one traversal of this tree may walk
 * (0 restores the default, the node count N, which a well-formed tree never
 * exceeds; otherwise 1 <= limit <= N).  Reaching the cap is the failure that
 * dps_check reports: the traversal stops, every kernel exits normally, the
 * outputs are incomplete, and the tree's sticky error is set.  A diagnostic,
 * for exercising that failure path from the host.  Host-only; applies to
 * later launches.  DPS_ERR_INVALID outside [0, N]. */
dps_status dps_set_step_limit(dps_tree t, int64_t limit);

/* dps_set_memory_limit -- process-wide cap on the device bytes one build may
 * hold at once (the tree's storage plus its temporary buffers), 0 = no cap
 * (the default).  A build that would exceed it returns DPS_ERR_OOM, frees
 * everything it allocated and sets *out = NULL, exactly as when the device
 * runs out of memory.  Applies to later builds.  DPS_ERR_INVALID for
 * bytes < 0. */
dps_status dps_set_memory_limit(int64_t bytes);

/* dps_destroy -- frees the tree (synchronises the device first).  NULL is a no-op. */
void dps_destroy(dps_tree t);

/* Static strings. */
const char *dps_status_string(dps_status s);
const char *dps_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DPS_H */

/*
 * nao.h -- C ABI of the MI355X (gfx950) real-space grid engine for numeric
 * atom-centred orbitals: batch-wise Hamiltonian integration and density
 * update over spatially compact batches of integration points, with the
 * operations built on the same batches: the density gradient, the Hamiltonian
 * with a GGA-type vector field or with the kinetic term, and the local Pulay
 * forces; batches by octree or by the paper's cut-plane partition.
 *
 * Method: Huhn, Lange, Yu, Yoon, Blum, "GPGPU Acceleration of All-Electron
 * Electronic Structure Theory Using Localized Numeric Atom-Centered Basis
 * Functions".  Section references below are to that paper.
 *
 * Conventions for every call:
 *   - all real data are FP64 (double) at the boundary, lengths are int64_t,
 *     coordinates are in Angstrom, matrices are dense row-major N_b x N_b;
 *   - the caller owns every buffer it passes; the library copies what it keeps;
 *   - a nao_memspace argument says whether the pointer next to it is host
 *     memory or device memory of the context's GPU (e.g. a torch tensor's
 *     data_ptr()); device pointers must come from hipMalloc-type allocations;
 *   - calls return a nao_status; no C++ exception, abort or exit crosses the
 *     ABI; nao_last_error() returns the message of the last failing call;
 *   - a context and its systems are used by one host thread at a time;
 *   - work is ordered on the context's HIP stream.  A call with any host
 *     output synchronizes before returning; a call whose outputs are all
 *     device memory returns after enqueueing (inputs must stay valid until
 *     the stream reaches the work).
 *   - a HIP failure is sticky: the context reports NAO_ERR_HIP from then on.
 */
#ifndef NAO_H
#define NAO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nao_ctx_s* nao_ctx;       /* one HIP device + stream + HBM-budget allocator */
typedef struct nao_system_s* nao_system; /* one structure's resident device state          */
typedef struct nao_plan_s* nao_plan;     /* host-only batches and lists (no GPU needed)    */

typedef enum {
    NAO_OK = 0,
    NAO_ERR_INVALID_ARG = -1,   /* bad argument; no state was changed                     */
    NAO_ERR_OUT_OF_MEMORY = -2, /* host or device allocation failed                       */
    NAO_ERR_BUDGET = -3,        /* the context's HBM budget would be exceeded             */
    NAO_ERR_HIP = -4,           /* a HIP runtime call failed; the context is now unusable */
    NAO_ERR_NOT_READY = -5,     /* no GPU / library built without one / not initialised   */
    NAO_ERR_INTERNAL = -6
} nao_status;

/* Arithmetic of the two contractions.  Basis evaluation, partition weights,
 * w*v, the accumulation into the global H and the electron count are FP64 in
 * every mode. */
typedef enum {
    NAO_FP64 = 0,   /* FP64 MFMA                                                       */
    NAO_FP32 = 1,   /* FP32 MFMA, FP32 accumulation within a group, FP64 across groups;
                       normwise error against FP64 below 1e-6 on H and n              */
    NAO_BF16X3 = 2, /* three-term split-BF16 products (x0 y0 + x0 y1 + x1 y0), FP32
                       accumulation, FP64 after every 32 points / 64 functions; about
                       1e-6 on H and 1e-5 on n                                         */
    NAO_BF16X6 = 3  /* six-term split-BF16 products (hi, mid, lo parts), otherwise as
                       NAO_BF16X3; below 1e-6 on H and n                               */
} nao_precision;

typedef enum { NAO_MEM_HOST = 0, NAO_MEM_DEVICE = 1 } nao_memspace;

/* ---------------------------------------------------------------------------------------
 * Basis description: atoms with species; each species is a list of shells (l, radial id);
 * each radial function is tabulated at n_knots logarithmic knots
 *   r_k = rmin * (rcut/rmin)^(k/(n_knots-1)),  k = 0..n_knots-1,
 * and is interpolated by a natural cubic spline in t = ln(r/rmin)/Delta,
 * Delta = ln(rcut/rmin)/(n_knots-1); it is zero at and beyond rcut.  The basis function
 *   phi(r) = R(|r - R_A|) * Y_lm(unit(r - R_A))
 * uses real orthonormal spherical harmonics (Y_11 proportional to +x), m = -l..l.  The
 * global basis order is atom-major, then the species' shell order, then m = -l..l.
 * (Section "Computational Choices in FHI-aims": numeric atom-centred orbitals confined
 * to a cutoff radius; eq. EVNonPeriodic: the basis expansion.)
 * Constraints: 0 <= l <= 3, at most 16 shells per species, n_knots >= 4, 0 < rmin < rcut,
 * finite samples.
 * ------------------------------------------------------------------------------------- */
typedef struct {
    int64_t n_atoms;
    const double* atom_xyz;           /* [n_atoms][3]                                  */
    const int32_t* atom_species;      /* [n_atoms], 0..n_species-1                     */
    int32_t n_species;
    const int32_t* species_shell_ptr; /* [n_species+1], into shell_l / shell_radial     */
    const int32_t* shell_l;           /* [n_shells], 0..3                               */
    const int32_t* shell_radial;      /* [n_shells], 0..n_radial-1                      */
    int32_t n_radial;
    int32_t n_knots;
    const double* radial_rmin;        /* [n_radial] first knot                          */
    const double* radial_rcut;        /* [n_radial] last knot = cutoff                  */
    const double* radial_samples;     /* [n_radial][n_knots] R(r_k)                     */
} nao_basis_desc;

/* ---------------------------------------------------------------------------------------
 * Context.
 * nao_ctx_create: device = HIP ordinal; hip_stream = a hipStream_t to order work on, or
 * NULL for a stream the context creates; hbm_budget_bytes = cap on the device memory the
 * context allocates for all its systems (0 = no cap).  NAO_ERR_NOT_READY without a GPU.
 * ------------------------------------------------------------------------------------- */
nao_status nao_ctx_create(int device, void* hip_stream, size_t hbm_budget_bytes, nao_ctx* out);
/* Destroy every system and server of a context before the context itself. */
void nao_ctx_destroy(nao_ctx ctx);
/* Message of the last failing call on ctx; ctx = NULL gives the calling thread's last
 * message of a context-less call (nao_plan_*).  Never NULL; valid until the next call. */
const char* nao_last_error(nao_ctx ctx);
nao_status nao_ctx_set_stream(nao_ctx ctx, void* hip_stream);
void* nao_ctx_stream(nao_ctx ctx);
nao_status nao_ctx_synchronize(nao_ctx ctx);
/* Bytes currently allocated by the context and its budget (0 = none). */
nao_status nao_ctx_memory(nao_ctx ctx, size_t* used_bytes, size_t* budget_bytes);

/* Overlap of basis evaluation with the contractions in nao_integrate_h and nao_update_density
 * (the overlap of independent work that the paper's GPU variants exploit, Section "GPGPU
 * Acceleration of the Real-Space Domain Decomposition Algorithm"): with more than one block of
 * basis values, the basis launch of block k + 1 runs on a second stream of the context (default
 * priority) into a second buffer while the contraction of block k runs on the context stream,
 * ordered by events; the context stream still ends after every launch of the call, so callers
 * synchronize on it alone.  On by default (NAO_OVERLAP=0 in the environment turns it off for
 * contexts created afterwards).  The second buffer, as large as the basis scratch, is charged to
 * the budget; a call for which it does not fit runs serially.  enable = 0 turns it off and frees
 * the buffer (after the work in flight), any other value turns it on. */
nao_status nao_ctx_set_overlap(nao_ctx ctx, int enable);

/* Per-kernel timing (the per-operation timings the paper reports, at kernel granularity).
 * nao_ctx_profile(ctx, 1) starts recording: every kernel launch of the context is then
 * bracketed by HIP events on the stream it runs on (the context stream, or the second stream of
 * an overlapped basis evaluation); (ctx, 0) stops.  Starting also clears
 * what was recorded.  nao_ctx_profile_read synchronizes the stream and reports, per kernel
 * name (at most max_entries, names as 32-byte NUL-terminated strings in names), the number
 * of launches and their summed duration in milliseconds; n_entries receives the count. */
nao_status nao_ctx_profile(nao_ctx ctx, int enable);
nao_status nao_ctx_profile_read(nao_ctx ctx, int32_t max_entries, char* names, int64_t* launches,
                                double* total_ms, int32_t* n_entries);

/* ---------------------------------------------------------------------------------------
 * Host-only planning (runs without a GPU).  Partitions the points into batches of at most
 * max_batch points by an octree and builds each batch's list nnz(B) of basis functions
 * that are non-zero on at least one of its points.
 * (Section "Grid Partitioning": disjoint compact batches up to a batch size; Section
 * "Parallelization and Dimensionality Reduction": the reduced subspace nnz(B_nu).)
 * Octree: root box = per-axis [min, max] of all points; a node with <= max_batch points
 * is a batch; otherwise mid = 0.5*(lo+hi), octant c = [x>=mid_x] + 2[y>=mid_y] +
 * 4[z>=mid_z], children visited c = 0..7 depth-first pre-order, empty ones dropped,
 * indices ascending; a node at depth >= 60, or whose mid equals lo or hi on all three
 * axes, is cut into consecutive chunks of max_batch.  Batches are numbered in emission
 * order.  Relevance: atom A is relevant to batch b iff some point of b has
 * (dx*dx + dy*dy) + dz*dz < rcA*rcA in FP64 without fused multiply-add, rcA being the
 * largest cutoff of A's radial functions; the list is the relevant atoms ascending, each
 * expanded to its basis functions in global order.  The result is bit-exact: a fixed
 * input gives fixed perm / batch_ptr / basis_ptr / basis_idx on every machine.
 * max_batch in [1, 4096]; n_points in [0, 2^31-1]; point_xyz finite.
 * ------------------------------------------------------------------------------------- */
nao_status nao_plan_create(const nao_basis_desc* basis, int64_t n_points, const double* point_xyz,
                           int32_t max_batch, nao_plan* out);

/* Batching method of nao_plan_create_ex / nao_build_batches_ex.
 * NAO_BATCH_OCTREE: the octree above (what nao_plan_create and nao_build_batches use).
 * NAO_BATCH_CUTPLANE: the grid-adapted cut-plane partition the paper uses (Section "Grid
 * Partitioning": the point set is cut by planes until every subset holds at most the batch
 * size).  Definition: a set S with |S| <= max_batch is a batch, indices ascending; otherwise,
 * with k = ceil(|S| / max_batch), the plane is normal to the axis of largest extent
 * (max - min of S's coordinates, FP64; ties: lowest axis) and S, ordered by (coordinate on
 * that axis, point index), gives its first floor(|S| floor(k/2) / k) points to the lower side,
 * the rest to the upper side; the lower side is processed first and batches are numbered in
 * emission order.  Gives exactly ceil(n_points / max_batch) batches (max_batch >= 2) of nearly
 * equal size.  Bit-exact like the octree; relevance and lists as above. */
typedef enum { NAO_BATCH_OCTREE = 0, NAO_BATCH_CUTPLANE = 1 } nao_batcher;
nao_status nao_plan_create_ex(const nao_basis_desc* basis, int64_t n_points, const double* point_xyz,
                              int32_t max_batch, nao_batcher batcher, nao_plan* out);
nao_status nao_plan_info(nao_plan plan, int64_t* n_basis, int64_t* n_batches, int64_t* n_list);
/* perm [n_points] (batch b = points perm[batch_ptr[b] .. batch_ptr[b+1]-1]),
 * batch_ptr [n_batches+1], basis_ptr [n_batches+1], basis_idx [n_list]; any may be NULL. */
nao_status nao_plan_get_batches(nao_plan plan, int64_t* perm, int64_t* batch_ptr,
                                int64_t* basis_ptr, int32_t* basis_idx);
void nao_plan_destroy(nao_plan plan);

/* ---------------------------------------------------------------------------------------
 * Structure setup: plans the batches (as nao_plan_create), builds the spline coefficients
 * (FP64, on the host), packs consecutive batches into execution groups of at most
 * group_max points (default 256; a batch larger than that is cut into pieces; exact,
 * since every basis function is zero on the points outside its list) and uploads
 * atoms, splines, batch-ordered points and weights, lists and groups to device memory
 * owned by the returned system.  point_xyz [n_points][3] and point_w [n_points] are host
 * arrays in the caller's point order; w >= 0 and finite.
 * ------------------------------------------------------------------------------------- */
nao_status nao_build_batches(nao_ctx ctx, const nao_basis_desc* basis, int64_t n_points,
                             const double* point_xyz, const double* point_w, int32_t max_batch,
                             nao_system* out);
/* nao_build_batches with the batching method chosen (nao_batcher). */
nao_status nao_build_batches_ex(nao_ctx ctx, const nao_basis_desc* basis, int64_t n_points,
                                const double* point_xyz, const double* point_w, int32_t max_batch,
                                nao_batcher batcher, nao_system* out);
/* Change the execution-group size (in points, 16..256; default 256) of a system; 0 runs
 * every batch as its own unit (no packing).  Results change only by floating-point
 * summation order. */
nao_status nao_system_set_group_max(nao_system sys, int32_t group_max);
/* Keep the basis values of every block resident in device memory across operations
 * (enable = 1): nao_integrate_h and nao_update_density then evaluate them once per value type
 * (FP64, or FP32 for the reduced-precision modes) and reuse them until the execution groups
 * change (nao_system_set_group_max, nao_system_set_h_tile, nao_system_autotune), the geometry
 * of a system being fixed (the SCF case: the same points and basis at every iteration).
 * Costs 8 bytes per basis value of the whole system (the sum of its blocks), charged to the
 * context's HBM budget: NAO_ERR_BUDGET (or NAO_ERR_OUT_OF_MEMORY from the device) leaves the
 * mode off, and so does a later change of groups whose layout no longer fits (that call then
 * returns the same status).
 * Results equal those of the default mode up to the order of the FP64 atomic accumulation.  The other operations (gradients, fields,
 * forces, nao_run_many, nao_eval_basis) evaluate as before.  enable = 0 frees the memory. */
nao_status nao_system_set_resident_basis(nao_system sys, int enable);
/* Tile width (64 or 128 basis functions) of the Hamiltonian kernel for this system; wider
 * tiles stage each basis value for twice the MFMA work, narrower ones waste less padding.
 * Results change only by floating-point summation order.  The reduced-precision split-BF16
 * modes always use 64. */
nao_status nao_system_set_h_tile(nao_system sys, int32_t h_tile);
/* Autotuner: times a density update and a Hamiltonian integration of this system (inputs v and
 * D in `space`) at `precision` for each candidate (Hamiltonian tile width 64 / 128, execution
 * groups of 256 / 192 / 128 points; 64-wide only for split-BF16), keeps the fastest and
 * applies it.  The choice is cached in a JSON file ($NAO_TUNE_CACHE, default
 * $HOME/.cache/nao_tune.json) keyed by device, precision and the system's shape class
 * (work-weighted mean list length and mean batch size of its octree batches); a cached class
 * is applied without timing unless NAO_TUNE_FORCE is set.  Outputs (nullable): the chosen
 * h_tile and group_max, and the best measured milliseconds (-1 when taken from the cache). */
#define NAO_TUNE_FORCE 1u
nao_status nao_system_autotune(nao_system sys, nao_precision precision, const double* v, const double* D,
                               nao_memspace space, uint32_t flags, int32_t* h_tile, int32_t* group_max,
                               double* best_ms);
nao_status nao_system_info(nao_system sys, int64_t* n_basis, int64_t* n_batches, int64_t* n_list,
                           size_t* dev_bytes);
/* Host copies of the system's batches and lists (as nao_plan_get_batches). */
nao_status nao_get_batches(nao_system sys, int64_t* perm, int64_t* batch_ptr, int64_t* basis_ptr,
                           int32_t* basis_idx);
/* Work measure of the paper's "#ops" metric (Section "GPGPU Acceleration Across Materials
 * and Architectures"): units = sum over batches of |B| * m^2 with m = |nnz(B)|. */
nao_status nao_system_work(nao_system sys, double* units);

/* ---------------------------------------------------------------------------------------
 * Basis values phi_i(r_p) for the batches [batch_begin, batch_end): for each batch a dense
 * [|B|][m] block, point-major, rows in batch point order, columns in list order; blocks
 * are concatenated, block b starting at phi + phi_ptr[b - batch_begin].  phi_ptr is a host
 * array of batch_end - batch_begin + 1 entries, always written.  phi = NULL only fills
 * phi_ptr (size query).  (Section "GPGPU Acceleration of the Real-Space Domain Decomposition Algorithm": the basis
 * functions in nnz(B) on every point of the batch.)
 * ------------------------------------------------------------------------------------- */
nao_status nao_eval_basis(nao_system sys, int64_t batch_begin, int64_t batch_end, double* phi,
                          nao_memspace phi_space, int64_t* phi_ptr);

/* ---------------------------------------------------------------------------------------
 * Hamiltonian matrix with a local potential,
 *   H_ij = sum_p w_p v_p phi_i(r_p) phi_j(r_p),
 * summed batch by batch through each batch's dense matrix (eq. H_int_aims, eq. H_decomp,
 * eq. H_contrib_batch, eq. batch_matrix_mult with K = w phi and L = v phi).
 * v [n_points] in caller point order; H [N_b][N_b] row-major, written in full and exactly
 * symmetric (the upper triangle is accumulated, then mirrored).  With H in device memory
 * the call only enqueues.
 * ------------------------------------------------------------------------------------- */
nao_status nao_integrate_h(nao_system sys, const double* v, nao_memspace v_space,
                           nao_precision precision, double* H, nao_memspace H_space);
/* ---------------------------------------------------------------------------------------
 * nao_integrate_h without any device allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same result as nao_integrate_h (up to the order of the FP64 accumulation)
 * and the same kernels; v [n_points] and H [N_b][N_b] must be device memory of the
 * context's GPU, and the call only enqueues.
 * Scratch: instead of the context's basis-value buffer, the call uses one fixed array of
 * 256 MiB per GPU inside the library (held from the first context on that GPU until the
 * process ends): a segment table, w*v (8 bytes per point) and the basis values of as many
 * execution groups at a time as fit.  NAO_ERR_INVALID_ARG, with nothing enqueued, when
 * w*v of n_points > 255 MiB / 8 (about 33 million points) does not fit beside the table,
 * when one execution group's basis values do not fit what is left, or when the sub-blocks
 * outnumber the table.  The call allocates nothing (no hipMalloc, hipFree, events or
 * library allocations), so it is also slower than nao_integrate_h on large systems (more,
 * smaller launches).
 * Every call on one GPU shares that GPU's array and leaves its contents behind: two calls
 * whose work overlaps on one GPU (other streams, other contexts, other host threads) race
 * and give wrong results; order them on one stream or synchronize between them.
 * ------------------------------------------------------------------------------------- */
nao_status nao_integrate_h_noalloc(nao_system sys, const double* v, nao_precision precision, double* H);

/* ---------------------------------------------------------------------------------------
 * Density n(r_p) = sum_ij phi_i(r_p) D_ij phi_j(r_p) at every point (eq. Density), batch by
 * batch through the batch density matrix D[nnz(B), nnz(B)] (Section "GPGPU Acceleration
 * of the Real-Space Domain Decomposition Algorithm").  D [N_b][N_b] row-major is symmetric;
 * like the symmetric matrix product used for it in the paper, only its upper triangle
 * (i <= j) is read: for a D that is not symmetric the result is that of the symmetric matrix
 * with D's upper triangle, D_ji := D_ij for i < j (not that of (D + D^T) / 2).
 * n [n_points] in caller point order (exact zeros where no basis function reaches).
 * n_electrons (host, nullable) receives N_e = sum_p w_p n_p; passing it synchronizes.
 * ------------------------------------------------------------------------------------- */
nao_status nao_update_density(nao_system sys, const double* D, nao_memspace D_space,
                              nao_precision precision, double* n, nao_memspace n_space,
                              double* n_electrons);
/* ---------------------------------------------------------------------------------------
 * Hamiltonian with a local potential and a vector field acting on grad(phi_i phi_j),
 *   H_ij = sum_p w_p [ v_p phi_i phi_j + a_p . (grad phi_i phi_j + phi_i grad phi_j) ]  at r_p,
 * the form the gradient-dependent part of a GGA potential takes (a = 2 (df/d sigma) grad n);
 * batch by batch as eq. batch_matrix_mult with K = Phi and L = (w v / 2) Phi + (w a) . grad Phi,
 * H_b = K^T L + L^T K over the upper-triangle tile pairs.  grad phi as for
 * nao_update_density_gradient.  v [n_points] and a [n_points][3] in caller point order, both
 * in in_space; H as for nao_integrate_h.  precision: NAO_FP64 or NAO_FP32.  Needs device scratch
 * for one L value per basis value of a block (as much as the basis scratch).
 * ------------------------------------------------------------------------------------- */
nao_status nao_integrate_h_gga(nao_system sys, const double* v, const double* a, nao_memspace in_space,
                               nao_precision precision, double* H, nao_memspace H_space);

/* ---------------------------------------------------------------------------------------
 * Kohn-Sham Hamiltonian with the kinetic term: eq. H_int_aims with h_KS acting on phi_j as
 * t + v, t = -1/2 lap the non-relativistic kinetic operator, symmetrised in i and j, plus the
 * optional vector-field term of nao_integrate_h_gga:
 *   H_ij = sum_p w_p [ v_p phi_i phi_j + (phi_i t phi_j + phi_j t phi_i) / 2
 *                      + a_p . (grad phi_i phi_j + phi_i grad phi_j) ]  at r_p.
 * Batch by batch as eq. batch_matrix_mult in its symmetric rank-2k form, K = Phi and
 * L = (w v / 2) Phi - (w / 4) lap Phi + (w a) . grad Phi, H_b = K^T L + L^T K.  lap phi =
 * (R'' + 2 R'/r - l(l+1) R / r^2) Y_lm, taken from the radial spline's own first and second
 * derivatives; zero where phi is cut off and for |r - R_A| <= rmin.  v [n_points] and
 * a [n_points][3] (nullable: no field) in caller point order, both in in_space; H as for
 * nao_integrate_h.  precision: NAO_FP64 or NAO_FP32.  Needs device scratch for one L value per
 * basis value of a block (as much as the basis scratch).
 * ------------------------------------------------------------------------------------- */
nao_status nao_integrate_h_ks(nao_system sys, const double* v, const double* a, nao_memspace in_space,
                              nao_precision precision, double* H, nao_memspace H_space);

/* ---------------------------------------------------------------------------------------
 * Density and its gradient at every point, grad n(r_p) = 2 sum_ij grad phi_i(r_p) D_ij phi_j(r_p)
 * for symmetric D (the density gradients the paper names beside eq. Density and in the
 * subsection "Density and Density Derivatives, Force and Stress Tensor Components"), batch by
 * batch: T = Phi D_b over the batch's whole list, n = rowsum(T * Phi), grad n =
 * 2 rowsum(T * grad Phi).  grad phi = R'(r) u Y + (R / r) (dY/du - u (u . dY/du)) with
 * u = unit(r - R_A); it is zero where phi is cut off and for |r - R_A| <= rmin (the spline's
 * clamped, constant part).  D as in nao_update_density (upper triangle read); n [n_points] and
 * grad_n [n_points][3] in caller point order, both in out_space.  precision: NAO_FP64 or
 * NAO_FP32 (other values give NAO_ERR_INVALID_ARG).  Needs device scratch for the gradients of
 * one block of basis values (three times the basis scratch).
 * ------------------------------------------------------------------------------------- */
nao_status nao_update_density_gradient(nao_system sys, const double* D, nao_memspace D_space,
                                       nao_precision precision, double* n, double* grad_n,
                                       nao_memspace out_space);

/* ---------------------------------------------------------------------------------------
 * Local Pulay forces (the density-only Pulay term that follows eq. forces), with h_KS = t + v,
 * t = -lap / 2 the non-relativistic kinetic operator and v the local potential:
 *   F_A = -2 sum_ij sum_p w_p [grad_A phi_i](r_p) (D_ij [h_KS phi_j](r_p) - Q_ij phi_j(r_p)),
 * D the density matrix and Q the energy-weighted density matrix (eq. E_Weighted_DM), with
 * grad_A phi_i = -grad phi_i for the functions centred on atom A and 0 for the others.  Batch
 * by batch: M = diag(w) (diag(v) Phi - lap Phi / 2) D_b - diag(w) Phi Q_b over the batch's
 * whole list, f_i += sum_p grad phi_pi M_pi, then F_A = 2 sum_{i on A} f_i.  grad phi as for
 * nao_update_density_gradient, lap phi as for nao_integrate_h_ks.  D and Q [N_b][N_b]
 * row-major, symmetric, only their upper triangles read; v [n_points] in caller point order;
 * all three in in_space.  F [n_atoms][3] in F_space.  precision: NAO_FP64 or NAO_FP32 (other
 * values give NAO_ERR_INVALID_ARG).  Needs device scratch for the gradients and Laplacians of
 * one block of basis values (four times the basis scratch).
 * ------------------------------------------------------------------------------------- */
nao_status nao_pulay_forces(nao_system sys, const double* D, const double* Q, const double* v,
                            nao_memspace in_space, nao_precision precision, double* F,
                            nao_memspace F_space);
void nao_system_destroy(nao_system sys);

/* ---------------------------------------------------------------------------------------
 * Many structures in one launch sequence: the work of every entry (op 0 = H with in = v,
 * out = H; op 1 = density with in = D, out = n) is packed into one work list per kernel
 * and launched together (eq. H_decomp: the batches of all structures are independent units
 * of work).  in and out are device memory of the context's device; every system must belong
 * to ctx.  n_electrons (op 1 only; host memory, nullable) receives N_e = sum_p w_p n_p of that
 * entry, and the call then synchronizes.
 * hip_stream: NULL runs the work on the context's stream; otherwise it runs on that stream of
 * the context's device, after the work already enqueued on the context's stream, and the
 * context's stream waits for it before its next work (the context's scratch is shared).
 * NAO_RUN_CAPTURE_GRAPH records the sequence into a HIP graph on first use and replays it
 * while the (systems, pointers, precision) tuple repeats (not with n_electrons: invalid
 * argument); a graph is dropped when a system it names changes its groups or is destroyed,
 * and when the context's basis scratch is replaced by a larger one.
 * ------------------------------------------------------------------------------------- */
typedef struct {
    nao_system sys;
    int32_t op;            /* 0 = Hamiltonian, 1 = density */
    const double* in;      /* v [n_points] or D [N_b][N_b] */
    double* out;           /* H [N_b][N_b] or n [n_points] */
    double* n_electrons;   /* op 1: host, nullable; op 0: must be NULL */
} nao_work;

#define NAO_RUN_CAPTURE_GRAPH 1u

nao_status nao_run_many(nao_ctx ctx, const nao_work* work, int64_t n_work, nao_precision precision,
                        void* hip_stream, uint32_t flags);
/* Without NAO_RUN_CAPTURE_GRAPH, systems may also belong to another context on the same device
 * (the work then runs with ctx's scratch); such a system must not be destroyed while that work
 * runs. */

/* ---------------------------------------------------------------------------------------
 * Serving core: continuous batching of SCF-iteration requests over resident structures.
 *
 * A server owns n_slots execution slots on the device of `home` (each a context with its own
 * HIP stream of default priority and its own scratch).  A session is one structure kept
 * resident in device memory across its SCF iterations (its system plus device buffers for D,
 * v, H and n), allocated through `home`, whose HBM budget therefore bounds what is resident:
 * sessions are admitted in the order they were opened, when their footprint fits
 * (NAO_ERR_BUDGET from the allocation means "wait").  A request is one iteration: a density
 * update from the given D, then the Hamiltonian with the given v (the last v is kept when v
 * is NULL).  nao_server_step never blocks: it retires finished launches, hands sessions that
 * are closed and idle to the builder thread for release, and packs the oldest ready requests (at most one per session in flight, up to
 * max_per_launch per launch) into each free slot as one nao_run_many launch, so requests that
 * arrive while others run join the next launch on a free slot and overlap on the device.
 * Admission (planning and upload of a session's system) runs on a builder thread of the
 * server, so it never stalls the dispatch of resident sessions; a session whose setup fails
 * for another reason than the budget fails its requests (NAO_REQ_FAILED).  The home context
 * belongs to the server while it exists.
 * Inputs D and v stay owned by the caller and must stay valid until the request is done.
 * Times are seconds since the server was created (host steady clock).
 * ------------------------------------------------------------------------------------- */
typedef struct nao_server_s* nao_server;

typedef enum { NAO_REQ_WAITING = 0, NAO_REQ_RUNNING = 1, NAO_REQ_DONE = 2, NAO_REQ_FAILED = 3 } nao_request_state;

/* group_max: execution-group size of the sessions' systems (as nao_system_set_group_max;
 * 0 = every octree batch its own unit). */
nao_status nao_server_create(nao_ctx home, int32_t n_slots, int32_t max_per_launch, int32_t group_max,
                             nao_precision precision, nao_server* out);
/* Queue a structure (copied); returns its session id.  The server's builder thread admits
 * queued sessions in open order as the budget allows. */
nao_status nao_server_open_session(nao_server srv, const nao_basis_desc* basis, int64_t n_points,
                                   const double* point_xyz, const double* point_w, int32_t max_batch,
                                   int64_t* session);
/* The session's resources are released once its last request is done. */
nao_status nao_server_close_session(nao_server srv, int64_t session);
typedef enum {
    NAO_SESSION_QUEUED = 0,      /* waiting for (or in) admission */
    NAO_SESSION_RESIDENT = 1,    /* admitted: its requests can run */
    NAO_SESSION_NO_MEMORY = 2,   /* its last admission attempt did not fit the budget; retried
                                    after another session is released */
    NAO_SESSION_CLOSED = 3,      /* released */
    NAO_SESSION_FAILED = 4       /* admission failed for another reason (see nao_last_error of
                                    the home context) */
} nao_session_state;
/* state: a nao_session_state; bytes: its device footprint (0 unless resident). */
nao_status nao_server_session_info(nao_server srv, int64_t session, int32_t* state, size_t* bytes,
                                   int64_t* n_basis, int64_t* n_points);
nao_status nao_server_submit(nao_server srv, int64_t session, const double* D, nao_memspace D_space,
                             const double* v, nao_memspace v_space, uint64_t* ticket);
/* A launch that cannot be enqueued or that reports a failure on completion fails its requests
 * (NAO_REQ_FAILED) and returns that status; their sessions stay usable.  A request without v
 * whose session has no potential on the device (its only earlier v came with a request that
 * failed) fails at launch with NAO_ERR_INVALID_ARG. */
nao_status nao_server_step(nao_server srv, int32_t* n_running, int32_t* n_waiting);
nao_status nao_server_poll(nao_server srv, uint64_t ticket, int32_t* state, double* t_submit, double* t_start,
                           double* t_end);
/* Copy a done request's H [N_b][N_b] and/or n [n_points] (caller order) out; either may be NULL.
 * A session keeps one H and n: the result is available until the session's next request
 * starts, after which this call returns NAO_ERR_INVALID_ARG (read a result before submitting
 * the next iteration when every iteration's result is needed).  NAO_ERR_NOT_READY while the
 * request is waiting or running, or when it failed. */
nao_status nao_server_result(nao_server srv, uint64_t ticket, double* H, double* n, nao_memspace space);
void nao_server_destroy(nao_server srv);

#ifdef __cplusplus
}
#endif

#endif /* NAO_H */

/*
 * cpm.h - C ABI of the MI355X (gfx950) Schwarz-preconditioned closest point
 * method solver.
 *
 * Problem (May, Haynes, Ruuth, "Schwarz solvers and preconditioners for the
 * closest point method", arXiv:1909.08734, Section 1): the surface positive
 * Helmholtz equation (c - Delta_S) u = f, c > 0, discretised by the closest
 * point method with the stabilised operator of Section 2.1
 *     A = c I - Delta_S^h,  Delta_S^h = -(6/h^2) I + (Delta^h + (6/h^2) [I 0]) E,
 * and solved by GMRES preconditioned with restricted additive Schwarz (RAS,
 * Dirichlet transmission rows, Section 5.1) or optimized RAS (ORAS, Robin
 * rows of eq. robfo, Section 5.2, with the cross-point weight of Section 5.2.2):
 *     M^{-1} = sum_j R~_j^T A_j^{-1} R_j        (eq. algRAS).
 *
 * Call order (state machine): cpm_create -> cpm_build_band -> cpm_build_operator
 * -> cpm_partition -> cpm_factor -> cpm_solve*. A new operator or partition
 * invalidates the factors (cpm_factor must run again). Calls out of order
 * return CPM_ESTATE; a failed call leaves the previous state intact unless
 * stated otherwise.
 *
 * Vectors: length N_A (number of active band nodes), float64, in band order
 * (active nodes sorted by linear grid index L = (i n1 + j) n2 + k).
 * Pointers named *_dev are device pointers on the context's device, used on
 * the context's stream; all other pointers are host pointers. Every call is
 * synchronous (returns after the device work it issued has finished) unless
 * stated otherwise. Ownership: the context owns all device memory it
 * allocates; caller buffers are only borrowed for the duration of a call.
 *
 * Errors: 0 on success, negative CPM_E* on failure, CPM_ENOTCONV (> 0) as a
 * warning from the solve. cpm_last_error() describes the most recent failure.
 * No C++ exception crosses this boundary.
 */
#ifndef CPM_H
#define CPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cpm_ctx cpm_ctx;

enum {
  CPM_OK = 0,
  CPM_ENOTCONV = 1,    /* solve hit max_iter; u holds the last iterate */
  CPM_EINVAL = -1,     /* invalid argument (message says which) */
  CPM_ESTATE = -2,     /* call out of order */
  CPM_ENOMEM = -3,     /* host or device allocation failed */
  CPM_ESINGULAR = -4,  /* exactly zero pivot in a local LU */
  CPM_EDEVICE = -5,    /* HIP runtime error, or no device (host-only context) */
  CPM_ECALLBACK = -6   /* the closest-point callback returned non-zero */
};

enum { CPM_RAS = 0, CPM_ORAS = 1 };                 /* transmission condition */
enum { CPM_FP64 = 0, CPM_FP32 = 1 };                /* local factor precision */
enum { CPM_PART_OCTANT = 0, CPM_PART_RCB = 1, CPM_PART_GRAPH = 2 };  /* disjoint partition */
enum { CPM_PART_ALIGN = 16 };  /* flag: align interfaces with the surface normals (Section 3.2) */

/*
 * Closest-point callback (the surface representation CP_S of Section 2.1).
 * x: n query points, row-major n x 3. Writes cp (n x 3) = closest points and
 * nrm (n x 3) = unit surface normals at those points. A non-finite cp marks a
 * point whose closest point is undefined (treated as outside every band).
 * Returns 0 on success. Must give the same value for a point however the
 * queries are batched. Called from the thread that called cpm_build_band.
 */
typedef int (*cpm_cp_fn)(void* user, int64_t n, const double* x, double* cp, double* nrm);

typedef struct {
  int32_t iters;        /* total GMRES iterations (preconditioner applications) */
  int32_t cycles;       /* restart cycles */
  int32_t status;       /* CPM_OK or CPM_ENOTCONV */
  int32_t reserved;
  double relres_true;   /* ||f - A u||_2 / ||f||_2 at exit, computed on the device */
  double relres_est;    /* GMRES residual estimate / ||f||_2 at exit */
  double ms;            /* wall time of the solve on the device stream */
  /* Device time of the solve's phases in ms, filled while per-kernel timing
   * is on (cpm_set_timing), else 0: [0] preconditioner applies (eq. algRAS),
   * [1] operator applies (extension and stencil, Section 2.1, including the
   * true residual at each restart; the stencil carries the first
   * Gram-Schmidt pass's dot products), [2] orthogonalisation, norms and the
   * Givens least-squares updates, [3] solution updates and vector copies.
   * For a lockstep batch these are the batch's totals. */
  double phase_ms[4];
} cpm_solve_info;

/* Create a context on HIP device `device` (>= 0). device < 0 gives a
 * host-only context: set-up and queries work, factor/solve return
 * CPM_EDEVICE. The context creates and owns one HIP stream, which it uses
 * until cpm_set_stream names another. */
int cpm_create(cpm_ctx** out, int device);
void cpm_destroy(cpm_ctx* ctx);

/*
 * Stream for the context's device work. caller != 0: the caller's HIP stream
 * `hip_stream` on the context's device (NULL = the device's null stream); it
 * is borrowed, not destroyed, and must stay valid while the context uses it.
 * caller == 0: the context's own stream again (hip_stream ignored). Device
 * work a call issues is queued on that stream after whatever the caller queued
 * there before, so device inputs written by earlier work on the same stream
 * need no device-wide synchronisation; calls still return after their own
 * device work has finished (they synchronise that stream only). On the null
 * stream FGMRES iterations are launched directly (HIP graphs cannot be
 * captured there). EDEVICE for a host-only context. Takes effect at the next
 * call.
 */
int cpm_set_stream(cpm_ctx* ctx, int caller, void* hip_stream);

/*
 * New context on `device` (as cpm_create) holding a copy of src's host
 * set-up: band, operator constant and partition (Sections 2.1, 3, 4). The
 * copy is at src's state capped at "partitioned", so it needs cpm_factor; a
 * different c is set with cpm_build_operator, which keeps the partition. This
 * lets one band and partition serve factorisations for several values of c.
 * src is only read (it may be host-only). ESTATE if src has no band; on error
 * *out is NULL.
 */
int cpm_clone(const cpm_ctx* src, int device, cpm_ctx** out);

/*
 * Thread use: distinct contexts may be used concurrently from different host
 * threads (each has its own device memory and, unless cpm_set_stream names a
 * shared one, its own stream); one context must not be used by two threads at
 * once.
 */
const char* cpm_last_error(const cpm_ctx* ctx);

/*
 * Band (Section 2.1): grid lo + (i,j,k) h covering the box [lo, hi]
 * (n_a = floor((hi_a - lo_a)/h + 1/2) + 1 nodes per axis), active nodes
 * = nodes within rho h of their closest point (tube-radius construction,
 * rho = band_factor, or sqrt(3)(degree+1)/2 when band_factor <= 0), closed
 * so that every interpolation stencil is active; ghost nodes complete the
 * 7-point stencils. Extension rows interpolate with tensor-product Lagrange
 * polynomials of `degree` (2 or 3) at CP(x) (Figure 1). EINVAL if h <= 0,
 * the degree is unsupported, or a ghost or stencil node leaves the box.
 */
int cpm_build_band(cpm_ctx* ctx, cpm_cp_fn fn, void* user, const double lo[3],
                   const double hi[3], double h, int degree, double band_factor);

/* Operator A = c I - Delta_S^h (Section 2.1). EINVAL if c <= 0 or not finite. */
int cpm_build_operator(cpm_ctx* ctx, double c);

/*
 * Change c in the operator A = c I - Delta_S^h (Section 2.1) and keep the
 * factors: they stay those of the c they were made for (c_f), so the
 * preconditioner becomes the Schwarz operator of c_f I - Delta_S^h, and the
 * FGMRES of cpm_solve* still stops on the true residual of the new A (c only
 * moves the diagonal, c + 6/h^2). For serving many values of c from a few
 * cached factorisations. ESTATE before cpm_build_operator; the state is
 * unchanged (factored stays factored).
 * EINVAL if c <= 0 or not finite. cpm_factor_c reports c_f (0 before any
 * factorisation).
 */
int cpm_set_operator_c(cpm_ctx* ctx, double c);
double cpm_factor_c(const cpm_ctx* ctx);

/*
 * Overlapping decomposition (Sections 3, 4, 5).
 * method: CPM_PART_OCTANT (n_sub must be 8), CPM_PART_RCB (recursive
 *   coordinate bisection into n_sub parts; weights = n_sub target weights for
 *   weighted bisection, or NULL) or CPM_PART_GRAPH (recursive bisection of the
 *   6-neighbour graph of the active nodes by breadth-first distance from a
 *   pseudo-peripheral node, Section 3.1's graph view; weights as for RCB),
 *   optionally OR'ed with CPM_PART_ALIGN: degree + 1 passes in which every
 *   node with a neighbour in another part moves to the part of the grid node
 *   nearest to its closest point (Section 3.2). EINVAL if a part ends empty.
 * overlap: N_O >= 0 layers (>= 1 for ORAS).
 * kind: CPM_RAS or CPM_ORAS; alpha: Robin weight (ORAS, > 0);
 * alpha_cross: weight for boundary nodes within 2 N_O h of a cross point
 *   (Section 5.2.2); 0 disables the modification.
 */
int cpm_partition(cpm_ctx* ctx, int method, int n_sub, const double* weights, int overlap,
                  int kind, double alpha, double alpha_cross);

/*
 * Device memory for the factorisation's work arrays (the bordered local
 * matrices and panel scratch): subdomains are factored in consecutive groups
 * whose work arrays fit in `bytes` together (one subdomain larger than that is
 * a group of its own); only W_j stays resident. The result does not depend on
 * the grouping. 0 restores the default, 64 GiB. Takes effect at the next
 * cpm_factor; also used by cpm_footprint_estimate.
 */
int cpm_set_factor_workspace(cpm_ctx* ctx, size_t bytes);
/* Number of subdomain groups the last cpm_factor used (0 before any). */
int cpm_factor_groups(const cpm_ctx* ctx);
/*
 * Preconditioner apply layout. By default v|Sigma_j is staged whole in LDS
 * (160 KB per CU: |Sigma_j| <= 20480); larger subdomains use the chunked form
 * (v staged `columns` at a time, partial row sums kept in LDS). columns > 0
 * forces the chunked form with that width (a multiple of 8, at most 16384);
 * 0 restores the default. Takes effect at the next cpm_factor. EINVAL for
 * other values. cpm_precond_chunk reports the width in use (0: unchunked).
 */
int cpm_set_precond_chunk(cpm_ctx* ctx, int columns);
int cpm_precond_chunk(const cpm_ctx* ctx);

/*
 * Tiling of the (unchunked, single right-hand side) preconditioner apply:
 * rows of W_j each wave streams at once, 16-byte chunks in flight per row and
 * apply blocks per resident block slot. 0: 2 rows, 2 chunks, 2 blocks per
 * slot (default after cpm_factor); 1: 4, 1, 2; 2: 2, 2, 1.5; 3: 4, 1, 3;
 * 4: 4, 4, 1; 5: 4, 4, 2; 6: 8, 2, 2; 7: 4, 2, 2. Every tiling forms each
 * row's sum in the same order, so results do not depend on it; only the
 * speed does.
 * cpm_set_precond_tiling re-plans the apply blocks for the tiling's occupancy
 * (ESTATE before cpm_factor or with the chunked apply, EINVAL out of range).
 * cpm_autotune_precond times every tiling `reps` times on the resident factors,
 * each apply taking a vector that an operator apply has just written (as
 * inside FGMRES; per-launch HIP events on the context stream, the kernel
 * timers of cpm_kernel_time left unchanged), keeps the fastest and returns it
 * in *best (may be NULL); ms (may be NULL) receives the CPM_PRECOND_TILINGS
 * average apply times in ms.
 */
#define CPM_PRECOND_TILINGS 8
int cpm_set_precond_tiling(cpm_ctx* ctx, int tiling);
int cpm_precond_tiling(const cpm_ctx* ctx);
int cpm_autotune_precond(cpm_ctx* ctx, int reps, int* best, double* ms);

/*
 * Tile of the LU's matrix-core trailing updates (the Schur-complement update
 * after each outer block of 128 columns): rows x 64 columns with rows = 64 or
 * 128; 0 (default) takes the tile cpm_autotune_factor chose for this device
 * architecture and precision in this process, else 128. Both tiles form every
 * element's sum in the same order, so the factors have the same values; only
 * the speed differs. Takes effect at the next cpm_factor. cpm_factor_tile reports
 * the tile of the resident factors (0 before any). EINVAL for other values.
 *
 * cpm_autotune_factor factors the partitioned problem in `prec` once with
 * each tile, times the update launches (HIP events; kernel timers left
 * unchanged), caches the faster for the architecture and precision (used by
 * later factorisations with tile 0, any context) and leaves the factors of the
 * faster resident, as cpm_factor would. *best (may be NULL) receives its rows,
 * ms (may be NULL) the two update times in ms (64, then 128).
 */
int cpm_set_factor_tile(cpm_ctx* ctx, int rows);
int cpm_factor_tile(const cpm_ctx* ctx);
int cpm_autotune_factor(cpm_ctx* ctx, int prec, int* best, double* ms);

/*
 * Matrix-core work of the resident factorisation's Schur-complement updates
 * (Section 5, LU of the local problems): 2 x rows x cols x k flops for every
 * update tile computed, whole tiles as the matrix cores run them. Tiles whose
 * multipliers or U12 block are exactly zero are not computed (they would
 * change nothing), so this is well below the dense count of the bordered
 * matrices. *flops receives it; ESTATE before cpm_factor.
 */
int cpm_factor_flops(const cpm_ctx* ctx, double* flops);

/*
 * Tiling of the apply for several right-hand sides at once (the lockstep
 * batches of cpm_solve_device). A tiling names rows of W_j per wave, 16-byte
 * chunks in flight per row, whether each wave alternates two such register
 * sets (the loads of the next chunks issued before the products of the
 * current ones), and the apply blocks planned per resident block slot:
 *   0: 8, 1, -, 1   1: 8, 1, -, 2 (FP32 default after cpm_factor)   2: 8, 1, -, 4
 *   3: 4, 2, two sets, 1   4: 4, 2, two sets, 2   5: 4, 2, two sets, 4 (FP64 default)
 *   6: 4, 1, two sets, 2   7: 4, 2, -, 2
 * Every tiling forms each right-hand side's sums as the single apply does, so
 * results do not depend on it. cpm_set_multi_tiling needs resident factors
 * (ESTATE before cpm_factor; a new factorisation restores the default) and
 * re-plans the blocks. cpm_autotune_multi times every tiling `reps` times on
 * the resident factors with the widest batch that fits (ESTATE when none
 * does), keeps the fastest, returns it in *best and the CPM_MULTI_TILINGS
 * average apply times in ms (both may be NULL); kernel timers are left
 * unchanged.
 */
#define CPM_MULTI_TILINGS 8
int cpm_set_multi_tiling(cpm_ctx* ctx, int tiling);
int cpm_multi_tiling(const cpm_ctx* ctx);
int cpm_autotune_multi(cpm_ctx* ctx, int reps, int* best, double* ms);

/*
 * Kernel of the operator apply's extension step (Section 2.1, e = E x over
 * the band): 0 (default) reads each row in a compact form (its local stencil
 * coordinates, from which the Lagrange weights are formed, and its z-line
 * starts as 16-bit increments: 64 bytes a row for degree 3) and gathers its
 * (p+1)^3 stencil values of x from device memory; 1 groups the rows by the
 * grid position of their stencils and stages each group's x values, p+1
 * contiguous intervals of band indices, in LDS first (used while the largest
 * group's x fits in 64 KB); 2 reads the full stored rows (weights and every
 * z-line start, 160 bytes a row for degree 3) and gathers. A kernel that
 * cannot be used falls back to 2.
 * Both form every sum in the same order, so results do not depend on the
 * choice. cpm_operator_kernel reports the kernel in use. EINVAL for other
 * values.
 */
int cpm_set_operator_kernel(cpm_ctx* ctx, int kernel);
int cpm_operator_kernel(const cpm_ctx* ctx);

/*
 * FGMRES iterations as HIP graphs (off by default): each iteration's kernels
 * for a given position k in the restart cycle are captured once and replayed;
 * the graphs are dropped whenever the factors, the operator, the Krylov space
 * or the apply plan change. Results are the same either way (replaying costs
 * a few microseconds more per iteration than direct launches on ROCm 7, hence
 * the default). Not used while per-kernel timing is on, nor for batches of
 * right-hand sides.
 */
int cpm_set_graphs(cpm_ctx* ctx, int on);

/*
 * Local operators A_j (eq. localOP) assembled on the device and factored by
 * batched dense LU with partial pivoting (Section 5) in `prec`; the factors
 * are reduced to the restricted local solution operators
 * W_j = R~_j A_j^{-1} R_j^T (rows Sigma~_j, columns Sigma_j) kept resident.
 * ESINGULAR if a pivot is exactly zero; ENOMEM if the device memory is short.
 */
int cpm_factor(cpm_ctx* ctx, int prec);

/*
 * Solve A u = f for nrhs right-hand sides (column-major N_A x nrhs, host
 * pointers) with restarted right-preconditioned FGMRES(restart), x0 = 0,
 * until ||f - A u|| <= tol ||f|| (true residual). info may be NULL (else
 * nrhs entries). EINVAL for tol <= 0, max_iter < 1, restart < 1 or > 64,
 * or a non-finite f. Returns CPM_ENOTCONV if some RHS hit max_iter.
 */
int cpm_solve(cpm_ctx* ctx, const double* f, double* u, int nrhs, double tol, int max_iter,
              int restart, cpm_solve_info* info);
/*
 * Same with device pointers (inputs resident in HBM). With nrhs >= 2 the
 * right-hand sides are solved in lockstep batches of up to 4 that share each
 * pass over the factors (when v|Sigma_j of all of them fits in LDS); every
 * right-hand side follows the single-solve sequence, so results, iteration
 * counts and statuses equal separate solves; info[q].ms is the batch's time.
 */
int cpm_solve_device(cpm_ctx* ctx, const double* f_dev, double* u_dev, int nrhs, double tol,
                     int max_iter, int restart, cpm_solve_info* info);

/*
 * Implicit steps with resident factors (repeated right-hand sides, e.g.
 * backward Euler for u_t = Delta_S u with c = 1/dt, which solves
 * (c - Delta_S) u^{n+1} = c u^n): u_0 solves A u_0 = f, and u_k solves
 * A u_k = scale * u_{k-1} for k = 1 .. nsteps-1, each by the FGMRES of
 * cpm_solve. Device pointers: f_dev (N_A), u_dev (N_A x nsteps,
 * column-major, caller-owned). info may be NULL (else nsteps entries).
 * EINVAL for nsteps < 0, a non-finite scale, or the arguments cpm_solve
 * rejects; returns CPM_ENOTCONV if some step hit max_iter.
 */
int cpm_solve_steps(cpm_ctx* ctx, const double* f_dev, double* u_dev, int nsteps, double scale,
                    double tol, int max_iter, int restart, cpm_solve_info* info);

/*
 * The paper's formulation (Section 2.2 preconditions on the left; Section 6
 * stops when the residual norm has fallen by 10^6): GMRES(restart) on
 * M^{-1} A u = M^{-1} f from u = 0 until ||M^{-1}(f - A u)|| <= tol
 * ||M^{-1} f|| (use tol = 1e-6 for the paper's rule), CGS2 Arnoldi; device
 * pointers, one right-hand side. info->relres_est is that preconditioned
 * ratio at exit, info->relres_true = ||f - A u|| / ||f||; the true residual
 * this rule leaves depends on M (and so on the factor precision), which is
 * why cpm_solve stops on the true residual instead. Same errors as cpm_solve;
 * CPM_ENOTCONV at max_iter.
 */
int cpm_solve_left(cpm_ctx* ctx, const double* f_dev, double* u_dev, double tol, int max_iter, int restart,
                   cpm_solve_info* info);

/* (O)RAS as a stationary solver (eq. algRAS): u <- u + M^{-1}(f - A u) from
 * u = 0 until ||f - A u|| <= tol ||f|| or max_iter updates; device pointers
 * (N_A, float64). info->iters = updates applied, relres_true = final true
 * relative residual. Same errors as cpm_solve; CPM_ENOTCONV at max_iter. */
int cpm_solve_stationary(cpm_ctx* ctx, const double* f_dev, double* u_dev, double tol, int max_iter,
                         cpm_solve_info* info);

/* Single applications on device vectors, for checking and profiling.
 * y = A x (Section 2.1);  z = M^{-1} v (eq. algRAS) after cpm_factor. */
int cpm_apply_operator(cpm_ctx* ctx, const double* x_dev, double* y_dev);
int cpm_apply_precond(cpm_ctx* ctx, const double* v_dev, double* z_dev);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): y = A x
 * exactly as cpm_apply_operator, with the extension values E x held in a
 * static device array of the library (one per device, 2^21 rows = 16 MiB,
 * held until the process ends) instead of the context's scratch. Calls no
 * allocating routine. EINVAL if the band has more than 2^21 rows (N_A + N_G).
 * All contexts on a device share its array, so calls that overlap on one
 * device (from different threads or streams) race; calls on one stream are
 * ordered and every call writes all the rows it reads.
 */
int cpm_apply_operator_noalloc(cpm_ctx* ctx, const double* x_dev, double* y_dev);

/* ---- queries (host copies of the set-up; any pointer may be NULL) ---- */
int cpm_band_sizes(const cpm_ctx* ctx, int64_t* n_act, int64_t* n_ghost, int64_t shape[3]);
/* lin: N_T linear indices (actives then ghosts); cp, nrm: N_T x 3; nbr: N_A x 6
 * band indices (x-,x+,y-,y+,z-,z+); base: N_T x 3 first stencil node per axis;
 * wts: N_T x 3 x (degree+1) one-dimensional weights. */
int cpm_band_arrays(const cpm_ctx* ctx, int64_t* lin, double* cp, double* nrm, int32_t* nbr,
                    int32_t* base, double* wts);
int cpm_partition_info(const cpm_ctx* ctx, int* n_sub, int32_t* part, uint8_t* cross);
/* sizes[5] = |Sigma~_j|, |Sigma_j|, |F_j|, |Sigma_j^G|, |B_j| */
int cpm_subdomain_sizes(const cpm_ctx* ctx, int j, int64_t sizes[5]);
/* sorted band indices of each set; xstar, s, alpha are per B node (ORAS). */
int cpm_subdomain_sets(const cpm_ctx* ctx, int j, int32_t* tilde, int32_t* sigma, int32_t* fin,
                       int32_t* ghost, int32_t* bnd, int32_t* xstar, double* s, double* alpha);
/* Elimination order of the local unknowns used by cpm_factor (Section 5: the
 * local problems are solved by LU): *n_unk receives n_j (|Sigma_j| + |B_j| for
 * ORAS, |Sigma_j| for RAS) and order[p] the local unknown at position p, an
 * index into [Sigma_j ; B_j] (either pointer may be NULL). Reverse
 * Cuthill-McKee on the symmetrised pattern of A_j, computed by cpm_partition;
 * it decides which products of the bordered LU are exactly zero, and leaves
 * W_j as it is up to rounding. */
int cpm_subdomain_order(const cpm_ctx* ctx, int j, int64_t* n_unk, int32_t* order);
/* W_j (|Sigma~_j| x |Sigma_j|, row-major) copied to host as float64. */
int cpm_factor_export(cpm_ctx* ctx, int j, double* w);
/* Device bytes held for the band, operator, factors and Krylov workspace. */
size_t cpm_footprint_bytes(const cpm_ctx* ctx);
/*
 * Device bytes a factorisation in `prec` would need, before making it
 * (partitioned context, host-only allowed): *resident = held afterwards with
 * a Krylov space of `restart` vectors (0: none), *peak = the most held while
 * cpm_factor runs. For admission of work by memory footprint. Either output
 * may be NULL. ESTATE before cpm_partition; EINVAL for an unknown prec or
 * restart outside [0, 64].
 */
int cpm_footprint_estimate(const cpm_ctx* ctx, int prec, int restart, size_t* resident,
                           size_t* peak);

/*
 * Cache of large device work buffers (the bordered local matrices of a
 * factorisation and the W arenas, buffers of 64 MiB or more), process-wide
 * with one cache per device. Returning such a buffer to the driver becomes
 * slow once the device memory that was never used has been handed out
 * (tenths of a second per 10 GB), so released buffers are kept and reused by
 * later factorisations on the same device, from any context, by requests of
 * at least eight ninths of a buffer's size (a much larger buffer is not lent
 * out, so a request holds about what its caller budgeted). At most `bytes`
 * idle bytes are kept per device (default 64 GiB; the longest idle buffer is
 * freed first); 0 keeps none. Lowering the cap frees idle buffers at once.
 * An allocation that fails empties its device's cache and is tried again.
 * The idle bytes are not part of cpm_footprint_bytes or of the estimates
 * above: callers that budget device memory should set a cap they can
 * afford. Returns 0; *idle_before (may be NULL) gets the idle bytes held on
 * all devices before the call.
 */
int cpm_set_workspace_cache(size_t bytes, size_t* idle_before);
/* The cap, the idle bytes held and the cached buffers in use on `device`
 * (any output may be NULL). EINVAL for a negative device. */
int cpm_workspace_cache(int device, size_t* cap, size_t* idle, size_t* in_use);

/* Per-kernel timing with HIP events on the context stream (off by default;
 * the events ride on the kernel dispatches, no extra packets). which:
 * 0 = preconditioner apply, 1 = extension apply, 2 = stencil apply (also in
 * its fused form with the first Gram-Schmidt dot products), 3 = LU trailing
 * update, 4 = orthogonalisation, norms and least squares, 5 = solution
 * updates and vector copies. total_ms and launches since the last reset. */
#define CPM_N_TIMERS 6
int cpm_set_timing(cpm_ctx* ctx, int on);
int cpm_kernel_time(cpm_ctx* ctx, int which, double* total_ms, int64_t* launches);

/* Diagnostic: run the matrix-core tile of the LU trailing update once on
 * device `device`: c (64x64, row-major, in/out) -= a (64 x kb, row stride 128)
 * * b (kb x 64, row-major), 1 <= kb <= 128, in `prec` (CPM_FP64 or CPM_FP32;
 * values are rounded to float for CPM_FP32). Host pointers. */
int cpm_selftest_tile(int device, int prec, const double* a, const double* b, double* c, int kb);

#ifdef __cplusplus
}
#endif
#endif /* CPM_H */

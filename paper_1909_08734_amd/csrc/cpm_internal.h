// Internal declarations of the CPM Schwarz library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "cpm.h"

namespace cpm {

struct HostSlot;

// Band and extension data (Section 2.1). Band order: actives sorted by L, then ghosts.
struct Band {
  double lo[3] = {0, 0, 0};
  double h = 0;
  int p = 0;
  int64_t n[3] = {0, 0, 0};
  int64_t n_act = 0, n_ghost = 0;
  std::vector<int64_t> lin;    // N_T linear indices
  std::vector<int32_t> ijk;    // N_T x 3
  std::vector<double> xyz;     // N_T x 3 node coordinates
  std::vector<double> cp;      // N_T x 3 closest points
  std::vector<double> nrm;     // N_T x 3 normals at the closest points
  std::vector<int32_t> nbr;    // N_A x 6 band indices (x-,x+,y-,y+,z-,z+)
  std::vector<int32_t> base;   // N_T x 3 first stencil node per axis
  std::vector<double> wts;     // N_T x 3 x (p+1) one-dimensional weights
  std::vector<int32_t> lines;  // N_T x (p+1)^2 band index of each stencil z-line's first node
  int64_t total() const { return n_act + n_ghost; }
};

struct Sub {
  std::vector<int32_t> tilde, sigma, fin, ghost, bnd, xstar;
  std::vector<double> s, alpha;
  // Elimination order of the local unknowns for the factorisation: position p
  // holds local unknown order[p] (an index into [Sigma_j ; B_j]); reverse
  // Cuthill-McKee on the pattern of A_j, so that the LU factors stay inside a
  // narrow profile and most of the bordered update is exactly zero.
  std::vector<int32_t> order;
  // reach[c]: one past the last position whose row of A_j has its first
  // nonzero in a column <= c (in elimination order). Rows below reach[c] are
  // zero in columns <= c and stay so under partial pivoting, so the
  // elimination of column c only involves positions below reach[c].
  std::vector<int32_t> reach;
};

struct Decomp {
  int n_sub = 0, kind = CPM_RAS, overlap = 0;
  double alpha = 0, alpha_cross = 0;
  std::vector<int32_t> part;
  std::vector<uint8_t> cross;
  std::vector<Sub> subs;
};

// Host set-up (setup_band.cpp, setup_partition.cpp). Return CPM_* codes.
int build_band(Band& b, cpm_cp_fn fn, void* user, const double lo[3], const double hi[3],
               double h, int p, double band_factor, std::string& err);
int build_decomposition(const Band& b, Decomp& d, int method, int n_sub, const double* weights,
                        int overlap, int kind, double alpha, double alpha_cross,
                        std::string& err);

// Per-subdomain descriptor shared by the factor and apply kernels.
struct SubDesc {
  int32_t m;         // |Sigma_j|
  int32_t n;         // local unknowns: m (+ |B_j| for ORAS)
  int32_t t;         // |Sigma~_j|
  int32_t u_off;     // offset of the unknown list / lookup tables
  int32_t t_off;     // offset of Sigma~_j lists
  int32_t ldw;       // row stride of W_j
  int64_t w_off;     // element offset of W_j in the W arena
  int64_t a_off;     // element offset of the augmented matrix in the factor arena
  int32_t lda;       // row stride of the augmented matrix
  int32_t rows;      // n + t
  int32_t cols;      // n + m
  int32_t blk_off;   // first apply block of this subdomain
  int32_t rpb;       // rows of W_j per apply block
  int32_t pb_off;    // first entry of this subdomain in the panel row-bound table
};

// A group of extension rows for the LDS-staged operator apply: rows whose
// interpolation stencils start in grid plane i = bi and in a window of
// columns j; the x values all their stencils read lie, plane by plane, in P+1
// contiguous intervals of band indices [lo[a], lo[a] + off[a+1] - off[a]),
// staged in LDS at off[a].
struct ExtGroup {
  int32_t row0;    // first row of the group in apply order
  int32_t nrows;   // rows in the group
  int32_t lo[4];   // first band index of each plane's interval
  int32_t off[5];  // LDS offsets of the intervals; off[P+1] = values staged
  int32_t pad;
};

enum {
  TIMER_PRECOND = 0,
  TIMER_EXTEND = 1,
  TIMER_STENCIL = 2,
  TIMER_LU_GEMM = 3,
  TIMER_KRYLOV = 4,  // orthogonalisation, norms, least squares
  TIMER_UPDATE = 5,  // solution updates and vector copies
  N_TIMERS = CPM_N_TIMERS
};

struct Timer {
  bool on = false;
  double ms[N_TIMERS] = {};
  int64_t count[N_TIMERS] = {};
  std::vector<hipEvent_t> pool;   // event pairs recorded since the last harvest
  std::vector<int> which;
  size_t used = 0;
};

// Device-resident state.
struct Dev {
  // operator (extension rows stored in apply order: grouped by stencil base)
  int32_t* lines = nullptr;   // N_T x (p+1)^2, apply order
  double* wts = nullptr;      // N_T x 3(p+1), apply order
  int32_t* ext_perm = nullptr;  // apply position -> band row
  int32_t* ext_pos = nullptr;   // band row -> apply position
  ExtGroup* ext_groups = nullptr;
  int n_ext_groups = 0;
  size_t ext_lds = 0;           // LDS bytes of the largest group
  int op_kernel = 0;            // 0: compact rows, gathers; 1: LDS-staged groups; 2: full rows, gathers
  double* ext_s = nullptr;      // compact rows: 3 x N_T local stencil coordinates (apply order)
  int32_t* ext_start = nullptr; // (p+1) x N_T first z-line start of each stencil plane
  uint16_t* ext_step = nullptr; // (p+1) p x N_T increments between a plane's z-line starts
  bool compact = false;         // the compact rows exist (increments fit 16 bits)
  int32_t* nbr = nullptr;     // 6 x N_A (structure of arrays)
  double* e = nullptr;        // N_T extension scratch
  double* static_e = nullptr; // device address of the static extension scratch (no-allocation apply)
  // preconditioner
  SubDesc* desc = nullptr;
  int32_t* blk_sub = nullptr;   // apply block -> subdomain
  int32_t* sig_idx = nullptr;   // concatenated Sigma_j (band indices)
  int32_t* tilde_idx = nullptr; // concatenated Sigma~_j (band indices)
  void* W = nullptr;            // W arena (float or double)
  int prec = -1;
  int n_blocks = 0;
  int max_m = 0;
  int n_groups = 0;             // subdomain groups of the last factorisation
  int chunk = 0;                // 0: v|Sigma_j staged whole; else columns per pass (chunked apply)
  int tiling = 0;               // tiling of the unchunked apply (see dev_set_tiling)
  int multi_tiling = 0;         // tiling of the several-right-hand-side apply
  SubDesc* mdesc = nullptr;     // its plan: descriptors with their own block fields
  int32_t* mblk_sub = nullptr;  // its block -> subdomain table
  int m_n_blocks = 0;
  int factor_tile = 0;          // rows of the LU trailing-update tile: 0 = tuned (or 128), 64 or 128
  int factor_tile_used = 0;     // the tile of the resident factors
  double factor_flops = 0;      // matrix-core flops of the last factorisation's Schur-complement updates
  std::vector<SubDesc> hdesc;   // host copy of the apply descriptors
  int chunk_req = 0;            // requested chunk (0: only when v|Sigma_j exceeds LDS)
  size_t ws_limit = size_t(64) << 30;  // factor workspace per group, bytes
  size_t w_bytes = 0;
  // Krylov workspace
  int restart = 0;
  int64_t ld = 0;               // padded vector length
  double* V = nullptr;          // (restart+1) x ld
  double* Z = nullptr;          // restart x ld
  double* F = nullptr;          // right-hand side of the current implicit step (ld)
  double* part = nullptr;       // partial sums
  double* small = nullptr;      // H, cs, sn, g, y, h1, h2, scalars
  struct HostSlot* slots = nullptr;  // mapped pinned scalars, one slot per step (host view)
  struct HostSlot* slots_dev = nullptr;  // the same memory, device view
  unsigned long long ticket = 0;     // last ticket handed out
  size_t krylov_bytes = 0;
  // Krylov workspace of a batch of right-hand sides solved in lockstep
  int b_restart = 0, b_n = 0;
  double* bV = nullptr;         // b_n x (restart+1) x ld
  double* bZ = nullptr;         // b_n x restart x ld
  double* bE = nullptr;         // b_n x N_T extension scratch
  double* bpart = nullptr;      // b_n x partial sums
  double* bsmall = nullptr;     // b_n x small buffer
  struct HostSlot* bslots = nullptr;      // b_n x (restart+2), host view
  struct HostSlot* bslots_dev = nullptr;  // device view
  size_t batch_bytes = 0;
  // FGMRES iteration k captured as HIP graph k (single right-hand side)
  bool use_graphs = false;
  std::vector<hipGraphExec_t> graphs;
  size_t op_bytes = 0;
};

}  // namespace cpm

struct cpm_ctx {
  int device = -1;
  bool host_only = true;
  hipStream_t own_stream = nullptr;  // created with the context
  hipStream_t stream = nullptr;      // the stream in use: own_stream or the caller's
  std::string err;
  int state = 0;  // 0 created, 1 band, 2 operator, 3 partition, 4 factored
  double c = 0;         // c of the operator A = c I - Delta_S^h
  double c_factor = 0;  // c the resident factors were made for
  cpm::Band band;
  cpm::Decomp dec;
  cpm::Dev dev;
  cpm::Timer timer;
};

namespace cpm {
// Device orchestration (device.hip).
// Uploads the operator arrays of `b`; on success the context's previous
// device state (operator, factors, Krylov space) is freed and replaced, on
// failure it is left as it was.
int dev_upload_operator(cpm_ctx* ctx, const Band& b);
int dev_factor(cpm_ctx* ctx, int prec);
int dev_apply_operator(cpm_ctx* ctx, const double* x, double* y);
// Rows of the static extension scratch used by dev_apply_operator_noalloc.
constexpr int64_t NOALLOC_ROWS = int64_t(1) << 21;
int dev_init_context(cpm_ctx* ctx);  // once per context, device current
int dev_apply_operator_noalloc(cpm_ctx* ctx, const double* x, double* y);
int dev_apply_precond(cpm_ctx* ctx, const double* v, double* z);
int dev_solve(cpm_ctx* ctx, const double* f, double* u, double tol, int max_iter, int restart,
              cpm_solve_info* info);
int dev_solve_left(cpm_ctx* ctx, const double* f, double* u, double tol, int max_iter, int restart,
                   cpm_solve_info* info);
int dev_stationary(cpm_ctx* ctx, const double* f, double* u, double tol, int max_iter, cpm_solve_info* info);
int dev_solve_batch(cpm_ctx* ctx, const double* f, double* u, int nb, double tol, int max_iter, int restart,
                    cpm_solve_info* info);
int dev_batch_width(cpm_ctx* ctx, int nrhs);
int dev_set_tiling(cpm_ctx* ctx, int t);
int dev_set_operator_kernel(cpm_ctx* ctx, int k);
int dev_set_multi_tiling(cpm_ctx* ctx, int t);
int tuned_factor_tile(cpm_ctx* ctx, int prec);
int dev_autotune_factor(cpm_ctx* ctx, int prec, int* best, double* ms);
int dev_autotune_multi(cpm_ctx* ctx, int reps, int* best, double* ms);
void drop_graphs(Dev& d);
int dev_autotune(cpm_ctx* ctx, int reps, int* best, double* ms);
int dev_solve_steps(cpm_ctx* ctx, const double* f, double* u, int nsteps, double scale, double tol, int max_iter,
                    int restart, cpm_solve_info* info);
int dev_export_w(cpm_ctx* ctx, int j, double* w);
void dev_estimate(const cpm_ctx* ctx, int prec, int restart, size_t* resident, size_t* peak);
void dev_free_all(cpm_ctx* ctx);
void dev_free_factor(cpm_ctx* ctx);
void timer_harvest(cpm_ctx* ctx);
// Per-device cache of large work buffers (device.hip): the cap on idle bytes
// per device (returns the idle bytes held before), and a device's figures.
size_t pool_set_cap(size_t bytes);
void pool_stats(int dev, size_t* cap, size_t* idle, size_t* in_use);
}  // namespace cpm

// Device orchestration: operator upload, local operator factorisation,
// preconditioner and operator applies, and the FGMRES driver.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include <map>
#include <mutex>
#include <unordered_map>

#include <hip/hip_ext.h>

#include "kernels.h"

namespace cpm {
namespace {

#define HIPCHK(expr)                                                            \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);             \
      return e_ == hipErrorOutOfMemory ? CPM_ENOMEM : CPM_EDEVICE;              \
    }                                                                           \
  } while (0)

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }
inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

template <class P>
void dfree(P*& p) {
  if (p) hipFree((void*)p);
  p = nullptr;
}

// ---------------------------------------------------------------------------
// Reuse of large device buffers. Giving a multi-gigabyte buffer back to the
// driver turns slow once the device memory that was never used has been
// handed out (measured on MI355X with ROCm 7: about 0.7 s per 25 GB freed,
// against about 0.2 s for a whole factorisation at that size), and every
// factorisation allocates its bordered matrices and a new W arena. Buffers of
// at least kPoolMin bytes are therefore released into a per-device cache and
// handed out again to requests of at least eight ninths of their size
// (smallest that fits; a much larger buffer is not lent out, so the memory a
// request holds stays close to what its caller budgeted for it). The cache
// keeps at most g_pool_cap idle bytes per device, evicting the longest idle
// first; an allocation that fails empties the device's cache and is tried
// once more. A buffer is released only after the work using it has finished
// (its stream synchronized), so any stream may take it next.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kPoolMin = size_t(64) << 20;
constexpr size_t kPoolCapDefault = size_t(64) << 30;
struct PoolBuf {
  void* p;
  size_t bytes;
  uint64_t stamp;
};
struct DevPool {
  std::mutex mu;
  std::vector<PoolBuf> idle;
  std::unordered_map<void*, size_t> live;  // pooled buffers in use -> their size
  size_t idle_bytes = 0;
  uint64_t clock = 0;
};
constexpr int kPoolDevices = 64;
DevPool g_pool[kPoolDevices];
std::atomic<size_t> g_pool_cap{kPoolCapDefault};

DevPool* pool_of(int dev) { return dev >= 0 && dev < kPoolDevices ? &g_pool[dev] : nullptr; }

// Free idle buffers of `pl` (longest idle first) until at most `keep` bytes stay.
void pool_shrink(DevPool& pl, size_t keep) {
  while (pl.idle_bytes > keep && !pl.idle.empty()) {
    size_t q = 0;
    for (size_t k = 1; k < pl.idle.size(); ++k)
      if (pl.idle[k].stamp < pl.idle[q].stamp) q = k;
    (void)hipFree(pl.idle[q].p);
    pl.idle_bytes -= pl.idle[q].bytes;
    pl.idle.erase(pl.idle.begin() + q);
  }
}
}  // namespace

// Device allocation through the cache (the calling thread's current device).
hipError_t pool_malloc(void** p, size_t bytes) {
  *p = nullptr;
  int dev = -1;
  (void)hipGetDevice(&dev);
  DevPool* pl = pool_of(dev);
  if (!pl || bytes < kPoolMin) return hipMalloc(p, bytes);
  {
    std::lock_guard<std::mutex> lk(pl->mu);
    size_t best = pl->idle.size();
    for (size_t k = 0; k < pl->idle.size(); ++k)
      if (pl->idle[k].bytes >= bytes && pl->idle[k].bytes - bytes <= bytes / 8 &&
          (best == pl->idle.size() || pl->idle[k].bytes < pl->idle[best].bytes))
        best = k;
    if (best < pl->idle.size()) {
      *p = pl->idle[best].p;
      pl->live[*p] = pl->idle[best].bytes;
      pl->idle_bytes -= pl->idle[best].bytes;
      pl->idle.erase(pl->idle.begin() + best);
      return hipSuccess;
    }
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    {
      std::lock_guard<std::mutex> lk(pl->mu);
      pool_shrink(*pl, 0);
    }
    e = hipMalloc(p, bytes);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    return e;
  }
  std::lock_guard<std::mutex> lk(pl->mu);
  pl->live[*p] = bytes;
  return hipSuccess;
}

// Release a buffer from pool_malloc (or hipMalloc) on the current device.
template <class P>
void pool_free(P*& p) {
  if (!p) return;
  int dev = -1;
  (void)hipGetDevice(&dev);
  DevPool* pl = pool_of(dev);
  bool pooled = false;
  if (pl) {
    std::lock_guard<std::mutex> lk(pl->mu);
    auto it = pl->live.find((void*)p);
    if (it != pl->live.end()) {
      pooled = true;
      pl->idle.push_back(PoolBuf{(void*)p, it->second, ++pl->clock});
      pl->idle_bytes += it->second;
      pl->live.erase(it);
      pool_shrink(*pl, g_pool_cap.load());
    }
  }
  if (!pooled) (void)hipFree((void*)p);
  p = nullptr;
}


template <class T>
int upload(cpm_ctx* ctx, T** dst, const std::vector<T>& src) {
  *dst = nullptr;
  if (src.empty()) return CPM_OK;
  HIPCHK(hipMalloc((void**)dst, src.size() * sizeof(T)));
  HIPCHK(hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, ctx->stream));
  return CPM_OK;
}

// Launch on the context stream; with per-kernel timing on, the dispatch
// itself carries the start/stop events (no extra packets in the stream).
template <typename... KArgs, typename... Args>
void launch(cpm_ctx* ctx, int which, void (*kernel)(KArgs...), dim3 grid, dim3 block, size_t lds,
            Args... args) {
  Timer& t = ctx->timer;
  if (!t.on) {
    hipLaunchKernelGGL(kernel, grid, block, lds, ctx->stream, static_cast<KArgs>(args)...);
    return;
  }
  if (t.used + 2 > t.pool.size()) {
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    t.pool.push_back(a);
    t.pool.push_back(b);
  }
  hipEvent_t e0 = t.pool[t.used], e1 = t.pool[t.used + 1];
  t.which.push_back(which);
  t.used += 2;
  hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)lds, ctx->stream, e0, e1, 0,
                        static_cast<KArgs>(args)...);
}

}  // namespace

void timer_harvest(cpm_ctx* ctx) {
  Timer& t = ctx->timer;
  if (t.used == 0) return;
  hipEventSynchronize(t.pool[t.used - 1]);  // the stop event of the last timed launch
  for (size_t q = 0; q < t.which.size(); ++q) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.pool[2 * q], t.pool[2 * q + 1]) == hipSuccess) {
      t.ms[t.which[q]] += ms;
      t.count[t.which[q]] += 1;
    }
  }
  t.which.clear();
  t.used = 0;
}

// Device time of a solve's phases from the kernel timers (timing on only):
// snapshot the totals before the solve, difference after it.
struct PhaseClock {
  bool on = false;
  double ms0[N_TIMERS] = {};
  void start(cpm_ctx* ctx) {
    on = ctx->timer.on;
    if (!on) return;
    timer_harvest(ctx);
    for (int q = 0; q < N_TIMERS; ++q) ms0[q] = ctx->timer.ms[q];
  }
  void stop(cpm_ctx* ctx, double phase[4]) {
    for (int q = 0; q < 4; ++q) phase[q] = 0.0;
    if (!on) return;
    timer_harvest(ctx);
    const double* t = ctx->timer.ms;
    phase[0] = t[TIMER_PRECOND] - ms0[TIMER_PRECOND];
    phase[1] = (t[TIMER_EXTEND] - ms0[TIMER_EXTEND]) + (t[TIMER_STENCIL] - ms0[TIMER_STENCIL]);
    phase[2] = t[TIMER_KRYLOV] - ms0[TIMER_KRYLOV];
    phase[3] = t[TIMER_UPDATE] - ms0[TIMER_UPDATE];
  }
};

// Captured iterations hold the device addresses and launch shapes of the
// moment they were captured: drop them whenever any of those change.
void drop_graphs(Dev& d) {
  for (hipGraphExec_t g : d.graphs)
    if (g) hipGraphExecDestroy(g);
  d.graphs.clear();
}

void dev_free_factor(cpm_ctx* ctx) {
  Dev& d = ctx->dev;
  hipStreamSynchronize(ctx->stream);
  drop_graphs(d);
  dfree(d.desc);
  dfree(d.blk_sub);
  dfree(d.mdesc);
  dfree(d.mblk_sub);
  d.m_n_blocks = 0;
  dfree(d.sig_idx);
  dfree(d.tilde_idx);
  pool_free(d.W);
  d.prec = -1;
  d.n_blocks = 0;
  d.w_bytes = 0;
}

static void free_krylov(cpm_ctx* ctx) {
  Dev& d = ctx->dev;
  drop_graphs(d);
  dfree(d.V);
  dfree(d.Z);
  dfree(d.F);
  dfree(d.part);
  dfree(d.small);
  if (d.slots) hipHostFree(d.slots);
  d.slots = nullptr;
  d.slots_dev = nullptr;
  dfree(d.bV);
  dfree(d.bZ);
  dfree(d.bE);
  dfree(d.bpart);
  dfree(d.bsmall);
  if (d.bslots) hipHostFree(d.bslots);
  d.bslots = nullptr;
  d.bslots_dev = nullptr;
  d.b_restart = d.b_n = 0;
  d.batch_bytes = 0;
  d.restart = 0;
  d.krylov_bytes = 0;
}

void dev_free_all(cpm_ctx* ctx) {
  Dev& d = ctx->dev;
  dev_free_factor(ctx);
  free_krylov(ctx);
  dfree(d.lines);
  dfree(d.wts);
  dfree(d.nbr);
  dfree(d.e);
  dfree(d.ext_perm);
  dfree(d.ext_pos);
  dfree(d.ext_groups);
  dfree(d.ext_s);
  dfree(d.ext_start);
  dfree(d.ext_step);
  d.compact = false;
  d.n_ext_groups = 0;
  d.ext_lds = 0;
  d.op_bytes = 0;
}

// Apply order of the extension rows and their groups for the LDS-staged
// apply: rows sorted by (stencil base plane, window of EXT_JW stencil base
// columns), band order inside; a run of equal keys is cut into groups of at
// most EXT_ROWS rows. The stencils of a group's rows read, in plane
// bi + a, only columns j0 .. j0 + EXT_JW - 1 + p, whose active nodes are one
// contiguous interval of band indices (band order is sorted by
// L = (i n1 + j) n2 + k).
constexpr int EXT_JW = 8;
constexpr int EXT_ROWS = 512;
constexpr size_t EXT_LDS_MAX = 64 * 1024;  // larger groups use the gathering kernel
struct ExtPlan {
  std::vector<int32_t> perm, pos;
  std::vector<ExtGroup> groups;
  size_t lds = 0;
};

static bool plan_extension(const Band& b, ExtPlan& E) {
  const int P1 = b.p + 1, NL = P1 * P1;
  const int64_t nt = b.total(), n1 = b.n[1], n2 = b.n[2];
  const int64_t nw = (n1 + EXT_JW - 1) / EXT_JW;
  std::vector<int64_t> key(nt);
  for (int64_t r = 0; r < nt; ++r) key[r] = (int64_t)b.base[3 * r] * nw + b.base[3 * r + 1] / EXT_JW;
  E.perm.resize(nt);
  for (int64_t r = 0; r < nt; ++r) E.perm[r] = (int32_t)r;
  std::stable_sort(E.perm.begin(), E.perm.end(), [&](int32_t x, int32_t y) { return key[x] < key[y]; });
  E.pos.assign(nt, 0);
  for (int64_t q = 0; q < nt; ++q) E.pos[E.perm[q]] = (int32_t)q;
  const int64_t* lin = b.lin.data();
  const int64_t na = b.n_act;
  for (int64_t q0 = 0; q0 < nt;) {
    int64_t q1 = q0;
    while (q1 < nt && key[E.perm[q1]] == key[E.perm[q0]]) ++q1;
    const int32_t r0 = E.perm[q0];
    const int64_t bi = b.base[3 * r0];
    const int64_t j0 = b.base[3 * r0 + 1] / EXT_JW * EXT_JW;
    const int64_t j1 = std::min<int64_t>(j0 + EXT_JW - 1 + b.p, n1 - 1);
    ExtGroup g{};
    g.off[0] = 0;
    for (int a = 0; a < P1; ++a) {
      const int64_t i = bi + a;
      const int64_t L0 = (i * n1 + j0) * n2, L1 = (i * n1 + j1 + 1) * n2;
      const int64_t lo = std::lower_bound(lin, lin + na, L0) - lin;
      const int64_t hi = std::lower_bound(lin, lin + na, L1) - lin;
      g.lo[a] = (int32_t)lo;
      g.off[a + 1] = g.off[a] + (int32_t)(hi - lo);
    }
    // every z-line of every row of the run lies inside its plane's interval
    for (int64_t q = q0; q < q1; ++q) {
      const int32_t r = E.perm[q];
      for (int a = 0; a < P1; ++a)
        for (int bb = 0; bb < P1; ++bb) {
          const int32_t s = b.lines[(int64_t)r * NL + a * P1 + bb];
          if (s < g.lo[a] || s + b.p >= g.lo[a] + (g.off[a + 1] - g.off[a])) return false;
        }
    }
    E.lds = std::max(E.lds, (size_t)g.off[P1] * sizeof(double));
    for (int64_t c = q0; c < q1; c += EXT_ROWS) {
      g.row0 = (int32_t)c;
      g.nrows = (int32_t)std::min<int64_t>(EXT_ROWS, q1 - c);
      E.groups.push_back(g);
    }
    q0 = q1;
  }
  return true;
}

int dev_upload_operator(cpm_ctx* ctx, const Band& b) {
  HIPCHK(hipSetDevice(ctx->device));
  int32_t* lines = nullptr;
  double* wts = nullptr;
  int32_t* nbr = nullptr;
  double* e = nullptr;
  int32_t *perm = nullptr, *pos = nullptr;
  ExtGroup* groups = nullptr;
  double* ext_s = nullptr;
  int32_t* ext_start = nullptr;
  uint16_t* ext_step = nullptr;
  auto undo = [&](int code) {
    hipStreamSynchronize(ctx->stream);
    dfree(lines);
    dfree(wts);
    dfree(nbr);
    dfree(e);
    dfree(perm);
    dfree(pos);
    dfree(groups);
    dfree(ext_s);
    dfree(ext_start);
    dfree(ext_step);
    return code;
  };
  int rc;
  ExtPlan E;
  if (!plan_extension(b, E)) {
    ctx->err = "operator upload: an interpolation stencil leaves its group's staged x (internal error)";
    return CPM_EINVAL;
  }
  {  // extension rows in apply order, structure of arrays
    const int P1 = b.p + 1, NL = P1 * P1, NW = 3 * P1;
    const int64_t nt = b.total();
    std::vector<int32_t> lp((size_t)nt * NL);
    std::vector<double> wp((size_t)nt * NW);
    for (int64_t q = 0; q < nt; ++q) {
      const int64_t r = E.perm[q];
      for (int l = 0; l < NL; ++l) lp[l * nt + q] = b.lines[r * NL + l];
      for (int c = 0; c < NW; ++c) wp[c * nt + q] = b.wts[r * NW + c];
    }
    if ((rc = upload(ctx, &lines, lp)) != CPM_OK) return undo(rc);
    if ((rc = upload(ctx, &wts, wp)) != CPM_OK) return undo(rc);
    // the uploads read pageable host memory: finished before the vectors go
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  // compact rows: local stencil coordinates s = t - base, t = (cp - lo) / h
  // (as the host set-up forms them), z-line starts as plane starts and
  // 16-bit increments (band order is sorted by L, so they are positive)
  bool compact = true;
  {
    const int P1 = b.p + 1, NL = P1 * P1;
    const int64_t nt = b.total();
    std::vector<double> sv((size_t)nt * 3);
    std::vector<int32_t> stv((size_t)nt * P1);
    std::vector<uint16_t> dv((size_t)nt * P1 * b.p);
    for (int64_t q = 0; q < nt && compact; ++q) {
      const int64_t r = E.perm[q];
      for (int a = 0; a < 3; ++a) {
        const double t = (b.cp[r * 3 + a] - b.lo[a]) / b.h;
        sv[a * nt + q] = t - (double)b.base[r * 3 + a];
      }
      for (int a = 0; a < P1; ++a) {
        stv[a * nt + q] = b.lines[r * NL + a * P1];
        for (int bb = 1; bb < P1; ++bb) {
          const int64_t inc = (int64_t)b.lines[r * NL + a * P1 + bb] - b.lines[r * NL + a * P1 + bb - 1];
          if (inc < 0 || inc > 65535) compact = false;
          dv[(a * b.p + bb - 1) * nt + q] = (uint16_t)inc;
        }
      }
    }
    if (compact) {
      if ((rc = upload(ctx, &ext_s, sv)) != CPM_OK) return undo(rc);
      if ((rc = upload(ctx, &ext_start, stv)) != CPM_OK) return undo(rc);
      if ((rc = upload(ctx, &ext_step, dv)) != CPM_OK) return undo(rc);
      HIPCHK(hipStreamSynchronize(ctx->stream));
    }
  }
  if ((rc = upload(ctx, &perm, E.perm)) != CPM_OK) return undo(rc);
  if ((rc = upload(ctx, &pos, E.pos)) != CPM_OK) return undo(rc);
  if ((rc = upload(ctx, &groups, E.groups)) != CPM_OK) return undo(rc);
  std::vector<int32_t> soa(b.n_act * 6);
  for (int64_t i = 0; i < b.n_act; ++i)
    for (int q = 0; q < 6; ++q) soa[q * b.n_act + i] = b.nbr[i * 6 + q];
  if ((rc = upload(ctx, &nbr, soa)) != CPM_OK) return undo(rc);
  hipError_t err = hipMalloc((void**)&e, b.total() * sizeof(double));
  if (err == hipSuccess) err = hipStreamSynchronize(ctx->stream);
  if (err != hipSuccess) {
    ctx->err = std::string("operator upload: ") + hipGetErrorString(err);
    return undo(err == hipErrorOutOfMemory ? CPM_ENOMEM : CPM_EDEVICE);
  }
  // everything is on the device: the previous state goes
  dev_free_all(ctx);
  Dev& d = ctx->dev;
  d.lines = lines;
  d.wts = wts;
  d.nbr = nbr;
  d.e = e;
  d.ext_perm = perm;
  d.ext_pos = pos;
  d.ext_groups = groups;
  d.n_ext_groups = (int)E.groups.size();
  d.ext_lds = E.lds;
  d.ext_s = ext_s;
  d.ext_start = ext_start;
  d.ext_step = ext_step;
  d.compact = compact;
  d.op_bytes = b.lines.size() * 4 + b.wts.size() * 8 + soa.size() * 4 + b.total() * 8 +
               2 * E.perm.size() * 4 + E.groups.size() * sizeof(ExtGroup) +
               (compact ? (size_t)b.total() * (3 * 8 + (b.p + 1) * 4 + (b.p + 1) * b.p * 2) : 0);
  return CPM_OK;
}

// e = E x over the whole band (active and ghost rows); nb right-hand sides
// x + q x_stride -> e + q e_stride
static void launch_extend(cpm_ctx* ctx, const double* x, double* e, int nb = 1, int64_t x_stride = 0,
                          int64_t e_stride = 0) {
  const Band& b = ctx->band;
  Dev& d = ctx->dev;
  const int64_t nt = b.total();
  if (d.op_kernel == 1 && d.n_ext_groups > 0 && d.ext_lds <= EXT_LDS_MAX) {
    const dim3 grid(d.n_ext_groups, nb);
    if (b.p == 3)
      launch(ctx, TIMER_EXTEND, k_extend_lds<3>, grid, dim3(256), d.ext_lds, (const ExtGroup*)d.ext_groups, nt,
             (const int32_t*)d.lines, (const double*)d.wts, (const int32_t*)d.ext_perm, x, e, x_stride, e_stride);
    else
      launch(ctx, TIMER_EXTEND, k_extend_lds<2>, grid, dim3(256), d.ext_lds, (const ExtGroup*)d.ext_groups, nt,
             (const int32_t*)d.lines, (const double*)d.wts, (const int32_t*)d.ext_perm, x, e, x_stride, e_stride);
    return;
  }
  const dim3 grid(nblk(nt, 256), nb);
  if (d.op_kernel == 0 && d.compact) {
    if (b.p == 3)
      launch(ctx, TIMER_EXTEND, k_extend_compact<3>, grid, dim3(256), 0, nt, (const double*)d.ext_s,
             (const int32_t*)d.ext_start, (const uint16_t*)d.ext_step, (const int32_t*)d.ext_perm, x, e, x_stride,
             e_stride);
    else
      launch(ctx, TIMER_EXTEND, k_extend_compact<2>, grid, dim3(256), 0, nt, (const double*)d.ext_s,
             (const int32_t*)d.ext_start, (const uint16_t*)d.ext_step, (const int32_t*)d.ext_perm, x, e, x_stride,
             e_stride);
    return;
  }
  if (b.p == 3)
    launch(ctx, TIMER_EXTEND, k_extend<3>, grid, dim3(256), 0, nt, (const int32_t*)d.lines, (const double*)d.wts,
           (const int32_t*)d.ext_perm, x, e, x_stride, e_stride);
  else
    launch(ctx, TIMER_EXTEND, k_extend<2>, grid, dim3(256), 0, nt, (const int32_t*)d.lines, (const double*)d.wts,
           (const int32_t*)d.ext_perm, x, e, x_stride, e_stride);
}

// e = E x, y = A x (or y = f - A x when f != nullptr); e in the context's
// extension scratch unless another buffer of N_T values is given
static void launch_operator(cpm_ctx* ctx, const double* x, double* y, const double* f, double* e = nullptr) {
  const Band& b = ctx->band;
  Dev& d = ctx->dev;
  const double ih2 = 1.0 / (b.h * b.h);
  const double diag = ctx->c + 6.0 * ih2;
  const int64_t na = b.n_act;
  if (!e) e = d.e;
  launch_extend(ctx, x, e);
  launch(ctx, TIMER_STENCIL, k_stencil, dim3(nblk(na, 256)), dim3(256), 0, na, diag, ih2, (const int32_t*)d.nbr, x,
         (const double*)e, f, y);
}

// Tilings of the single-right-hand-side apply: rows per wave, 16-byte chunks
// in flight per row, and apply blocks per resident block slot (in halves;
// with more blocks than slots the later blocks go to the slots that free
// first, which evens out the finish times). Index 0 is the default; every
// tiling gives bit-identical results.
constexpr int N_TILINGS = CPM_PRECOND_TILINGS;
struct Tiling {
  int rpw, unr, over2;
};
constexpr Tiling kTilings[N_TILINGS] = {{2, 2, 4}, {4, 1, 4}, {2, 2, 3}, {4, 1, 6},
                                        {4, 4, 2}, {4, 4, 4}, {8, 2, 4}, {4, 2, 4}};
// a wave's RPW rows must lie in one tile of W (the multi-vector tilings take
// 2, 4 or 8 rows per wave as well)
constexpr bool tilings_fit_tile() {
  for (const Tiling& t : kTilings)
    if (W_TILE % t.rpw != 0) return false;
  return W_TILE % 8 == 0;
}
static_assert(tilings_fit_tile(), "every tiling's rows per wave must divide W_TILE");

template <typename T>
static const void* tiled_fn(int t) {
  switch (t) {
    case 1:
    case 3: return (const void*)k_precond<T, 4, 1>;
    case 4:
    case 5: return (const void*)k_precond<T, 4, 4>;
    case 6: return (const void*)k_precond<T, 8, 2>;
    case 7: return (const void*)k_precond<T, 4, 2>;
    default: return (const void*)k_precond<T, 2, 2>;
  }
}

template <typename T>
static void launch_tiled(cpm_ctx* ctx, int t, size_t lds, const double* v, const double* scale, double* z) {
  Dev& d = ctx->dev;
  const dim3 g(d.n_blocks), b(PRECOND_THREADS);
  const SubDesc* desc = d.desc;
  const int32_t *bs = d.blk_sub, *si = d.sig_idx, *ti = d.tilde_idx;
  const T* W = (const T*)d.W;
  switch (t) {
    case 1:
    case 3: launch(ctx, TIMER_PRECOND, k_precond<T, 4, 1>, g, b, lds, desc, bs, si, ti, W, v, scale, z); break;
    case 4:
    case 5: launch(ctx, TIMER_PRECOND, k_precond<T, 4, 4>, g, b, lds, desc, bs, si, ti, W, v, scale, z); break;
    case 6: launch(ctx, TIMER_PRECOND, k_precond<T, 8, 2>, g, b, lds, desc, bs, si, ti, W, v, scale, z); break;
    case 7: launch(ctx, TIMER_PRECOND, k_precond<T, 4, 2>, g, b, lds, desc, bs, si, ti, W, v, scale, z); break;
    default: launch(ctx, TIMER_PRECOND, k_precond<T, 2, 2>, g, b, lds, desc, bs, si, ti, W, v, scale, z); break;
  }
}

// z = scale * M^{-1} v (scale: device scalar or nullptr for 1)
static void launch_precond(cpm_ctx* ctx, const double* v, double* z, const double* scale = nullptr) {
  Dev& d = ctx->dev;
  if (d.chunk > 0) {
    const size_t lds = (size_t)(d.chunk + PRECOND_RPB_MAX) * sizeof(double);
    if (d.prec == CPM_FP64)
      launch(ctx, TIMER_PRECOND, k_precond_chunked<double>, dim3(d.n_blocks), dim3(PRECOND_THREADS), lds,
             (const SubDesc*)d.desc, (const int32_t*)d.blk_sub, (const int32_t*)d.sig_idx,
             (const int32_t*)d.tilde_idx, (const double*)d.W, v, scale, z, d.chunk);
    else
      launch(ctx, TIMER_PRECOND, k_precond_chunked<float>, dim3(d.n_blocks), dim3(PRECOND_THREADS), lds,
             (const SubDesc*)d.desc, (const int32_t*)d.blk_sub, (const int32_t*)d.sig_idx,
             (const int32_t*)d.tilde_idx, (const float*)d.W, v, scale, z, d.chunk);
    return;
  }
  const size_t lds = (size_t)d.max_m * sizeof(double);
  if (d.prec == CPM_FP64)
    launch_tiled<double>(ctx, d.tiling, lds, v, scale, z);
  else
    launch_tiled<float>(ctx, d.tiling, lds, v, scale, z);
}

int dev_apply_operator(cpm_ctx* ctx, const double* x, double* y) {
  HIPCHK(hipSetDevice(ctx->device));
  launch_operator(ctx, x, y, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return CPM_OK;
}

// Extension scratch of cpm_apply_operator_noalloc: a static device array
// (each device holds its own copy for the life of the process). Host code
// uses only the device address looked up per device, never the array's name.
static __device__ __align__(256) double scratch[NOALLOC_ROWS];
static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_ptr;  // per device

int dev_init_context(cpm_ctx* ctx) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= ctx->device) g_scratch_ptr.resize(ctx->device + 1, nullptr);
  if (!g_scratch_ptr[ctx->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      ctx->err = std::string("device scratch lookup: ") + hipGetErrorString(e);
      return CPM_EDEVICE;
    }
    g_scratch_ptr[ctx->device] = (double*)p;
  }
  ctx->dev.static_e = g_scratch_ptr[ctx->device];
  return CPM_OK;
}

int dev_apply_operator_noalloc(cpm_ctx* ctx, const double* x, double* y) {
  const int64_t nt = ctx->band.total();
  if (nt > NOALLOC_ROWS) {
    ctx->err = "apply_operator_noalloc: the band has " + std::to_string(nt) + " rows, the static scratch holds " +
               std::to_string(NOALLOC_ROWS);
    return CPM_EINVAL;
  }
  if (!ctx->dev.static_e) {
    ctx->err = "apply_operator_noalloc: no device scratch";
    return CPM_EDEVICE;
  }
  HIPCHK(hipSetDevice(ctx->device));
  launch_operator(ctx, x, y, nullptr, ctx->dev.static_e);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return CPM_OK;
}

int dev_apply_precond(cpm_ctx* ctx, const double* v, double* z) {
  HIPCHK(hipSetDevice(ctx->device));
  launch_precond(ctx, v, z);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return CPM_OK;
}

// ---------------------------------------------------------------------------
// Factorisation
// ---------------------------------------------------------------------------
namespace {

struct FactorPlan {
  std::vector<SubDesc> desc;
  // U: [Sigma_j ; B_j] in band order (the apply reads Sigma_j from it); the
  // factorisation's unknowns in elimination order: fU (band index), rcol
  // (right-hand column of a Sigma_j unknown, -1 for B_j), usrt/upos (sorted
  // lookup of fU), bx/bs/ba (B_j data by position); border rows: tilde_pos
  // (position of the unit entry); W maps: wrow (W row -> border row), wcol
  // (W column -> right-hand column, indexed like U).
  std::vector<int32_t> U, fU, rcol, wrow, wcol, usrt, upos, bx, tilde_pos, tilde_idx, blk_sub;
  // per subdomain and panel (columns [k, k + LU_NB)): one past the last A_j
  // row and one past the last border row that can hold a nonzero in the
  // panel (absolute rows), from the structure of A_j
  std::vector<int32_t> pbound;
  std::vector<double> bs, ba;
  int64_t a_elems = 0, w_elems = 0, u_total = 0;
  int max_m = 0, max_n = 0, max_rows = 0, n_blocks = 0;
};

// Apply blocks per subdomain: `slots` blocks apportioned by W bytes (largest
// remainder, at least one each).
std::vector<int> apportion_blocks(const Decomp& D, int slots) {
  const int ns = D.n_sub;
  std::vector<double> bytes(ns);
  double total = 0;
  for (int j = 0; j < ns; ++j) total += bytes[j] = (double)D.subs[j].tilde.size() * D.subs[j].sigma.size();
  std::vector<int> want(ns, 1);
  if (slots <= ns || total <= 0) return want;
  std::vector<std::pair<double, int>> rem;
  int given = 0;
  for (int j = 0; j < ns; ++j) {
    const double share = bytes[j] / total * slots;
    want[j] = std::max(1, (int)std::floor(share));
    given += want[j];
    rem.push_back({share - std::floor(share), j});
  }
  std::sort(rem.begin(), rem.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
    return a.first != b.first ? a.first > b.first : a.second < b.second;
  });
  for (size_t q = 0; given < slots && q < rem.size(); ++q, ++given) want[rem[q].second] += 1;
  return want;
}

// Rows of W_j per apply block for `want` blocks: whole tiles, so that a
// block's waves read whole tiles.
inline int rows_per_block(int t, int want) {
  const int r = std::max(1, (t + want - 1) / want);
  return (r + W_TILE - 1) / W_TILE * W_TILE;
}

void make_plan(const cpm_ctx* ctx, FactorPlan& P, int block_slots, int rpb_max) {
  const Decomp& D = ctx->dec;
  const bool oras = D.kind == CPM_ORAS;
  std::vector<int> want_blocks = apportion_blocks(D, block_slots);
  if (rpb_max > 0)  // chunked apply: at most rpb_max rows per block
    for (int j = 0; j < D.n_sub; ++j)
      want_blocks[j] = std::max(want_blocks[j], (int)((D.subs[j].tilde.size() + rpb_max - 1) / rpb_max));
  int32_t u_off = 0, t_off = 0, blk = 0;
  int64_t a_off = 0, w_off = 0;
  for (int j = 0; j < D.n_sub; ++j) {
    const Sub& s = D.subs[j];
    SubDesc d{};
    d.m = (int32_t)s.sigma.size();
    d.n = d.m + (oras ? (int32_t)s.bnd.size() : 0);
    d.t = (int32_t)s.tilde.size();
    d.u_off = u_off;
    d.t_off = t_off;
    d.ldw = (int32_t)round_up(d.m, 8);
    d.w_off = w_off;
    d.rows = d.n + d.t;
    d.cols = d.n + d.m;
    d.lda = (int32_t)round_up(d.cols, 16);
    d.a_off = a_off;
    d.blk_off = blk;
    d.rpb = rows_per_block(d.t, want_blocks[j]);
    const int nb = (d.t + d.rpb - 1) / d.rpb;
    for (int q = 0; q < nb; ++q) P.blk_sub.push_back(j);
    blk += nb;
    a_off += (int64_t)d.rows * d.lda;
    w_off += w_rows_stored(d.t) * d.ldw;
    // unknowns [Sigma_j ; B_j]; the factorisation takes them in the
    // subdomain's elimination order (identity when none is set)
    std::vector<int32_t> u(s.sigma);
    if (oras) u.insert(u.end(), s.bnd.begin(), s.bnd.end());
    std::vector<int32_t> ord(s.order);
    if ((int)ord.size() != d.n) {
      ord.resize(d.n);
      for (int q = 0; q < d.n; ++q) ord[q] = q;
    }
    std::vector<int32_t> fu(d.n), pos_of(d.n), rc_of(d.m, 0);
    for (int q = 0; q < d.n; ++q) {
      fu[q] = u[ord[q]];
      pos_of[ord[q]] = q;
    }
    std::vector<int32_t> srt(d.n);
    for (int q = 0; q < d.n; ++q) srt[q] = q;
    std::sort(srt.begin(), srt.end(), [&](int32_t x, int32_t y) { return fu[x] < fu[y]; });
    int32_t rank = 0;
    for (int q = 0; q < d.n; ++q) {
      const int32_t li = ord[q];
      const bool isb = li >= d.m;
      P.U.push_back(u[q]);
      P.fU.push_back(fu[q]);
      P.usrt.push_back(fu[srt[q]]);
      P.upos.push_back(srt[q]);
      P.rcol.push_back(isb ? -1 : rank);
      if (!isb) rc_of[li] = rank++;
      P.bx.push_back(isb ? s.xstar[li - d.m] : 0);
      P.bs.push_back(isb ? s.s[li - d.m] : 0.0);
      P.ba.push_back(isb ? s.alpha[li - d.m] : 0.0);
    }
    for (int q = 0; q < d.n; ++q) P.wcol.push_back(q < d.m ? rc_of[q] : 0);
    // border rows: Sigma~_j (a subset of Sigma_j, both in band order) by position
    std::vector<std::pair<int32_t, int32_t>> brow;
    size_t p = 0;
    for (size_t q = 0; q < s.tilde.size(); ++q) {
      while (s.sigma[p] != s.tilde[q]) ++p;
      brow.push_back({pos_of[p], (int32_t)q});
      P.tilde_idx.push_back(s.tilde[q]);
    }
    std::sort(brow.begin(), brow.end());
    std::vector<int32_t> wrow(brow.size());
    for (size_t i = 0; i < brow.size(); ++i) {
      P.tilde_pos.push_back(brow[i].first);
      wrow[brow[i].second] = (int32_t)i;
    }
    P.wrow.insert(P.wrow.end(), wrow.begin(), wrow.end());
    // panel row bounds: A_j rows below reach[c], border rows whose unit entry
    // lies in a column <= c, c the panel's last column
    d.pb_off = (int32_t)(P.pbound.size() / 2);
    const bool have = (int)s.reach.size() == d.n && (int)s.order.size() == d.n;
    int32_t nb_rows = 0;
    for (int k = 0; k < d.n; k += LU_NB) {
      const int c = std::min(k + LU_NB, d.n) - 1;
      while (nb_rows < d.t && brow[nb_rows].first <= c) ++nb_rows;
      P.pbound.push_back(have ? std::max(s.reach[c], (int32_t)(c + 1)) : d.n);
      P.pbound.push_back(d.n + (have ? nb_rows : d.t));
    }
    u_off += d.n;
    t_off += d.t;
    P.max_m = std::max(P.max_m, (int)d.ldw);
    P.max_n = std::max(P.max_n, (int)d.n);
    P.max_rows = std::max(P.max_rows, (int)d.rows);
    P.desc.push_back(d);
  }
  P.a_elems = a_off;
  P.w_elems = w_off;
  P.u_total = u_off;
  P.n_blocks = blk;
}

// Factor workspace of one subdomain (bordered matrix, panel scratch in 64-row
// tiles, I - L11^{-1} of an outer block), elements.
inline int64_t factor_ws_elems(const SubDesc& d) {
  return (int64_t)d.rows * d.lda + (int64_t)LU_NB * round_up(d.rows, 64) + (int64_t)LU_KMAX * LU_KMAX;
}

// Consecutive groups of subdomains whose factor workspaces fit in `limit` bytes
// together (a subdomain larger than the limit forms a group of its own).
std::vector<std::pair<int, int>> factor_groups(const std::vector<SubDesc>& desc, size_t esz, size_t limit) {
  std::vector<std::pair<int, int>> g;
  int g0 = 0;
  size_t acc = 0;
  for (int j = 0; j < (int)desc.size(); ++j) {
    const size_t wj = (size_t)factor_ws_elems(desc[j]) * esz;
    if (j > g0 && acc + wj > limit) {
      g.push_back({g0, j});
      g0 = j;
      acc = 0;
    }
    acc += wj;
  }
  if (!desc.empty()) g.push_back({g0, (int)desc.size()});
  return g;
}

template <typename T>
int run_factor(cpm_ctx* ctx, const FactorPlan& P, int prec, int tile_r) {
  const Band& b = ctx->band;
  const Decomp& D = ctx->dec;
  Dev& dv = ctx->dev;
  const int ns = D.n_sub;
  const double ih2 = 1.0 / (b.h * b.h);
  const double diag = ctx->c + 6.0 * ih2;

  SubDesc *ddesc = nullptr, *gdesc = nullptr;
  int32_t *dU = nullptr, *dsrt = nullptr, *dpos = nullptr, *dbx = nullptr, *dtpos = nullptr, *dtidx = nullptr,
          *dblk = nullptr, *dipiv = nullptr, *dinfo = nullptr, *dpre = nullptr, *dfu = nullptr, *drc = nullptr,
          *dwrow = nullptr, *dwcol = nullptr, *drowhi = nullptr, *dntile = nullptr, *dpb = nullptr;
  int2* dlist = nullptr;
  unsigned long long* dflops = nullptr;
  double *dbs = nullptr, *dba = nullptr;
  LuJob* jobs_buf = nullptr;
  int64_t* dscr_off = nullptr;
  T* dscr = nullptr;
  T* dA = nullptr;
  T* dW = nullptr;
  T* dlm = nullptr;  // per subdomain of a group: I - L11^{-1} of the current outer block
  int rc = CPM_OK;
  auto free_group = [&]() {
    hipStreamSynchronize(ctx->stream);
    dfree(gdesc); pool_free(dA); dfree(dscr); dfree(dscr_off); dfree(jobs_buf); dfree(dpre); dfree(dlm);
    dfree(drowhi); dfree(dlist);
  };
  auto cleanup = [&]() {
    free_group();
    dfree(dsrt); dfree(dpos); dfree(dbx); dfree(dtpos); dfree(dipiv); dfree(dinfo);
    dfree(dbs); dfree(dba); dfree(dfu); dfree(drc); dfree(dwrow); dfree(dwcol); dfree(dntile); dfree(dflops); dfree(dpb);
  };
  auto bail = [&](int code) {
    cleanup();
    dfree(ddesc); dfree(dU); dfree(dtidx); dfree(dblk); pool_free(dW);
    return code;
  };
#define FCHK(expr)                                                      \
  do {                                                                  \
    int r_ = (expr);                                                    \
    if (r_ != CPM_OK) return bail(r_);                                  \
  } while (0)
#define FHIP(expr)                                                      \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess) {                                             \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);     \
      return bail(e_ == hipErrorOutOfMemory ? CPM_ENOMEM : CPM_EDEVICE); \
    }                                                                   \
  } while (0)

  FCHK(upload(ctx, &ddesc, P.desc));
  FCHK(upload(ctx, &dU, P.U));
  FCHK(upload(ctx, &dsrt, P.usrt));
  FCHK(upload(ctx, &dpos, P.upos));
  FCHK(upload(ctx, &dbx, P.bx));
  FCHK(upload(ctx, &dbs, P.bs));
  FCHK(upload(ctx, &dba, P.ba));
  FCHK(upload(ctx, &dtpos, P.tilde_pos));
  FCHK(upload(ctx, &dtidx, P.tilde_idx));
  FCHK(upload(ctx, &dblk, P.blk_sub));
  FCHK(upload(ctx, &dfu, P.fU));
  FCHK(upload(ctx, &drc, P.rcol));
  FCHK(upload(ctx, &dwrow, P.wrow));
  FCHK(upload(ctx, &dwcol, P.wcol));
  FCHK(upload(ctx, &dpb, P.pbound));
  FHIP(hipMalloc((void**)&dntile, sizeof(int32_t)));
  FHIP(hipMalloc((void**)&dflops, sizeof(unsigned long long)));
  FHIP(hipMemsetAsync(dflops, 0, sizeof(unsigned long long), ctx->stream));
  FHIP(hipMalloc((void**)&dipiv, P.u_total * sizeof(int32_t)));
  FHIP(hipMalloc((void**)&dinfo, ns * sizeof(int32_t)));
  FHIP(hipMemsetAsync(dinfo, 0, ns * sizeof(int32_t), ctx->stream));
  FHIP(pool_malloc((void**)&dW, P.w_elems * sizeof(T)));

  // Subdomains are factored group by group so that the bordered matrices of a
  // group fit in the workspace limit; every subdomain's arithmetic is the same
  // whatever group it is in. Within a group the arrays are addressed through
  // rebased descriptors (a_off, u_off, t_off relative to the group; w_off
  // global, into the resident W arena).
  const std::vector<std::pair<int, int>> groups = factor_groups(P.desc, sizeof(T), dv.ws_limit);
  // the panel's dynamic LDS (register + LDS rows of its fast form) exceeds the default limit
  FHIP(hipFuncSetAttribute((const void*)k_lu_panel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                           (int)panel_lds_bytes<T>()));
  FHIP(hipFuncSetAttribute((const void*)k_lu_panel_fast<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                           (int)panel_lds_bytes<T>()));
  // resident blocks of the listed trailing update
  int trail_grid = 0;
  {
    int n_cu = 0, per_cu = 0;
    FHIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
    if (tile_r == GEMM_TILE_R)
      FHIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_lu_gemm_list<T, GEMM_TILE_R, GEMM_TILE>, 256, 0));
    else
      FHIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_lu_gemm_list<T, GEMM_TILE, GEMM_TILE>, 256, 0));
    trail_grid = std::max(8, n_cu * std::max(1, per_cu) / 8 * 8);  // a multiple of 8 (one share per XCD)
  }
  for (const auto& gr : groups) {
    const int g0 = gr.first, gn = gr.second - gr.first;
    std::vector<SubDesc> gd(P.desc.begin() + g0, P.desc.begin() + gr.second);
    const int64_t a0 = gd[0].a_off;
    const int32_t u0 = gd[0].u_off, t0 = gd[0].t_off, pb0 = gd[0].pb_off;
    int64_t a_elems = 0;
    int max_n = 0, max_rows = 0, tmax = 0;
    for (SubDesc& d : gd) {
      d.a_off -= a0;
      d.u_off -= u0;
      d.t_off -= t0;
      d.pb_off -= pb0;
      a_elems = std::max(a_elems, d.a_off + (int64_t)d.rows * d.lda);
      max_n = std::max(max_n, (int)d.n);
      max_rows = std::max(max_rows, (int)d.rows);
      tmax = std::max(tmax, (int)d.t);
    }
    int32_t* gU = dfu + u0;
    int32_t* grc = drc + u0;
    int32_t* gsrt = dsrt + u0;
    int32_t* gpos = dpos + u0;
    int32_t* gbx = dbx + u0;
    double* gbs = dbs + u0;
    double* gba = dba + u0;
    int32_t* gtpos = dtpos + t0;
    int32_t* gipiv = dipiv + u0;
    int32_t* ginfo = dinfo + g0;
    FCHK(upload(ctx, &gdesc, gd));
    FHIP(pool_malloc((void**)&dA, a_elems * sizeof(T)));
    FHIP(hipMemsetAsync(dA, 0, a_elems * sizeof(T), ctx->stream));

    // Assembly of the augmented local matrices.
    {
      dim3 grid(nblk(max_rows, 256), gn);
      if (b.p == 3)
        k_assemble<T, 3><<<grid, 256, 0, ctx->stream>>>(gdesc, b.n_act, b.total(), dv.lines, dv.wts, dv.nbr, gU, gsrt, gpos,
                                                        gbx, gbs, gba, gtpos, grc, dv.ext_pos, diag, ih2,
                                                        D.kind == CPM_ORAS, dA);
      else
        k_assemble<T, 2><<<grid, 256, 0, ctx->stream>>>(gdesc, b.n_act, b.total(), dv.lines, dv.wts, dv.nbr, gU, gsrt, gpos,
                                                        gbx, gbs, gba, gtpos, grc, dv.ext_pos, diag, ih2,
                                                        D.kind == CPM_ORAS, dA);
      FHIP(hipGetLastError());
    }

    // Two-level blocked LU. Outer blocks of LU_KMAX columns; inside one, each
    // LU_NB-wide panel is first brought up to date left-looking (row
    // interchanges + unit-lower solve + MFMA update from the block's earlier
    // panels), then factored; its interchanges are applied to the block's
    // earlier L columns. After the outer block, the trailing matrix gets the
    // block's interchanges, the unit-lower solve with the LU_KMAX x LU_KMAX L11
    // and one MFMA update with K = LU_KMAX.
    enum { L_PANEL = 0, L_SWAP_TRSM = 1, L_SWAP = 2, L_GEMM = 3, L_GEMM_TRAIL = 4, L_LINV = 5, L_GEMM_U = 6, L_BORDER = 7,
           L_PANEL_FAST = 8 };
    struct Launch {
      int kind, k, job_off, n_jobs, units;
    };
    std::vector<LuJob> jobs;
    std::vector<int32_t> prefix;  // per launch: n_jobs entries (job_off-aligned)
    std::vector<Launch> lplan;
    auto add = [&](int kind, int k, const std::vector<std::pair<LuJob, int>>& list) {
      Launch L{kind, k, (int)jobs.size(), 0, 0};
      for (const auto& e : list) {
        if (e.second <= 0) continue;
        jobs.push_back(e.first);
        prefix.push_back(L.units);
        L.units += e.second;
        L.n_jobs++;
      }
      if (L.n_jobs > 0) lplan.push_back(L);
    };
    auto cdiv = [](int a, int b) { return (a + b - 1) / b; };
    for (int K0 = 0; K0 < max_n; K0 += LU_KMAX) {
      for (int p = 0; p < LU_KMAX / LU_NB; ++p) {
        const int k = K0 + p * LU_NB;
        if (k >= max_n) break;
        if (p > 0) {
          std::vector<std::pair<LuJob, int>> ts, gm;
          for (int j = 0; j < gn; ++j) {
            const SubDesc& d = gd[j];
            if (k >= d.n) continue;
            const int kb = std::min(LU_NB, d.n - k);
            const LuJob jb{j, K0, k - K0, k, k, k + kb};
            ts.push_back({jb, 1});
            gm.push_back({jb, cdiv(d.rows - k, GEMM_TILE)});
          }
          add(L_SWAP_TRSM, k, ts);
          add(L_GEMM, k, gm);
        }
        {  // the register + LDS form when every panel of the launch is full width and fits
          bool fast = true;
          for (int j = 0; j < gn && fast; ++j) {
            const SubDesc& d = gd[j];
            if (k >= d.n) continue;
            const int ga = std::min(P.pbound[2 * ((size_t)d.pb_off + pb0 + k / LU_NB)] - k, d.n - k);
            fast = d.n - k >= LU_NB && ga <= PANEL_FAST_RR * PANEL_FAST_THREADS + PanelLds<T>::ROWS;
          }
          lplan.push_back(Launch{fast ? L_PANEL_FAST : L_PANEL, k, 0, 0, gn});
        }
        {  // border rows that may be nonzero in this panel: 256 per block
          int nbl = 0;
          for (int j = 0; j < gn; ++j) {
            const SubDesc& d = gd[j];
            if (k >= d.n) continue;
            const int n_b = P.pbound[2 * ((size_t)d.pb_off + pb0 + k / LU_NB) + 1] - d.n;
            nbl = std::max(nbl, cdiv(n_b, 256));
          }
          if (nbl > 0) lplan.push_back(Launch{L_BORDER, k, 0, 0, nbl});
        }
        if (p > 0) {
          std::vector<std::pair<LuJob, int>> sw;
          for (int j = 0; j < gn; ++j) {
            const SubDesc& d = gd[j];
            if (k >= d.n) continue;
            sw.push_back({LuJob{j, k, std::min(LU_NB, d.n - k), 0, K0, k}, cdiv(k - K0, TRSM_COLS)});
          }
          add(L_SWAP, k, sw);
        }
      }
      // trailing: interchanges, U12 = L11^{-1} U12 (as Lm = I - L11^{-1}, then
      // U12 -= Lm U12 on matrix cores), then A22 -= L21 U12
      std::vector<std::pair<LuJob, int>> sw, li, gu, gm;
      for (int j = 0; j < gn; ++j) {
        const SubDesc& d = gd[j];
        if (K0 >= d.n) continue;
        const int K1 = std::min(K0 + LU_KMAX, d.n);
        const LuJob jb{j, K0, K1 - K0, K1, K1, d.cols};
        sw.push_back({jb, cdiv(d.cols - K1, TRSM_COLS)});
        li.push_back({LuJob{j, K0, K1 - K0, 0, 0, LU_KMAX}, LU_KMAX / TRSM_COLS});
        gu.push_back({LuJob{j, K0, K1 - K0, K0, K1, d.cols}, cdiv(d.cols - K1, GEMM_TILE)});
        gm.push_back({jb, cdiv(d.rows - K1, tile_r) * cdiv(d.cols - K1, GEMM_TILE)});
      }
      add(L_SWAP, K0, sw);
      add(L_LINV, K0, li);
      add(L_GEMM_U, K0, gu);
      add(L_GEMM_TRAIL, K0, gm);
    }
    FCHK(upload(ctx, &jobs_buf, jobs));
    FCHK(upload(ctx, &dpre, prefix));
    // panel scratch, LU_NB x rows_j (rounded to 64-row tiles) per subdomain
    std::vector<int64_t> scr_off(gn);
    int64_t scr_total = 0;
    for (int j = 0; j < gn; ++j) {
      scr_off[j] = scr_total;
      scr_total += (int64_t)LU_NB * round_up(gd[j].rows, 64);
    }
    FCHK(upload(ctx, &dscr_off, scr_off));
    FHIP(hipMalloc((void**)&dscr, scr_total * sizeof(T)));
    FHIP(hipMalloc((void**)&dlm, (size_t)gn * LU_KMAX * LU_KMAX * sizeof(T)));
    FHIP(hipMalloc((void**)&drowhi, (size_t)gn * 2 * sizeof(int32_t)));
    int list_cap = 1;
    for (const Launch& L : lplan)
      if (L.kind == L_GEMM_TRAIL) list_cap = std::max(list_cap, L.units);
    FHIP(hipMalloc((void**)&dlist, (size_t)list_cap * sizeof(int2)));
    const LuJob* ujobs = nullptr;  // the jobs of the last U12 launch
    for (const Launch& L : lplan) {
      const LuJob* jb = jobs_buf + L.job_off;
      const int32_t* pre = dpre + L.job_off;
      switch (L.kind) {
        case L_PANEL:
          k_lu_panel<T><<<gn, PANEL_THREADS, panel_lds_bytes<T>(), ctx->stream>>>(
              gdesc, dA, L.k, gipiv, ginfo, dscr, dscr_off, dpb + 2 * (int64_t)pb0, drowhi);
          break;
        case L_PANEL_FAST:
          k_lu_panel_fast<T><<<gn, PANEL_FAST_THREADS, panel_lds_bytes<T>(), ctx->stream>>>(
              gdesc, dA, L.k, gipiv, ginfo, dpb + 2 * (int64_t)pb0, drowhi);
          break;
        case L_BORDER:
          k_lu_border<T><<<dim3(L.units, gn), 256, 0, ctx->stream>>>(gdesc, dA, L.k, dpb + 2 * (int64_t)pb0);
          break;
        case L_SWAP_TRSM:
          k_lu_swap_trsm<T, true><<<L.units, TRSM_COLS, 0, ctx->stream>>>(gdesc, dA, gipiv, jb, pre, L.n_jobs);
          break;
        case L_SWAP:
          k_lu_swap_trsm<T, false><<<L.units, TRSM_COLS, 0, ctx->stream>>>(gdesc, dA, gipiv, jb, pre, L.n_jobs);
          break;
        case L_LINV:
          k_lu_linv<T><<<L.units, TRSM_COLS, 0, ctx->stream>>>(gdesc, dA, jb, pre, L.n_jobs, dlm, dntile);
          break;
        case L_GEMM_U:  // not in the LU-update timer, which covers the Schur-complement updates
          k_lu_gemm_u<T><<<L.units, 256, 0, ctx->stream>>>(gdesc, dA, jb, pre, L.n_jobs, dlm, drowhi, tile_r, dlist,
                                                           dntile, dflops);
          ujobs = jb;
          break;
        case L_GEMM_TRAIL:  // the tiles k_lu_gemm_u listed, on a grid of resident blocks
          if (tile_r == GEMM_TILE_R)
            launch(ctx, TIMER_LU_GEMM, k_lu_gemm_list<T, GEMM_TILE_R, GEMM_TILE>, dim3(trail_grid), dim3(256), 0,
                   (const SubDesc*)gdesc, dA, ujobs, (const int2*)dlist, (const int32_t*)dntile);
          else
            launch(ctx, TIMER_LU_GEMM, k_lu_gemm_list<T, GEMM_TILE, GEMM_TILE>, dim3(trail_grid), dim3(256), 0,
                   (const SubDesc*)gdesc, dA, ujobs, (const int2*)dlist, (const int32_t*)dntile);
          break;
        case L_GEMM:
          launch(ctx, TIMER_LU_GEMM, k_lu_gemm<T>, dim3(L.units), dim3(256), 0, (const SubDesc*)gdesc, dA, jb, pre,
                 L.n_jobs, (const int32_t*)drowhi, dflops);
          break;
      }
    }
    FHIP(hipGetLastError());
    {
      dim3 grid(tmax, gn);
      k_extract_w<T><<<grid, 256, 0, ctx->stream>>>(gdesc, dA, dwrow + t0, dwcol + u0, dW);
      FHIP(hipGetLastError());
    }
    free_group();
  }
  std::vector<int32_t> info(ns);
  unsigned long long flops = 0;
  FHIP(hipMemcpyAsync(info.data(), dinfo, ns * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
  FHIP(hipMemcpyAsync(&flops, dflops, sizeof(flops), hipMemcpyDeviceToHost, ctx->stream));
  FHIP(hipStreamSynchronize(ctx->stream));
  dv.factor_flops = (double)flops;
  for (int j = 0; j < ns; ++j)
    if (info[j] != 0) {
      ctx->err = "factor: zero pivot in subdomain " + std::to_string(j) + " at column " + std::to_string(info[j] - 1);
      return bail(CPM_ESINGULAR);
    }
  cleanup();
  dv.desc = ddesc;
  dv.hdesc = P.desc;
  dv.factor_tile_used = tile_r;
  dv.tiling = 0;
  dv.multi_tiling = prec == CPM_FP64 ? 5 : 1;  // the measured best at the benchmark size (planned by dev_factor)
  dv.sig_idx = dU;
  dv.tilde_idx = dtidx;
  dv.blk_sub = dblk;
  dv.W = dW;
  dv.prec = prec;
  dv.n_blocks = P.n_blocks;
  dv.max_m = P.max_m;
  dv.n_groups = (int)groups.size();
  dv.w_bytes = P.w_elems * sizeof(T) + P.desc.size() * sizeof(SubDesc) + (P.U.size() + P.tilde_idx.size() +
               P.blk_sub.size()) * sizeof(int32_t);
  return rc;
#undef FCHK
#undef FHIP
}

}  // namespace

int plan_multi(cpm_ctx* ctx);

int dev_factor(cpm_ctx* ctx, int prec) {
  HIPCHK(hipSetDevice(ctx->device));
  dev_free_factor(ctx);
  // Apply blocks resident at once (registers and the LDS copy of v|Sigma_j
  // decide how many fit on a CU); the W bytes are spread evenly over them.
  int n_cu = 0;
  HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  int64_t max_m = 0;
  for (const Sub& s : ctx->dec.subs) max_m = std::max<int64_t>(max_m, round_up(s.sigma.size(), 8));
  // v|Sigma_j is staged whole in LDS when it fits, else in chunks (or when a
  // chunk width is requested).
  Dev& dv = ctx->dev;
  dv.chunk = 0;
  size_t lds = (size_t)max_m * sizeof(double);
  if (dv.chunk_req > 0 || lds > 160 * 1024) {
    dv.chunk = dv.chunk_req > 0 ? dv.chunk_req : PRECOND_CHUNK;
    lds = (size_t)(dv.chunk + PRECOND_RPB_MAX) * sizeof(double);
  }
  int per_cu = 0;
  if (dv.chunk > 0) {
    if (lds > 64 * 1024) {
      hipFuncSetAttribute((const void*)k_precond_chunked<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipFuncSetAttribute((const void*)k_precond_chunked<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    }
    if (prec == CPM_FP64)
      HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_precond_chunked<double>, PRECOND_THREADS, lds));
    else
      HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_precond_chunked<float>, PRECOND_THREADS, lds));
  } else {  // the default tiling's kernel
    const void* fn = prec == CPM_FP64 ? tiled_fn<double>(0) : tiled_fn<float>(0);
    if (lds > 64 * 1024) hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, PRECOND_THREADS, lds));
  }
  per_cu = std::max(1, per_cu);
  FactorPlan P;
  make_plan(ctx, P, dv.chunk > 0 ? n_cu * per_cu : n_cu * per_cu * kTilings[0].over2 / 2,
            dv.chunk > 0 ? PRECOND_RPB_MAX : 0);
  const int tile_r = dv.factor_tile ? dv.factor_tile : tuned_factor_tile(ctx, prec);
  int rc = prec == CPM_FP64 ? run_factor<double>(ctx, P, prec, tile_r) : run_factor<float>(ctx, P, prec, tile_r);
  if (rc == CPM_OK) rc = plan_multi(ctx);
  return rc;
}

// Rows of the trailing-update tile chosen by cpm_autotune_factor, per device
// architecture and precision, for the life of the process (128 until tuned).
static std::mutex g_tile_mu;
static std::map<std::pair<std::string, int>, int> g_tile_cache;

static std::string arch_name(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  return prop.gcnArchName;
}

int tuned_factor_tile(cpm_ctx* ctx, int prec) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  const auto it = g_tile_cache.find({arch_name(ctx->device), prec});
  return it == g_tile_cache.end() ? GEMM_TILE_R : it->second;
}

// Factor with each trailing-update tile (64 x 64, 128 x 64), time the
// matrix-core update launches (HIP events; the caller's kernel timers are
// left as they were), cache the faster for this architecture and precision,
// and leave the factors of the faster in place. Both tiles form every
// element's sum in the same order, so the factors are identical.
int dev_autotune_factor(cpm_ctx* ctx, int prec, int* best, double* ms) {
  Dev& dv = ctx->dev;
  Timer& tm = ctx->timer;
  timer_harvest(ctx);
  const bool was_on = tm.on;
  double ms0[N_TIMERS];
  int64_t n0[N_TIMERS];
  for (int q = 0; q < N_TIMERS; ++q) {
    ms0[q] = tm.ms[q];
    n0[q] = tm.count[q];
  }
  const int saved = dv.factor_tile;
  const int tiles[2] = {GEMM_TILE, GEMM_TILE_R};
  double t[2] = {0, 0};
  int rc = CPM_OK;
  for (int q = 0; q < 2 && rc == CPM_OK; ++q) {
    dv.factor_tile = tiles[q];
    tm.on = true;
    const double m0 = tm.ms[TIMER_LU_GEMM];
    rc = dev_factor(ctx, prec);
    timer_harvest(ctx);
    t[q] = tm.ms[TIMER_LU_GEMM] - m0;
  }
  tm.on = was_on;
  for (int q = 0; q < N_TIMERS; ++q) {
    tm.ms[q] = ms0[q];
    tm.count[q] = n0[q];
  }
  if (rc == CPM_OK) {
    const int arg = t[0] < t[1] ? 0 : 1;
    {
      std::lock_guard<std::mutex> lk(g_tile_mu);
      g_tile_cache[{arch_name(ctx->device), prec}] = tiles[arg];
    }
    if (best) *best = tiles[arg];
    if (ms) {
      ms[0] = t[0];
      ms[1] = t[1];
    }
    dv.factor_tile = saved;
    if (arg == 0) {  // the last factorisation used the other tile
      dv.factor_tile = tiles[0];
      rc = dev_factor(ctx, prec);
      dv.factor_tile = saved;
    }
  }
  dv.factor_tile = saved;
  return rc;
}

int dev_export_w(cpm_ctx* ctx, int j, double* w) {
  HIPCHK(hipSetDevice(ctx->device));
  Dev& dv = ctx->dev;
  SubDesc d;
  HIPCHK(hipMemcpy(&d, dv.desc + j, sizeof(SubDesc), hipMemcpyDeviceToHost));
  const size_t esz = dv.prec == CPM_FP64 ? 8 : 4;
  const int cw = esz == 8 ? W_CW<double> : W_CW<float>;
  std::vector<char> buf((size_t)w_rows_stored(d.t) * d.ldw * esz);
  HIPCHK(hipMemcpy(buf.data(), (char*)dv.W + d.w_off * esz, buf.size(), hipMemcpyDeviceToHost));
  for (int q = 0; q < d.t; ++q)
    for (int c = 0; c < d.m; ++c) {
      const size_t at = (size_t)w_tile_index(d.ldw, cw, q, c);
      w[(size_t)q * d.m + c] = esz == 8 ? ((const double*)buf.data())[at] : (double)((const float*)buf.data())[at];
    }
  return CPM_OK;
}

// ---------------------------------------------------------------------------
// FGMRES(m), right preconditioned, CGS2 Arnoldi, x0 = 0.
// ---------------------------------------------------------------------------
static size_t krylov_bytes(int64_t na, int m) {
  const SmallLayout L{m};
  return ((size_t)(2 * m + 2) * round_up(na, 64) + RED_MAX_BLOCKS * PART_LD + L.size()) * sizeof(double);
}

static int ensure_krylov(cpm_ctx* ctx, int m) {
  Dev& d = ctx->dev;
  if (d.restart == m && d.V) return CPM_OK;
  free_krylov(ctx);
  const int64_t na = ctx->band.n_act;
  d.ld = round_up(na, 64);
  SmallLayout L{m};
  HIPCHK(hipMalloc((void**)&d.V, (size_t)(m + 1) * d.ld * sizeof(double)));
  HIPCHK(hipMalloc((void**)&d.Z, (size_t)m * d.ld * sizeof(double)));
  HIPCHK(hipMalloc((void**)&d.F, (size_t)d.ld * sizeof(double)));
  HIPCHK(hipMalloc((void**)&d.part, (size_t)RED_MAX_BLOCKS * PART_LD * sizeof(double)));
  HIPCHK(hipMalloc((void**)&d.small, (size_t)L.size() * sizeof(double)));
  HIPCHK(hipHostMalloc((void**)&d.slots, (size_t)(m + 2) * sizeof(HostSlot),
                       hipHostMallocMapped | hipHostMallocCoherent));
  std::memset((void*)d.slots, 0, (size_t)(m + 2) * sizeof(HostSlot));
  HIPCHK(hipHostGetDevicePointer((void**)&d.slots_dev, d.slots, 0));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  d.restart = m;
  d.krylov_bytes = krylov_bytes(na, m);
  return CPM_OK;
}

int dev_solve(cpm_ctx* ctx, const double* f, double* u, double tol, int max_iter, int m, cpm_solve_info* info) {
  HIPCHK(hipSetDevice(ctx->device));
  int rc = ensure_krylov(ctx, m);
  if (rc != CPM_OK) return rc;
  Dev& d = ctx->dev;
  const int64_t na = ctx->band.n_act;
  const SmallLayout L{m};
  double* sm = d.small;
  double* scal = sm + L.scal();
  hipStream_t st = ctx->stream;
  const unsigned gv = nblk(na, 256);
  const double ih2 = 1.0 / (ctx->band.h * ctx->band.h);
  const double diag = ctx->c + 6.0 * ih2;
  PhaseClock clock;
  clock.start(ctx);
  hipEvent_t t0, t1;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  HIPCHK(hipEventRecord(t0, st));

  // k_arnoldi / k_norm_finish write the scalars of a step into mapped pinned
  // memory and then the step's ticket; the host polls for it (and checks the
  // stream for errors while it waits).
  HostSlot* slots = d.slots;
  HostSlot* slots_dev = d.slots_dev;
  std::vector<unsigned long long> expect(m + 2, 0);
  auto ticket_for = [&](int slot) -> unsigned long long {
    expect[slot] = ++d.ticket;
    return expect[slot];
  };
  auto wait = [&](int slot, const double** out) -> int {
    volatile unsigned long long* tk = &slots[slot].ticket;
    for (long spin = 0;; ++spin) {
      if (*tk == expect[slot]) break;
      if ((spin & 1023) == 1023) {
        const hipError_t q = hipStreamQuery(st);
        if (q != hipSuccess && q != hipErrorNotReady) {
          ctx->err = std::string("solve: device error ") + hipGetErrorString(q);
          return CPM_EDEVICE;
        }
        if (q == hipSuccess && *tk != expect[slot]) {
          ctx->err = "solve: stream idle but the step's result never arrived";
          return CPM_EDEVICE;
        }
      }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    *out = (const double*)slots[slot].v;
    return CPM_OK;
  };
  auto finish = [&](int code, int iters, int cycles, double rel_true, double rel_est) -> int {
    hipEventRecord(t1, st);
    hipEventSynchronize(t1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, t0, t1);
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    if (info) {
      info->iters = iters;
      info->cycles = cycles;
      info->status = code;
      info->relres_true = rel_true;
      info->relres_est = rel_est;
      info->ms = ms;
      clock.stop(ctx, info->phase_ms);
    }
    return code;
  };

  // ||f||, with V[0] = f (x0 = 0) as the first residual
  launch(ctx, TIMER_UPDATE, k_copy, dim3(gv), dim3(256), 0, na, f, d.V);
  launch(ctx, TIMER_UPDATE, k_fill, dim3(gv), dim3(256), 0, na, u, 0.0);
  const int rb = red_blocks(na);
  launch(ctx, TIMER_KRYLOV, k_dots, dim3(rb), dim3(RED_THREADS), 0, na, d.V, 0, 1, d.V, d.part, -1, nullptr);
  launch(ctx, TIMER_KRYLOV, k_norm_finish, dim3(1), dim3(RED_THREADS), 0, d.part, rb, L, sm, slots_dev + (m + 1), ticket_for(m + 1));
  const double* hv = nullptr;
  if ((rc = wait(m + 1, &hv)) != CPM_OK) return rc;
  const double bnorm = hv[S_BETA];
  if (!std::isfinite(bnorm)) {
    finish(CPM_EINVAL, 0, 0, NAN, NAN);
    ctx->err = "solve: right-hand side is not finite";
    return CPM_EINVAL;
  }
  if (bnorm == 0.0) return finish(CPM_OK, 0, 0, 0.0, 0.0);

  int iters = 0, cycles = 0;
  double rel_true = 1.0, rel_est = 1.0;
  int status = CPM_ENOTCONV;
  auto kernels_of_iteration = [&](int k, unsigned long long ticket) {
    double* vk = d.V + (size_t)k * d.ld;
    double* w = d.V + (size_t)(k + 1) * d.ld;
    double* zk = d.Z + (size_t)k * d.ld;
    launch_precond(ctx, vk, zk, scal + S_INV);  // z_k = M^{-1} (V[k] / ||V[k]||)
    launch_extend(ctx, zk, d.e);                // e = E z_k
    // w = A z_k fused with CGS pass 1 (normalising V[k] in place), then pass 2,
    // ||w|| and the Givens update
    const BatchStrides one{};
    launch(ctx, TIMER_STENCIL, k_stencil_dots, dim3(rb), dim3(RED_THREADS), 0, na, diag, ih2, d.nbr, zk, d.e, w, d.V, d.ld, k + 1, d.part, k,
                                               scal + S_INV, one);
    launch(ctx, TIMER_KRYLOV, k_reduce_cols, dim3(k + 1), dim3(RED_THREADS), 0, d.part, rb, sm + L.h1(), one);
    launch(ctx, TIMER_KRYLOV, k_axpy_dots, dim3(rb), dim3(RED_THREADS), 0, na, d.V, d.ld, k, sm + L.h1(), w, d.part, 0, one);
    launch(ctx, TIMER_KRYLOV, k_reduce_cols, dim3(k + 1), dim3(RED_THREADS), 0, d.part, rb, sm + L.h2(), one);
    launch(ctx, TIMER_KRYLOV, k_axpy_dots, dim3(rb), dim3(RED_THREADS), 0, na, d.V, d.ld, k, sm + L.h2(), w, d.part, 1, one);
    launch(ctx, TIMER_KRYLOV, k_arnoldi, dim3(1), dim3(RED_THREADS), 0, d.part, rb, k, L, sm, slots_dev + k, ticket, one);
  };
  // With graphs, iteration k is captured once (ticket 1 baked in) and replayed;
  // the host clears slot k's ticket before each replay, which is safe because
  // the slot's previous write finished before the host's last wait in this
  // stream order.
  const bool graphs = d.use_graphs && !ctx->timer.on && st != nullptr;  // no capture on the null stream
  if (graphs && (int)d.graphs.size() != m) {
    drop_graphs(d);
    d.graphs.assign(m, nullptr);
  }
  auto enqueue_iteration = [&](int k) -> int {
    if (!graphs) {
      kernels_of_iteration(k, ticket_for(k));
      return CPM_OK;
    }
    if (!d.graphs[k]) {
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      kernels_of_iteration(k, 1);
      HIPCHK(hipStreamEndCapture(st, &g));
      const hipError_t e = hipGraphInstantiate(&d.graphs[k], g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      HIPCHK(e);
    }
    *(volatile unsigned long long*)&slots[k].ticket = 0;
    expect[k] = 1;
    HIPCHK(hipGraphLaunch(d.graphs[k], st));
    return CPM_OK;
  };
  for (;;) {
    // Iteration k is checked while iteration k+1 already runs (at most one
    // iteration of work is discarded when the cycle stops).
    int kk = 0;
    if ((rc = enqueue_iteration(0)) != CPM_OK) return rc;
    for (int k = 0; k < m; ++k) {
      const bool more = k + 1 < m && iters + 1 < max_iter;
      if (more && (rc = enqueue_iteration(k + 1)) != CPM_OK) return rc;
      const double* hs = nullptr;
      if ((rc = wait(k, &hs)) != CPM_OK) return rc;
      ++iters;
      kk = k + 1;
      rel_est = hs[S_EST] / bnorm;
      if (!(hs[S_EST] > tol * bnorm) || hs[S_HK1] == 0.0 || !more) break;
    }
    launch(ctx, TIMER_KRYLOV, k_backsolve, dim3(1), dim3(64), 0, kk, L, sm);
    launch(ctx, TIMER_UPDATE, k_update_x, dim3(gv), dim3(256), 0, na, d.Z, d.ld, kk, sm + L.y(), u);
    launch_operator(ctx, u, d.V, f);  // new residual into V[0]
    launch(ctx, TIMER_KRYLOV, k_dots, dim3(rb), dim3(RED_THREADS), 0, na, d.V, 0, 1, d.V, d.part, -1, nullptr);
    launch(ctx, TIMER_KRYLOV, k_norm_finish, dim3(1), dim3(RED_THREADS), 0, d.part, rb, L, sm, slots_dev + (m + 1), ticket_for(m + 1));
    if ((rc = wait(m + 1, &hv)) != CPM_OK) return rc;
    ++cycles;
    rel_true = hv[S_BETA] / bnorm;
    if (rel_true <= tol) { status = CPM_OK; break; }
    if (iters >= max_iter || !std::isfinite(rel_true)) break;
  }
  HIPCHK(hipGetLastError());
  return finish(status, iters, cycles, rel_true, rel_est);
}

// ---------------------------------------------------------------------------
// GMRES(m) on the left-preconditioned system M^{-1} A u = M^{-1} f, the form
// the paper gives (Section 2.2), with its stopping rule (Section 6): the
// preconditioned residual ||M^{-1}(f - A u)|| reduced to tol ||M^{-1} f||.
// x0 = 0, CGS2 Arnoldi, Givens; the basis vector V[k] is normalised on the fly
// (M^{-1} A is linear: M^{-1} A (V[k] / ||V[k]||) is formed from the raw V[k]
// with the scale folded into the preconditioner apply), and the solution is
// u += V y. Z[0] holds A V[k] and the residual f - A u.
// ---------------------------------------------------------------------------
int dev_solve_left(cpm_ctx* ctx, const double* f, double* u, double tol, int max_iter, int m, cpm_solve_info* info) {
  HIPCHK(hipSetDevice(ctx->device));
  int rc = ensure_krylov(ctx, m);
  if (rc != CPM_OK) return rc;
  Dev& d = ctx->dev;
  const int64_t na = ctx->band.n_act;
  const SmallLayout L{m};
  double* sm = d.small;
  double* scal = sm + L.scal();
  double* T = d.Z;
  hipStream_t st = ctx->stream;
  const unsigned gv = nblk(na, 256);
  const int rb = red_blocks(na);
  const double ih2 = 1.0 / (ctx->band.h * ctx->band.h);
  const double diag = ctx->c + 6.0 * ih2;
  PhaseClock clock;
  clock.start(ctx);
  hipEvent_t t0, t1;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  HIPCHK(hipEventRecord(t0, st));
  HostSlot* slots = d.slots;
  std::vector<unsigned long long> expect(m + 2, 0);
  auto ticket_for = [&](int slot) -> unsigned long long {
    expect[slot] = ++d.ticket;
    return expect[slot];
  };
  auto wait = [&](int slot, const double** out) -> int {
    volatile unsigned long long* tk = &slots[slot].ticket;
    for (long spin = 0;; ++spin) {
      if (*tk == expect[slot]) break;
      if ((spin & 1023) == 1023) {
        const hipError_t q = hipStreamQuery(st);
        if (q != hipSuccess && q != hipErrorNotReady) {
          ctx->err = std::string("solve_left: device error ") + hipGetErrorString(q);
          return CPM_EDEVICE;
        }
        if (q == hipSuccess && *tk != expect[slot]) {
          ctx->err = "solve_left: stream idle but the step's result never arrived";
          return CPM_EDEVICE;
        }
      }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    *out = (const double*)slots[slot].v;
    return CPM_OK;
  };
  // ||x|| of a device vector (its S_INV lands in the scalars, as for a basis vector)
  auto norm_of = [&](const double* x, double* out) -> int {
    launch(ctx, TIMER_KRYLOV, k_dots, dim3(rb), dim3(RED_THREADS), 0, na, const_cast<double*>(x), (int64_t)0, 1, x,
           d.part, -1, (const double*)nullptr);
    launch(ctx, TIMER_KRYLOV, k_norm_finish, dim3(1), dim3(RED_THREADS), 0, (const double*)d.part, rb, L, sm,
           d.slots_dev + (m + 1), ticket_for(m + 1));
    const double* hv = nullptr;
    const int r = wait(m + 1, &hv);
    if (r == CPM_OK) *out = hv[S_BETA];
    return r;
  };
  auto finish = [&](int code, int iters, int cycles, double rel_true, double rel_est) -> int {
    hipEventRecord(t1, st);
    hipEventSynchronize(t1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, t0, t1);
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    if (info) {
      info->iters = iters;
      info->cycles = cycles;
      info->status = code;
      info->relres_true = rel_true;
      info->relres_est = rel_est;
      info->ms = ms;
      clock.stop(ctx, info->phase_ms);
    }
    return code;
  };
  launch(ctx, TIMER_UPDATE, k_fill, dim3(gv), dim3(256), 0, na, u, 0.0);
  double fnorm = 0.0, beta0 = 0.0;
  if ((rc = norm_of(f, &fnorm)) != CPM_OK) return rc;
  if (!std::isfinite(fnorm)) {
    finish(CPM_EINVAL, 0, 0, NAN, NAN);
    ctx->err = "solve_left: right-hand side is not finite";
    return CPM_EINVAL;
  }
  if (fnorm == 0.0) return finish(CPM_OK, 0, 0, 0.0, 0.0);
  launch_precond(ctx, f, d.V);  // V[0] = M^{-1} f (x0 = 0)
  if ((rc = norm_of(d.V, &beta0)) != CPM_OK) return rc;
  if (!(beta0 > 0.0) || !std::isfinite(beta0)) {
    finish(CPM_EINVAL, 0, 0, NAN, NAN);
    ctx->err = "solve_left: preconditioned right-hand side is zero or not finite";
    return CPM_EINVAL;
  }
  int iters = 0, cycles = 0;
  double rel = 1.0;
  int status = CPM_ENOTCONV;
  auto enqueue_iteration = [&](int k) {
    double* vk = d.V + (size_t)k * d.ld;
    double* w = d.V + (size_t)(k + 1) * d.ld;
    const BatchStrides one{};
    launch_extend(ctx, vk, d.e);  // T = A V[k] (raw), then w = M^{-1} T / ||V[k]||
    launch(ctx, TIMER_STENCIL, k_stencil, dim3(gv), dim3(256), 0, na, diag, ih2, (const int32_t*)d.nbr,
           (const double*)vk, (const double*)d.e, (const double*)nullptr, T);
    launch_precond(ctx, T, w, scal + S_INV);
    // CGS pass 1 (normalising V[k] in place), pass 2, ||w|| and the Givens update
    launch(ctx, TIMER_KRYLOV, k_dots, dim3(rb), dim3(RED_THREADS), 0, na, d.V, d.ld, k + 1, (const double*)w, d.part,
           k, (const double*)(scal + S_INV));
    launch(ctx, TIMER_KRYLOV, k_reduce_cols, dim3(k + 1), dim3(RED_THREADS), 0, (const double*)d.part, rb,
           sm + L.h1(), one);
    launch(ctx, TIMER_KRYLOV, k_axpy_dots, dim3(rb), dim3(RED_THREADS), 0, na, (const double*)d.V, d.ld, k,
           (const double*)(sm + L.h1()), w, d.part, 0, one);
    launch(ctx, TIMER_KRYLOV, k_reduce_cols, dim3(k + 1), dim3(RED_THREADS), 0, (const double*)d.part, rb,
           sm + L.h2(), one);
    launch(ctx, TIMER_KRYLOV, k_axpy_dots, dim3(rb), dim3(RED_THREADS), 0, na, (const double*)d.V, d.ld, k,
           (const double*)(sm + L.h2()), w, d.part, 1, one);
    launch(ctx, TIMER_KRYLOV, k_arnoldi, dim3(1), dim3(RED_THREADS), 0, (const double*)d.part, rb, k, L, sm,
           d.slots_dev + k, ticket_for(k), one);
  };
  for (;;) {
    int kk = 0;
    enqueue_iteration(0);
    for (int k = 0; k < m; ++k) {
      // iteration k+1 is queued before iteration k is checked
      const bool more = k + 1 < m && iters + 1 < max_iter;
      if (more) enqueue_iteration(k + 1);
      const double* hs = nullptr;
      if ((rc = wait(k, &hs)) != CPM_OK) return rc;
      ++iters;
      kk = k + 1;
      if (!(hs[S_EST] > tol * beta0) || hs[S_HK1] == 0.0 || !more) break;
    }
    launch(ctx, TIMER_KRYLOV, k_backsolve, dim3(1), dim3(64), 0, kk, L, sm);
    launch(ctx, TIMER_UPDATE, k_update_x, dim3(gv), dim3(256), 0, na, (const double*)d.V, d.ld, kk,
           (const double*)(sm + L.y()), u);
    launch_operator(ctx, u, T, f);  // T = f - A u
    launch_precond(ctx, T, d.V);    // V[0] = M^{-1}(f - A u)
    double beta = 0.0;
    if ((rc = norm_of(d.V, &beta)) != CPM_OK) return rc;
    ++cycles;
    rel = beta / beta0;
    if (rel <= tol) {
      status = CPM_OK;
      break;
    }
    if (iters >= max_iter || !std::isfinite(rel)) break;
  }
  double rnorm = 0.0;  // ||f - A u||: T still holds it
  if ((rc = norm_of(T, &rnorm)) != CPM_OK) return rc;
  HIPCHK(hipGetLastError());
  return finish(status, iters, cycles, rnorm / fnorm, rel);
}

// ---------------------------------------------------------------------------
// Several right-hand sides in lockstep: the per-iteration kernels run for the
// whole batch in one launch each (blockIdx.y = right-hand side) and the
// preconditioner streams W once for all of them. Each right-hand side follows
// exactly the single-solve sequence (same kernels, same sums, same restarts;
// one that has stopped within a cycle idles until the cycle ends), so the
// results equal separate solves bit for bit.
// ---------------------------------------------------------------------------
static int ensure_krylov_batch(cpm_ctx* ctx, int m, int nb) {
  Dev& d = ctx->dev;
  if (d.b_restart == m && d.b_n >= nb && d.bV) return CPM_OK;
  dfree(d.bV);
  dfree(d.bZ);
  dfree(d.bE);
  dfree(d.bpart);
  dfree(d.bsmall);
  if (d.bslots) hipHostFree(d.bslots);
  d.bslots = d.bslots_dev = nullptr;
  d.b_restart = d.b_n = 0;
  const int64_t na = ctx->band.n_act, nt = ctx->band.total();
  const int64_t ld = round_up(na, 64);
  const SmallLayout L{m};
  HIPCHK(hipMalloc((void**)&d.bV, (size_t)nb * (m + 1) * ld * sizeof(double)));
  HIPCHK(hipMalloc((void**)&d.bZ, (size_t)nb * m * ld * sizeof(double)));
  HIPCHK(hipMalloc((void**)&d.bE, (size_t)nb * round_up(nt, 64) * sizeof(double)));
  HIPCHK(hipMalloc((void**)&d.bpart, (size_t)nb * RED_MAX_BLOCKS * PART_LD * sizeof(double)));
  HIPCHK(hipMalloc((void**)&d.bsmall, (size_t)nb * L.size() * sizeof(double)));
  HIPCHK(hipHostMalloc((void**)&d.bslots, (size_t)nb * (m + 2) * sizeof(HostSlot),
                       hipHostMallocMapped | hipHostMallocCoherent));
  std::memset((void*)d.bslots, 0, (size_t)nb * (m + 2) * sizeof(HostSlot));
  HIPCHK(hipHostGetDevicePointer((void**)&d.bslots_dev, d.bslots, 0));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  d.b_restart = m;
  d.b_n = nb;
  d.batch_bytes = ((size_t)nb * ((2 * m + 1) * ld + round_up(nt, 64) + RED_MAX_BLOCKS * PART_LD + L.size())) *
                  sizeof(double);
  return CPM_OK;
}

// Right-hand sides one pass over W can serve: v_q|Sigma_j for all of them must
// fit in LDS next to each other (0: batching not available).
int dev_batch_width(cpm_ctx* ctx, int nrhs) {
  const Dev& d = ctx->dev;
  if (nrhs < 2 || d.chunk > 0 || d.prec < 0) return 0;
  const size_t per = (size_t)d.max_m * sizeof(double);
  for (int nb : {4, 2})
    if (nb <= nrhs && nb * per <= 160 * 1024) return nb;
  return 0;
}

// Tilings of the several-right-hand-side apply; every one gives the single
// apply's sums bit for bit. Each names rows per wave, chunks in flight per
// row, whether two register sets alternate (the next group's loads issued
// before the current group's products), and the blocks planned per resident
// block slot. One block holds every vector of the batch in LDS, so few fit on
// a CU and each block's gather of v|Sigma_j runs with little else beside it:
// fewer, larger blocks than the single apply's plan pay it less often.
struct MultiTiling {
  int rpw, unr;
  bool pipe;
  int over;
};
constexpr int N_MULTI_TILINGS = CPM_MULTI_TILINGS;
constexpr MultiTiling kMultiTilings[N_MULTI_TILINGS] = {{8, 1, false, 1}, {8, 1, false, 2}, {8, 1, false, 4},
                                                        {4, 2, true, 1},  {4, 2, true, 2},  {4, 2, true, 4},
                                                        {4, 1, true, 2},  {4, 2, false, 2}};

// Calls f with the kernel of tiling t.
template <typename T, int NB, int I, class F>
static void multi_fn_at(F&& f) {
  constexpr MultiTiling m = kMultiTilings[I];
  f(k_precond_multi<T, NB, m.rpw, m.unr, m.pipe>);
}
template <typename T, int NB, class F>
static void with_multi_fn(int t, F&& f) {
  static_assert(N_MULTI_TILINGS == 8, "one case per multi tiling");
  switch (t) {
    case 0: multi_fn_at<T, NB, 0>(f); break;
    case 1: multi_fn_at<T, NB, 1>(f); break;
    case 2: multi_fn_at<T, NB, 2>(f); break;
    case 3: multi_fn_at<T, NB, 3>(f); break;
    case 4: multi_fn_at<T, NB, 4>(f); break;
    case 5: multi_fn_at<T, NB, 5>(f); break;
    case 6: multi_fn_at<T, NB, 6>(f); break;
    default: multi_fn_at<T, NB, 7>(f); break;
  }
}

template <typename T, int NB>
static void launch_multi_typed(cpm_ctx* ctx, const double* v, int64_t v_stride, const double* scale,
                               int64_t scale_stride, double* z, int64_t z_stride) {
  Dev& d = ctx->dev;
  const size_t lds = (size_t)NB * d.max_m * sizeof(double);
  with_multi_fn<T, NB>(d.multi_tiling, [&](auto fn) {
    if (lds > 64 * 1024) hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    launch(ctx, TIMER_PRECOND, fn, dim3(d.m_n_blocks), dim3(PRECOND_THREADS), lds, (const SubDesc*)d.mdesc,
           (const int32_t*)d.mblk_sub, (const int32_t*)d.sig_idx, (const int32_t*)d.tilde_idx, (const T*)d.W, v,
           v_stride, scale, scale_stride, z, z_stride);
  });
}

template <int NB>
static void launch_precond_multi(cpm_ctx* ctx, const double* v, int64_t v_stride, const double* scale,
                                 int64_t scale_stride, double* z, int64_t z_stride) {
  if (ctx->dev.prec == CPM_FP64)
    launch_multi_typed<double, NB>(ctx, v, v_stride, scale, scale_stride, z, z_stride);
  else
    launch_multi_typed<float, NB>(ctx, v, v_stride, scale, scale_stride, z, z_stride);
}

// Plan of the several-right-hand-side apply for the current multi tiling:
// n_cu x (blocks of the widest batch that fit on a CU) x over blocks,
// apportioned to subdomains by W bytes and cut into whole tiles as the single
// apply's. (Rounding rows per block up to whole passes of the eight waves
// measured slower: it leaves fewer blocks than slots x over, so the CUs run
// uneven numbers of them.) No plan (and no batched apply) when no batch of
// two fits.
int plan_multi(cpm_ctx* ctx) {
  Dev& dv = ctx->dev;
  dfree(dv.mdesc);
  dfree(dv.mblk_sub);
  dv.m_n_blocks = 0;
  const int nb = dev_batch_width(ctx, 4);
  if (nb < 2) return CPM_OK;
  HIPCHK(hipSetDevice(ctx->device));
  const MultiTiling& mt = kMultiTilings[dv.multi_tiling];
  const size_t lds = (size_t)nb * dv.max_m * sizeof(double);
  int n_cu = 0, per_cu = 0;
  HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  hipError_t e = hipSuccess;
  auto occ = [&](auto fn) {
    if (lds > 64 * 1024) hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, PRECOND_THREADS, lds);
  };
  if (dv.prec == CPM_FP64)
    nb == 4 ? with_multi_fn<double, 4>(dv.multi_tiling, occ) : with_multi_fn<double, 2>(dv.multi_tiling, occ);
  else
    nb == 4 ? with_multi_fn<float, 4>(dv.multi_tiling, occ) : with_multi_fn<float, 2>(dv.multi_tiling, occ);
  HIPCHK(e);
  per_cu = std::max(1, per_cu);
  const std::vector<int> want = apportion_blocks(ctx->dec, n_cu * per_cu * mt.over);
  std::vector<SubDesc> hd = dv.hdesc;
  std::vector<int32_t> blk_sub;
  int32_t blk = 0;
  for (int j = 0; j < ctx->dec.n_sub; ++j) {
    SubDesc& d = hd[j];
    d.rpb = rows_per_block(d.t, want[j]);
    const int n = (d.t + d.rpb - 1) / d.rpb;
    d.blk_off = blk;
    for (int q = 0; q < n; ++q) blk_sub.push_back(j);
    blk += n;
  }
  int rc = upload(ctx, &dv.mdesc, hd);
  if (rc == CPM_OK) rc = upload(ctx, &dv.mblk_sub, blk_sub);
  if (rc != CPM_OK) {
    dfree(dv.mdesc);
    dfree(dv.mblk_sub);
    return rc;
  }
  dv.m_n_blocks = blk;
  return CPM_OK;
}

int dev_solve_batch(cpm_ctx* ctx, const double* f, double* u, int nb, double tol, int max_iter, int m,
                    cpm_solve_info* info) {
  HIPCHK(hipSetDevice(ctx->device));
  int rc = ensure_krylov_batch(ctx, m, nb);
  if (rc != CPM_OK) return rc;
  Dev& d = ctx->dev;
  const int64_t na = ctx->band.n_act;
  const int64_t ld = round_up(na, 64);
  const SmallLayout L{m};
  BatchStrides bs;
  bs.v = (int64_t)(m + 1) * ld;
  bs.z = (int64_t)m * ld;
  bs.e = round_up(ctx->band.total(), 64);
  bs.part = (int64_t)RED_MAX_BLOCKS * PART_LD;
  bs.small = L.size();
  bs.slot = m + 2;
  hipStream_t st = ctx->stream;
  const unsigned gv = nblk(na, 256);
  const int rb = red_blocks(na);
  const double ih2 = 1.0 / (ctx->band.h * ctx->band.h);
  const double diag = ctx->c + 6.0 * ih2;
  auto Vp = [&](int r, int k) { return d.bV + r * bs.v + (int64_t)k * ld; };
  auto Zp = [&](int r, int k) { return d.bZ + r * bs.z + (int64_t)k * ld; };
  auto SM = [&](int r) { return d.bsmall + r * bs.small; };
  auto PART = [&](int r) { return d.bpart + r * bs.part; };
  const double* fr[8];
  double* ur[8];
  for (int r = 0; r < nb; ++r) {
    fr[r] = f + (size_t)r * na;
    ur[r] = u + (size_t)r * na;
  }
  PhaseClock clock;
  clock.start(ctx);
  hipEvent_t t0, t1;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  HIPCHK(hipEventRecord(t0, st));
  std::vector<unsigned long long> expect(m + 2, 0);
  auto ticket_for = [&](int slot) -> unsigned long long {
    expect[slot] = ++d.ticket;
    return expect[slot];
  };
  auto wait = [&](int r, int slot, const double** out) -> int {
    HostSlot* hs = d.bslots + r * bs.slot + slot;
    volatile unsigned long long* tk = &hs->ticket;
    for (long spin = 0;; ++spin) {
      if (*tk == expect[slot]) break;
      if ((spin & 1023) == 1023) {
        const hipError_t q = hipStreamQuery(st);
        if (q != hipSuccess && q != hipErrorNotReady) {
          ctx->err = std::string("solve: device error ") + hipGetErrorString(q);
          return CPM_EDEVICE;
        }
        if (q == hipSuccess && *tk != expect[slot]) {
          ctx->err = "solve: stream idle but the step's result never arrived";
          return CPM_EDEVICE;
        }
      }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    *out = (const double*)hs->v;
    return CPM_OK;
  };
  std::vector<int> iters(nb, 0), cycles(nb, 0), kk(nb, 0), status(nb, CPM_ENOTCONV);
  std::vector<double> bnorm(nb, 0.0), rel_true(nb, 1.0), rel_est(nb, 1.0);
  std::vector<char> done(nb, 0), stopped(nb, 0);
  auto finish = [&](int code) -> int {
    hipEventRecord(t1, st);
    hipEventSynchronize(t1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, t0, t1);
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    double phase[4];
    clock.stop(ctx, phase);
    if (info)
      for (int r = 0; r < nb; ++r) {
        info[r].iters = iters[r];
        info[r].cycles = cycles[r];
        info[r].status = status[r];
        info[r].relres_true = rel_true[r];
        info[r].relres_est = rel_est[r];
        info[r].ms = ms;
        for (int q = 0; q < 4; ++q) info[r].phase_ms[q] = phase[q];
      }
    return code;
  };
  // ||f_r||, with V_r[0] = f_r (x0 = 0) as the first residual
  for (int r = 0; r < nb; ++r) {
    launch(ctx, TIMER_UPDATE, k_copy, dim3(gv), dim3(256), 0, na, fr[r], Vp(r, 0));
    launch(ctx, TIMER_UPDATE, k_fill, dim3(gv), dim3(256), 0, na, ur[r], 0.0);
    launch(ctx, TIMER_KRYLOV, k_dots, dim3(rb), dim3(RED_THREADS), 0, na, Vp(r, 0), 0, 1, Vp(r, 0), PART(r), -1, nullptr);
  }
  {
    const unsigned long long tk = ticket_for(m + 1);
    for (int r = 0; r < nb; ++r)
      launch(ctx, TIMER_KRYLOV, k_norm_finish, dim3(1), dim3(RED_THREADS), 0, PART(r), rb, L, SM(r), d.bslots_dev + r * bs.slot + (m + 1), tk);
  }
  for (int r = 0; r < nb; ++r) {
    const double* hv = nullptr;
    if ((rc = wait(r, m + 1, &hv)) != CPM_OK) return rc;
    bnorm[r] = hv[S_BETA];
    if (!std::isfinite(bnorm[r])) {
      finish(CPM_EINVAL);
      ctx->err = "solve: right-hand side is not finite";
      return CPM_EINVAL;
    }
    if (bnorm[r] == 0.0) {
      done[r] = 1;
      status[r] = CPM_OK;
      rel_true[r] = rel_est[r] = 0.0;
    }
  }
  auto enqueue_iteration = [&](int k) {
    double* scal_inv = d.bsmall + L.scal() + S_INV;
    if (nb == 4)
      launch_precond_multi<4>(ctx, Vp(0, k), bs.v, scal_inv, bs.small, Zp(0, k), bs.z);
    else
      launch_precond_multi<2>(ctx, Vp(0, k), bs.v, scal_inv, bs.small, Zp(0, k), bs.z);
    launch_extend(ctx, Zp(0, k), d.bE, nb, bs.z, bs.e);
    launch(ctx, TIMER_STENCIL, k_stencil_dots, dim3(rb, nb), dim3(RED_THREADS), 0, na, diag, ih2, d.nbr, Zp(0, k), d.bE, Vp(0, k + 1), d.bV,
                                                         ld, k + 1, d.bpart, k, scal_inv, bs);
    launch(ctx, TIMER_KRYLOV, k_reduce_cols, dim3(k + 1, nb), dim3(RED_THREADS), 0, d.bpart, rb, d.bsmall + L.h1(), bs);
    launch(ctx, TIMER_KRYLOV, k_axpy_dots, dim3(rb, nb), dim3(RED_THREADS), 0, na, d.bV, ld, k, d.bsmall + L.h1(), Vp(0, k + 1), d.bpart, 0,
                                                      bs);
    launch(ctx, TIMER_KRYLOV, k_reduce_cols, dim3(k + 1, nb), dim3(RED_THREADS), 0, d.bpart, rb, d.bsmall + L.h2(), bs);
    launch(ctx, TIMER_KRYLOV, k_axpy_dots, dim3(rb, nb), dim3(RED_THREADS), 0, na, d.bV, ld, k, d.bsmall + L.h2(), Vp(0, k + 1), d.bpart, 1,
                                                      bs);
    launch(ctx, TIMER_KRYLOV, k_arnoldi, dim3(1, nb), dim3(RED_THREADS), 0, d.bpart, rb, k, L, d.bsmall, d.bslots_dev + k, ticket_for(k), bs);
  };
  for (;;) {
    bool any = false;
    for (int r = 0; r < nb; ++r) {
      stopped[r] = done[r];
      kk[r] = 0;
      any |= !done[r];
    }
    if (!any) break;
    enqueue_iteration(0);
    for (int k = 0; k < m; ++k) {
      // iteration k+1 is queued before iteration k is checked (as in a single solve)
      bool more = false;
      for (int r = 0; r < nb; ++r)
        if (!stopped[r] && k + 1 < m && iters[r] + 1 < max_iter) more = true;
      if (more) enqueue_iteration(k + 1);
      bool all_stopped = true;
      for (int r = 0; r < nb; ++r) {
        if (stopped[r]) continue;
        const double* hs = nullptr;
        if ((rc = wait(r, k, &hs)) != CPM_OK) return rc;
        ++iters[r];
        kk[r] = k + 1;
        rel_est[r] = hs[S_EST] / bnorm[r];
        const bool more_r = k + 1 < m && iters[r] < max_iter;
        if (!(hs[S_EST] > tol * bnorm[r]) || hs[S_HK1] == 0.0 || !more_r) stopped[r] = 1;
        all_stopped &= (bool)stopped[r];
      }
      if (all_stopped || !more) break;
    }
    // cycle end: update, true residual and its norm for every right-hand side still running
    for (int r = 0; r < nb; ++r) {
      if (done[r]) continue;
      launch(ctx, TIMER_KRYLOV, k_backsolve, dim3(1), dim3(64), 0, kk[r], L, SM(r));
      launch(ctx, TIMER_UPDATE, k_update_x, dim3(gv), dim3(256), 0, na, Zp(r, 0), ld, kk[r], SM(r) + L.y(), ur[r]);
      launch_operator(ctx, ur[r], Vp(r, 0), fr[r]);
      launch(ctx, TIMER_KRYLOV, k_dots, dim3(rb), dim3(RED_THREADS), 0, na, Vp(r, 0), 0, 1, Vp(r, 0), PART(r), -1, nullptr);
    }
    const unsigned long long tk = ticket_for(m + 1);
    for (int r = 0; r < nb; ++r)
      if (!done[r])
        launch(ctx, TIMER_KRYLOV, k_norm_finish, dim3(1), dim3(RED_THREADS), 0, PART(r), rb, L, SM(r), d.bslots_dev + r * bs.slot + (m + 1), tk);
    for (int r = 0; r < nb; ++r) {
      if (done[r]) continue;
      const double* hv = nullptr;
      if ((rc = wait(r, m + 1, &hv)) != CPM_OK) return rc;
      ++cycles[r];
      rel_true[r] = hv[S_BETA] / bnorm[r];
      if (rel_true[r] <= tol) {
        status[r] = CPM_OK;
        done[r] = 1;
      } else if (iters[r] >= max_iter || !std::isfinite(rel_true[r])) {
        done[r] = 1;
      }
    }
  }
  HIPCHK(hipGetLastError());
  int worst = CPM_OK;
  for (int r = 0; r < nb; ++r) worst = std::max(worst, status[r]);
  return finish(worst);
}

// (O)RAS as a stationary solver: u <- u + M^{-1}(f - A u), u0 = 0. Each step
// applies z = M^{-1} r_n, u_{n+1} = u_n + z, then computes r_{n+1} = f - A u_{n+1}
// and its norm, which the host reads (one wait per step) for the stopping test.
int dev_stationary(cpm_ctx* ctx, const double* f, double* u, double tol, int max_iter, cpm_solve_info* info) {
  HIPCHK(hipSetDevice(ctx->device));
  const int m = ctx->dev.restart > 0 ? ctx->dev.restart : 2;
  int rc = ensure_krylov(ctx, m);
  if (rc != CPM_OK) return rc;
  Dev& d = ctx->dev;
  const int64_t na = ctx->band.n_act;
  const SmallLayout L{m};
  double* sm = d.small;
  hipStream_t st = ctx->stream;
  const unsigned gv = nblk(na, 256);
  const int rb = red_blocks(na);
  double* r = d.V;
  double* z = d.Z;
  unsigned long long expect[2] = {0, 0};
  PhaseClock clock;
  clock.start(ctx);
  hipEvent_t t0, t1;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  HIPCHK(hipEventRecord(t0, st));
  auto residual = [&](int slot) {
    launch_operator(ctx, u, r, f);  // r = f - A u
    launch(ctx, TIMER_KRYLOV, k_dots, dim3(rb), dim3(RED_THREADS), 0, na, r, 0, 1, r, d.part, -1, nullptr);
    expect[slot] = ++d.ticket;
    launch(ctx, TIMER_KRYLOV, k_norm_finish, dim3(1), dim3(RED_THREADS), 0, d.part, rb, L, sm, d.slots_dev + slot, expect[slot]);
  };
  auto wait = [&](int slot, double* out) -> int {
    volatile unsigned long long* tk = &d.slots[slot].ticket;
    for (long spin = 0;; ++spin) {
      if (*tk == expect[slot]) break;
      if ((spin & 1023) == 1023) {
        const hipError_t q = hipStreamQuery(st);
        if (q != hipSuccess && q != hipErrorNotReady) {
          ctx->err = std::string("solve_stationary: device error ") + hipGetErrorString(q);
          return CPM_EDEVICE;
        }
        if (q == hipSuccess && *tk != expect[slot]) {
          ctx->err = "solve_stationary: stream idle but the step's result never arrived";
          return CPM_EDEVICE;
        }
      }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    *out = d.slots[slot].v[S_BETA];
    return CPM_OK;
  };
  auto finish = [&](int code, int iters, double rel) -> int {
    hipEventRecord(t1, st);
    hipEventSynchronize(t1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, t0, t1);
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    if (info) {
      info->iters = iters;
      info->cycles = iters;
      info->status = code;
      info->relres_true = rel;
      info->relres_est = rel;
      info->ms = ms;
      clock.stop(ctx, info->phase_ms);
    }
    return code;
  };
  launch(ctx, TIMER_UPDATE, k_fill, dim3(gv), dim3(256), 0, na, u, 0.0);
  residual(0);
  double bnorm = 0.0;
  if ((rc = wait(0, &bnorm)) != CPM_OK) return rc;
  if (!std::isfinite(bnorm)) {
    finish(CPM_EINVAL, 0, NAN);
    ctx->err = "solve_stationary: right-hand side is not finite";
    return CPM_EINVAL;
  }
  if (bnorm == 0.0) return finish(CPM_OK, 0, 0.0);
  int n = 0;
  double rel = 1.0;
  for (;;) {
    // update n, then the residual of u_{n+1}
    launch_precond(ctx, r, z, nullptr);
    launch(ctx, TIMER_UPDATE, k_axpy, dim3(gv), dim3(256), 0, na, z, u);
    ++n;
    residual(n & 1);
    double bn = 0.0;
    if ((rc = wait(n & 1, &bn)) != CPM_OK) return rc;
    rel = bn / bnorm;
    if (rel <= tol) return finish(CPM_OK, n, rel);
    if (n >= max_iter || !std::isfinite(rel)) return finish(CPM_ENOTCONV, n, rel);
  }
}

// Device bytes of a factorisation before it is made: resident afterwards
// (operator arrays, W arena and its index lists, Krylov space of `restart`)
// and the peak while factoring (plus the bordered matrices, the assembly and
// elimination-order lists, the panel row bounds and the trailing-tile list). Mirrors the allocations of dev_upload_operator, make_plan,
// run_factor and ensure_krylov; the apply-block table is bounded by one entry
// per W row.
void dev_estimate(const cpm_ctx* ctx, int prec, int restart, size_t* resident, size_t* peak) {
  const Band& b = ctx->band;
  const Decomp& D = ctx->dec;
  const bool oras = D.kind == CPM_ORAS;
  const size_t esz = prec == CPM_FP64 ? 8 : 4;
  ExtPlan E;
  plan_extension(b, E);
  const size_t op = b.lines.size() * 4 + b.wts.size() * 8 + (size_t)b.n_act * 6 * 4 + (size_t)b.total() * 8 +
                    2 * E.perm.size() * 4 + E.groups.size() * sizeof(ExtGroup) +
                    (size_t)b.total() * (3 * 8 + (b.p + 1) * 4 + (b.p + 1) * b.p * 2);
  int64_t w_elems = 0, u_total = 0, t_total = 0;
  std::vector<SubDesc> desc(D.n_sub);
  for (int j = 0; j < D.n_sub; ++j) {
    const Sub& s = D.subs[j];
    SubDesc& d = desc[j];
    d.m = (int32_t)s.sigma.size();
    d.n = d.m + (oras ? (int32_t)s.bnd.size() : 0);
    d.t = (int32_t)s.tilde.size();
    d.rows = d.n + d.t;
    d.lda = (int32_t)round_up(d.n + d.m, 16);
    w_elems += w_rows_stored(d.t) * round_up(d.m, 8);
    u_total += d.n;
    t_total += d.t;
  }
  size_t ws = 0;  // largest group workspace: matrices, row bounds, tile list (64-row tiles at most)
  for (const auto& g : factor_groups(desc, esz, ctx->dev.ws_limit)) {
    size_t e = 0;
    for (int j = g.first; j < g.second; ++j) {
      const SubDesc& d = desc[j];
      e += (size_t)factor_ws_elems(d) * esz + 2 * 4 +
           (size_t)((d.rows + GEMM_TILE - 1) / GEMM_TILE) * ((d.n + d.m + GEMM_TILE - 1) / GEMM_TILE) * 8;
    }
    ws = std::max(ws, e);
  }
  const size_t lists = (size_t)D.n_sub * sizeof(SubDesc) + (size_t)(u_total + 2 * t_total) * 4;
  const size_t res = op + (size_t)w_elems * esz + lists + (restart > 0 ? krylov_bytes(b.n_act, restart) : 0);
  // per unknown: factor-order node, sorted lookup (2), B data index, pivot,
  // right-hand column, W column map, B data (2 doubles); per Sigma~ node: unit
  // entry position, W row map; per panel: two row bounds
  const size_t work = ws + (size_t)u_total * (7 * 4 + 2 * 8) + (size_t)t_total * 8 +
                      (size_t)(u_total / LU_NB + D.n_sub) * 8 + (size_t)D.n_sub * (4 + 8) + 16;
  if (resident) *resident = res;
  if (peak) *peak = res + work;
}

// Apply plan for tiling t: the resident block slots for its occupancy
// apportioned to subdomains as at factor time; the descriptors' block fields
// and the block -> subdomain table are rewritten on the device.
int dev_set_tiling(cpm_ctx* ctx, int t) {
  Dev& dv = ctx->dev;
  if (t < 0 || t >= N_TILINGS) {
    ctx->err = "precond tiling out of range";
    return CPM_EINVAL;
  }
  if (dv.prec < 0 || dv.chunk > 0) {
    ctx->err = "precond tiling: needs a factorisation with the unchunked apply";
    return CPM_ESTATE;
  }
  HIPCHK(hipSetDevice(ctx->device));
  const size_t lds = (size_t)dv.max_m * sizeof(double);
  const void* fn = dv.prec == CPM_FP64 ? tiled_fn<double>(t) : tiled_fn<float>(t);
  if (lds > 64 * 1024) hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  int n_cu = 0, per_cu = 0;
  HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, PRECOND_THREADS, lds));
  per_cu = std::max(1, per_cu);
  const std::vector<int> want = apportion_blocks(ctx->dec, n_cu * per_cu * kTilings[t].over2 / 2);
  std::vector<int32_t> blk_sub;
  int32_t blk = 0;
  for (int j = 0; j < ctx->dec.n_sub; ++j) {
    SubDesc& d = dv.hdesc[j];
    d.rpb = rows_per_block(d.t, want[j]);
    const int nb = (d.t + d.rpb - 1) / d.rpb;
    d.blk_off = blk;
    for (int q = 0; q < nb; ++q) blk_sub.push_back(j);
    blk += nb;
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  drop_graphs(dv);
  HIPCHK(hipMemcpy(dv.desc, dv.hdesc.data(), dv.hdesc.size() * sizeof(SubDesc), hipMemcpyHostToDevice));
  dfree(dv.blk_sub);
  int rc = upload(ctx, &dv.blk_sub, blk_sub);
  if (rc != CPM_OK) return rc;
  dv.n_blocks = blk;
  dv.tiling = t;
  return CPM_OK;
}

// Operator-apply kernel: 0 compact rows with gathers of x from device memory
// (when the increments fit 16 bits), 1 stages each group's x in LDS (when the
// largest group fits), 2 full rows with gathers; results are identical.
int dev_set_operator_kernel(cpm_ctx* ctx, int k) {
  if (k < 0 || k > 2) {
    ctx->err = "operator kernel must be 0, 1 or 2";
    return CPM_EINVAL;
  }
  ctx->dev.op_kernel = k;
  drop_graphs(ctx->dev);
  return CPM_OK;
}

// Time every tiling on the resident factors (one warm-up and `reps` applies
// each, HIP events on the context stream) and keep the fastest.
int dev_autotune(cpm_ctx* ctx, int reps, int* best, double* ms) {
  Dev& dv = ctx->dev;
  if (dv.prec < 0 || dv.chunk > 0) {
    ctx->err = "autotune: needs a factorisation with the unchunked apply";
    return CPM_ESTATE;
  }
  HIPCHK(hipSetDevice(ctx->device));
  const int64_t na = ctx->band.n_act;
  double *v = nullptr, *z = nullptr;
  HIPCHK(hipMalloc((void**)&v, na * sizeof(double)));
  HIPCHK(hipMalloc((void**)&z, na * sizeof(double)));
  k_fill<<<nblk(na, 256), 256, 0, ctx->stream>>>(na, z, 1.0);
  // Each timed apply takes a vector the operator has just written, as inside
  // FGMRES (z_k = M^{-1} v_k, then A z_k), so the gather of v|Sigma_j and the
  // caches are in the state of a solve; only the apply launches are timed
  // (per-launch events), and the caller's kernel timers are left as they were.
  Timer& tm = ctx->timer;
  timer_harvest(ctx);
  const bool was_on = tm.on;
  int rc = CPM_OK, arg = 0;
  double tbest = 0.0;
  for (int t = 0; t < N_TILINGS && rc == CPM_OK; ++t) {
    rc = dev_set_tiling(ctx, t);
    if (rc != CPM_OK) break;
    tm.on = false;
    launch_operator(ctx, z, v, nullptr);
    launch_precond(ctx, v, z);
    timer_harvest(ctx);
    double ms0[N_TIMERS];
    int64_t n0[N_TIMERS];
    for (int q = 0; q < N_TIMERS; ++q) {
      ms0[q] = tm.ms[q];
      n0[q] = tm.count[q];
    }
    tm.on = true;
    for (int r = 0; r < reps; ++r) {
      launch_operator(ctx, z, v, nullptr);
      launch_precond(ctx, v, z);
    }
    timer_harvest(ctx);
    tm.on = was_on;
    const int64_t n = tm.count[TIMER_PRECOND] - n0[TIMER_PRECOND];
    const double per = n > 0 ? (tm.ms[TIMER_PRECOND] - ms0[TIMER_PRECOND]) / n : 0.0;
    for (int q = 0; q < N_TIMERS; ++q) {  // the caller's totals as they were
      tm.ms[q] = ms0[q];
      tm.count[q] = n0[q];
    }
    if (ms) ms[t] = per;
    if (t == 0 || per < tbest) {
      tbest = per;
      arg = t;
    }
  }
  tm.on = was_on;
  hipStreamSynchronize(ctx->stream);
  dfree(v);
  dfree(z);
  if (rc != CPM_OK) return rc;
  if (best) *best = arg;
  return dev_set_tiling(ctx, arg);
}

// Tiling of the several-right-hand-side apply; autotune times each on the
// resident factors with the widest batch that fits (vectors an operator
// apply has just written), keeping the caller's kernel timers unchanged.
int dev_set_multi_tiling(cpm_ctx* ctx, int t) {
  if (t < 0 || t >= N_MULTI_TILINGS) {
    ctx->err = "multi tiling out of range";
    return CPM_EINVAL;
  }
  if (ctx->dev.prec < 0) {
    ctx->err = "multi tiling: factor first";
    return CPM_ESTATE;
  }
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->dev.multi_tiling = t;
  return plan_multi(ctx);
}

int dev_autotune_multi(cpm_ctx* ctx, int reps, int* best, double* ms) {
  Dev& dv = ctx->dev;
  const int nb = dev_batch_width(ctx, 4);
  if (nb < 2) {
    ctx->err = "autotune_multi: no batched apply for these factors";
    return CPM_ESTATE;
  }
  HIPCHK(hipSetDevice(ctx->device));
  const int64_t na = ctx->band.n_act;
  double *v = nullptr, *z = nullptr;
  HIPCHK(hipMalloc((void**)&v, (size_t)nb * na * sizeof(double)));
  if (hipMalloc((void**)&z, (size_t)nb * na * sizeof(double)) != hipSuccess) {
    dfree(v);
    ctx->err = "autotune_multi: device allocation failed";
    return CPM_ENOMEM;
  }
  k_fill<<<nblk((int64_t)nb * na, 256), 256, 0, ctx->stream>>>((int64_t)nb * na, z, 1.0);
  Timer& tm = ctx->timer;
  timer_harvest(ctx);
  const bool was_on = tm.on;
  double ms0[N_TIMERS];
  int64_t n0[N_TIMERS];
  for (int q = 0; q < N_TIMERS; ++q) {
    ms0[q] = tm.ms[q];
    n0[q] = tm.count[q];
  }
  auto pass = [&]() {
    for (int q = 0; q < nb; ++q) launch_operator(ctx, z + (size_t)q * na, v + (size_t)q * na, nullptr);
    if (nb == 4)
      launch_precond_multi<4>(ctx, v, na, nullptr, 0, z, na);
    else
      launch_precond_multi<2>(ctx, v, na, nullptr, 0, z, na);
  };
  int arg = 0;
  double tbest = 0.0;
  int rc = CPM_OK;
  for (int t = 0; t < N_MULTI_TILINGS && rc == CPM_OK; ++t) {
    hipStreamSynchronize(ctx->stream);  // the previous plan's launches are done
    dv.multi_tiling = t;
    rc = plan_multi(ctx);
    if (rc != CPM_OK) break;
    tm.on = false;
    pass();
    timer_harvest(ctx);
    const double m0 = tm.ms[TIMER_PRECOND];
    const int64_t c0 = tm.count[TIMER_PRECOND];
    tm.on = true;
    for (int r = 0; r < reps; ++r) pass();
    timer_harvest(ctx);
    const int64_t n = tm.count[TIMER_PRECOND] - c0;
    const double per = n > 0 ? (tm.ms[TIMER_PRECOND] - m0) / n : 0.0;
    if (ms) ms[t] = per;
    if (t == 0 || per < tbest) {
      tbest = per;
      arg = t;
    }
  }
  tm.on = was_on;
  for (int q = 0; q < N_TIMERS; ++q) {  // the caller's totals as they were
    tm.ms[q] = ms0[q];
    tm.count[q] = n0[q];
  }
  hipStreamSynchronize(ctx->stream);
  dfree(v);
  dfree(z);
  dv.multi_tiling = arg;
  if (rc == CPM_OK) rc = plan_multi(ctx);
  if (rc != CPM_OK) return rc;
  if (best) *best = arg;
  return CPM_OK;
}

// Implicit steps with resident factors: u_0 = A^{-1} f, u_k = A^{-1}(scale u_{k-1}).
int dev_solve_steps(cpm_ctx* ctx, const double* f, double* u, int nsteps, double scale, double tol, int max_iter,
                    int m, cpm_solve_info* info) {
  HIPCHK(hipSetDevice(ctx->device));
  int rc = ensure_krylov(ctx, m);
  if (rc != CPM_OK) return rc;
  const int64_t na = ctx->band.n_act;
  int worst = CPM_OK;
  for (int k = 0; k < nsteps; ++k) {
    const double* rhs = f;
    if (k > 0) {
      launch(ctx, TIMER_UPDATE, k_scale, dim3(nblk(na, 256)), dim3(256), 0, na, scale, u + (size_t)(k - 1) * na, ctx->dev.F);
      HIPCHK(hipGetLastError());
      rhs = ctx->dev.F;
    }
    cpm_solve_info tmp{};
    rc = dev_solve(ctx, rhs, u + (size_t)k * na, tol, max_iter, m, &tmp);
    if (info) info[k] = tmp;
    if (rc < 0) return rc;
    worst = std::max(worst, rc);
  }
  return worst;
}

template <typename T>
static int selftest_tile(const double* a, const double* b, double* c, int kdim) {
  std::vector<T> ha(GEMM_TILE * LU_KMAX, (T)0), hb(LU_KMAX * GEMM_TILE, (T)0), hc(GEMM_TILE * GEMM_TILE);
  for (int i = 0; i < GEMM_TILE; ++i)
    for (int q = 0; q < kdim; ++q) ha[i * LU_KMAX + q] = (T)a[i * LU_KMAX + q];
  for (int q = 0; q < kdim; ++q)
    for (int jx = 0; jx < GEMM_TILE; ++jx) hb[q * GEMM_TILE + jx] = (T)b[q * GEMM_TILE + jx];
  for (int q = 0; q < GEMM_TILE * GEMM_TILE; ++q) hc[q] = (T)c[q];
  T *da = nullptr, *db = nullptr, *dc = nullptr;
  if (hipMalloc((void**)&da, ha.size() * sizeof(T)) != hipSuccess) return CPM_ENOMEM;
  if (hipMalloc((void**)&db, hb.size() * sizeof(T)) != hipSuccess) { hipFree(da); return CPM_ENOMEM; }
  if (hipMalloc((void**)&dc, hc.size() * sizeof(T)) != hipSuccess) { hipFree(da); hipFree(db); return CPM_ENOMEM; }
  hipMemcpy(da, ha.data(), ha.size() * sizeof(T), hipMemcpyHostToDevice);
  hipMemcpy(db, hb.data(), hb.size() * sizeof(T), hipMemcpyHostToDevice);
  hipMemcpy(dc, hc.data(), hc.size() * sizeof(T), hipMemcpyHostToDevice);
  k_tile_selftest<T><<<1, 256>>>(dc, da, db, kdim);
  hipError_t e = hipDeviceSynchronize();
  hipMemcpy(hc.data(), dc, hc.size() * sizeof(T), hipMemcpyDeviceToHost);
  hipFree(da);
  hipFree(db);
  hipFree(dc);
  if (e != hipSuccess) return CPM_EDEVICE;
  for (int q = 0; q < GEMM_TILE * GEMM_TILE; ++q) c[q] = (double)hc[q];
  return CPM_OK;
}

// Cap of the work-buffer cache (see pool_malloc) and its figures per device.
size_t pool_set_cap(size_t bytes) {
  g_pool_cap.store(bytes);
  size_t before = 0;
  int cur = -1;
  (void)hipGetDevice(&cur);
  for (int d = 0; d < kPoolDevices; ++d) {
    DevPool& pl = g_pool[d];
    std::lock_guard<std::mutex> lk(pl.mu);
    before += pl.idle_bytes;
    if (pl.idle_bytes > bytes) {
      (void)hipSetDevice(d);
      pool_shrink(pl, bytes);
    }
  }
  if (cur >= 0) (void)hipSetDevice(cur);
  return before;
}

void pool_stats(int dev, size_t* cap, size_t* idle, size_t* live) {
  DevPool* pl = pool_of(dev);
  if (cap) *cap = g_pool_cap.load();
  size_t i = 0, l = 0;
  if (pl) {
    std::lock_guard<std::mutex> lk(pl->mu);
    i = pl->idle_bytes;
    for (const auto& kv : pl->live) l += kv.second;
  }
  if (idle) *idle = i;
  if (live) *live = l;
}

}  // namespace cpm

extern "C" int cpm_selftest_tile(int device, int prec, const double* a, const double* b, double* c, int kb) {
  if (!a || !b || !c || kb < 1 || kb > cpm::LU_KMAX) return CPM_EINVAL;
  if (prec != CPM_FP64 && prec != CPM_FP32) return CPM_EINVAL;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return CPM_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return CPM_EDEVICE;
  return prec == CPM_FP64 ? cpm::selftest_tile<double>(a, b, c, kb) : cpm::selftest_tile<float>(a, b, c, kb);
}

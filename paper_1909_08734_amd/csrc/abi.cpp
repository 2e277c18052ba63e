// C ABI of the CPM Schwarz solver: argument checks, call-order state machine,
// error reporting and host queries. Device work lives in device.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "cpm_internal.h"

namespace {

const char* kNull = "null context";

int fail(cpm_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

template <class F>
int guarded(cpm_ctx* ctx, F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(ctx, CPM_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(ctx, CPM_EINVAL, std::string("internal error: ") + e.what());
  } catch (...) {
    return fail(ctx, CPM_EINVAL, "internal error");
  }
}

}  // namespace

extern "C" {

int cpm_create(cpm_ctx** out, int device) {
  if (!out) return CPM_EINVAL;
  *out = nullptr;
  cpm_ctx* ctx = new (std::nothrow) cpm_ctx();
  if (!ctx) return CPM_ENOMEM;
  if (device >= 0) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device >= count) {
      delete ctx;
      return CPM_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess ||
        hipStreamCreateWithFlags(&ctx->own_stream, hipStreamNonBlocking) != hipSuccess) {
      delete ctx;
      return CPM_EDEVICE;
    }
    ctx->stream = ctx->own_stream;
    ctx->device = device;
    ctx->host_only = false;
    if (cpm::dev_init_context(ctx) != CPM_OK) {
      hipStreamDestroy(ctx->own_stream);
      delete ctx;
      return CPM_EDEVICE;
    }
  }
  *out = ctx;
  return CPM_OK;
}

void cpm_destroy(cpm_ctx* ctx) {
  if (!ctx) return;
  if (!ctx->host_only) {
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    cpm::dev_free_all(ctx);
    for (hipEvent_t e : ctx->timer.pool) hipEventDestroy(e);
    hipStreamDestroy(ctx->own_stream);
  }
  delete ctx;
}

int cpm_set_stream(cpm_ctx* ctx, int caller, void* hip_stream) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->host_only) return fail(ctx, CPM_EDEVICE, "set_stream: host-only context");
  hipStream_t next = caller ? (hipStream_t)hip_stream : ctx->own_stream;
  if (next == ctx->stream) return CPM_OK;
  hipSetDevice(ctx->device);
  // Every call returns after its device work has finished, so nothing of the
  // context is pending on the old stream (which other work may still be
  // using: it is not synchronised). The timers' events are read now.
  cpm::timer_harvest(ctx);
  ctx->stream = next;
  cpm::drop_graphs(ctx->dev);
  return CPM_OK;
}

const char* cpm_last_error(const cpm_ctx* ctx) { return ctx ? ctx->err.c_str() : kNull; }

int cpm_build_band(cpm_ctx* ctx, cpm_cp_fn fn, void* user, const double lo[3], const double hi[3],
                   double h, int degree, double band_factor) {
  if (!ctx) return CPM_EINVAL;
  if (!lo || !hi) return fail(ctx, CPM_EINVAL, "build_band: null box");
  return guarded(ctx, [&]() -> int {
    cpm::Band b;
    int rc = cpm::build_band(b, fn, user, lo, hi, h, degree, band_factor, ctx->err);
    if (rc != CPM_OK) return rc;
    // the new operator arrays replace the old device state only once they
    // are all on the device, so a failure leaves the previous band usable
    if (!ctx->host_only && (rc = cpm::dev_upload_operator(ctx, b)) != CPM_OK) return rc;
    ctx->band = std::move(b);
    ctx->dec = cpm::Decomp();
    ctx->c_factor = 0;
    ctx->state = 1;
    return CPM_OK;
  });
}

int cpm_clone(const cpm_ctx* src, int device, cpm_ctx** out) {
  if (!out) return CPM_EINVAL;
  *out = nullptr;
  if (!src) return CPM_EINVAL;
  if (src->state < 1) return CPM_ESTATE;
  cpm_ctx* ctx = nullptr;
  int rc = cpm_create(&ctx, device);
  if (rc != CPM_OK) return rc;
  rc = guarded(ctx, [&]() -> int {
    ctx->band = src->band;
    ctx->dec = src->dec;
    ctx->c = src->c;
    ctx->state = std::min(src->state, 3);
    return ctx->host_only ? CPM_OK : cpm::dev_upload_operator(ctx, ctx->band);
  });
  if (rc != CPM_OK) {
    cpm_destroy(ctx);
    return rc;
  }
  *out = ctx;
  return CPM_OK;
}

int cpm_build_operator(cpm_ctx* ctx, double c) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 1) return fail(ctx, CPM_ESTATE, "build_operator: build the band first");
  if (!(c > 0) || !std::isfinite(c)) return fail(ctx, CPM_EINVAL, "build_operator: c must be positive and finite");
  if (!ctx->host_only) cpm::dev_free_factor(ctx);
  ctx->c = c;
  ctx->c_factor = 0;
  ctx->state = ctx->dec.n_sub > 0 ? 3 : 2;
  return CPM_OK;
}

int cpm_set_operator_c(cpm_ctx* ctx, double c) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 2) return fail(ctx, CPM_ESTATE, "set_operator_c: build the operator first");
  if (!(c > 0) || !std::isfinite(c)) return fail(ctx, CPM_EINVAL, "set_operator_c: c must be positive and finite");
  if (c != ctx->c && !ctx->host_only) cpm::drop_graphs(ctx->dev);  // captured launches hold the diagonal
  ctx->c = c;
  return CPM_OK;
}

double cpm_factor_c(const cpm_ctx* ctx) { return ctx && ctx->state >= 4 ? ctx->c_factor : 0.0; }

int cpm_partition(cpm_ctx* ctx, int method, int n_sub, const double* weights, int overlap, int kind,
                  double alpha, double alpha_cross) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 2) return fail(ctx, CPM_ESTATE, "partition: build the operator first");
  return guarded(ctx, [&]() -> int {
    cpm::Decomp d;
    int rc = cpm::build_decomposition(ctx->band, d, method, n_sub, weights, overlap, kind, alpha,
                                      alpha_cross, ctx->err);
    if (rc != CPM_OK) return rc;
    if (!ctx->host_only) cpm::dev_free_factor(ctx);
    ctx->dec = std::move(d);
    ctx->state = 3;
    return CPM_OK;
  });
}

int cpm_factor(cpm_ctx* ctx, int prec) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 3) return fail(ctx, CPM_ESTATE, "factor: partition first");
  if (prec != CPM_FP64 && prec != CPM_FP32) return fail(ctx, CPM_EINVAL, "factor: precision must be FP64 or FP32");
  if (ctx->host_only) return fail(ctx, CPM_EDEVICE, "factor: host-only context");
  return guarded(ctx, [&]() -> int {
    int rc = cpm::dev_factor(ctx, prec);
    ctx->state = rc == CPM_OK ? 4 : 3;
    ctx->c_factor = rc == CPM_OK ? ctx->c : 0.0;
    return rc;
  });
}

// f and u are device pointers (N_A x nrhs, column-major).
static int solve_common(cpm_ctx* ctx, const double* f, double* u, int nrhs, double tol, int max_iter,
                        int restart, cpm_solve_info* info) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 4) return fail(ctx, CPM_ESTATE, "solve: factor first");
  if (!f || !u) return fail(ctx, CPM_EINVAL, "solve: null vector");
  if (nrhs < 0) return fail(ctx, CPM_EINVAL, "solve: nrhs < 0");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(ctx, CPM_EINVAL, "solve: tol must be positive");
  if (max_iter < 1) return fail(ctx, CPM_EINVAL, "solve: max_iter must be >= 1");
  if (restart < 1 || restart > 64) return fail(ctx, CPM_EINVAL, "solve: restart must be in [1, 64]");
  return guarded(ctx, [&]() -> int {
    const int64_t na = ctx->band.n_act;
    int worst = CPM_OK;
    for (int q = 0; q < nrhs;) {
      // several right-hand sides share each pass over the factors when they fit
      const int nb = cpm::dev_batch_width(ctx, nrhs - q);
      cpm_solve_info tmp[4] = {};
      int rc;
      if (nb >= 2) {
        rc = cpm::dev_solve_batch(ctx, f + (size_t)q * na, u + (size_t)q * na, nb, tol, max_iter, restart, tmp);
      } else {
        rc = cpm::dev_solve(ctx, f + (size_t)q * na, u + (size_t)q * na, tol, max_iter, restart, tmp);
      }
      const int took = nb >= 2 ? nb : 1;
      if (info)
        for (int r = 0; r < took; ++r) info[q + r] = tmp[r];
      if (rc < 0) return rc;
      if (rc > worst) worst = rc;
      q += took;
    }
    return worst;
  });
}

int cpm_solve(cpm_ctx* ctx, const double* f, double* u, int nrhs, double tol, int max_iter, int restart,
              cpm_solve_info* info) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 4) return fail(ctx, CPM_ESTATE, "solve: factor first");
  if (!f || !u) return fail(ctx, CPM_EINVAL, "solve: null vector");
  // Host vectors: stage through device buffers, one RHS at a time.
  const int64_t na = ctx->band.n_act;
  return guarded(ctx, [&]() -> int {
    double *df = nullptr, *du = nullptr;
    if (hipMalloc(&df, na * sizeof(double)) != hipSuccess) return fail(ctx, CPM_ENOMEM, "solve: device allocation failed");
    if (hipMalloc(&du, na * sizeof(double)) != hipSuccess) {
      hipFree(df);
      return fail(ctx, CPM_ENOMEM, "solve: device allocation failed");
    }
    int worst = CPM_OK;
    for (int q = 0; q < nrhs; ++q) {
      hipMemcpyAsync(df, f + (size_t)q * na, na * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
      cpm_solve_info tmp{};
      int rc = solve_common(ctx, df, du, 1, tol, max_iter, restart, &tmp);
      if (rc >= 0) {
        hipMemcpyAsync(u + (size_t)q * na, du, na * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
        hipStreamSynchronize(ctx->stream);
      }
      if (info) info[q] = tmp;
      if (rc < 0) {
        hipFree(df);
        hipFree(du);
        return rc;
      }
      if (rc > worst) worst = rc;
    }
    hipFree(df);
    hipFree(du);
    return worst;
  });
}

int cpm_solve_device(cpm_ctx* ctx, const double* f_dev, double* u_dev, int nrhs, double tol, int max_iter,
                     int restart, cpm_solve_info* info) {
  return solve_common(ctx, f_dev, u_dev, nrhs, tol, max_iter, restart, info);
}

int cpm_solve_steps(cpm_ctx* ctx, const double* f_dev, double* u_dev, int nsteps, double scale, double tol,
                    int max_iter, int restart, cpm_solve_info* info) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 4) return fail(ctx, CPM_ESTATE, "solve_steps: factor first");
  if (!f_dev || !u_dev) return fail(ctx, CPM_EINVAL, "solve_steps: null vector");
  if (nsteps < 0) return fail(ctx, CPM_EINVAL, "solve_steps: nsteps < 0");
  if (!std::isfinite(scale)) return fail(ctx, CPM_EINVAL, "solve_steps: scale must be finite");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(ctx, CPM_EINVAL, "solve_steps: tol must be positive");
  if (max_iter < 1) return fail(ctx, CPM_EINVAL, "solve_steps: max_iter must be >= 1");
  if (restart < 1 || restart > 64) return fail(ctx, CPM_EINVAL, "solve_steps: restart must be in [1, 64]");
  return guarded(ctx, [&]() -> int {
    return cpm::dev_solve_steps(ctx, f_dev, u_dev, nsteps, scale, tol, max_iter, restart, info);
  });
}

int cpm_solve_left(cpm_ctx* ctx, const double* f_dev, double* u_dev, double tol, int max_iter, int restart,
                   cpm_solve_info* info) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 4) return fail(ctx, CPM_ESTATE, "solve_left: factor first");
  if (!f_dev || !u_dev) return fail(ctx, CPM_EINVAL, "solve_left: null vector");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(ctx, CPM_EINVAL, "solve_left: tol must be positive");
  if (max_iter < 1) return fail(ctx, CPM_EINVAL, "solve_left: max_iter must be >= 1");
  if (restart < 1 || restart > 64) return fail(ctx, CPM_EINVAL, "solve_left: restart must be in [1, 64]");
  return guarded(ctx, [&]() -> int {
    cpm_solve_info tmp{};
    const int rc = cpm::dev_solve_left(ctx, f_dev, u_dev, tol, max_iter, restart, &tmp);
    if (info) *info = tmp;
    return rc;
  });
}

int cpm_solve_stationary(cpm_ctx* ctx, const double* f_dev, double* u_dev, double tol, int max_iter,
                         cpm_solve_info* info) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 4) return fail(ctx, CPM_ESTATE, "solve_stationary: factor first");
  if (!f_dev || !u_dev) return fail(ctx, CPM_EINVAL, "solve_stationary: null vector");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(ctx, CPM_EINVAL, "solve_stationary: tol must be positive");
  if (max_iter < 1) return fail(ctx, CPM_EINVAL, "solve_stationary: max_iter must be >= 1");
  return guarded(ctx, [&]() -> int {
    cpm_solve_info tmp{};
    const int rc = cpm::dev_stationary(ctx, f_dev, u_dev, tol, max_iter, &tmp);
    if (info) *info = tmp;
    return rc;
  });
}

int cpm_apply_operator(cpm_ctx* ctx, const double* x_dev, double* y_dev) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 2) return fail(ctx, CPM_ESTATE, "apply_operator: build the operator first");
  if (ctx->host_only) return fail(ctx, CPM_EDEVICE, "apply_operator: host-only context");
  if (!x_dev || !y_dev) return fail(ctx, CPM_EINVAL, "apply_operator: null vector");
  return cpm::dev_apply_operator(ctx, x_dev, y_dev);
}

int cpm_apply_operator_noalloc(cpm_ctx* ctx, const double* x_dev, double* y_dev) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 2) return fail(ctx, CPM_ESTATE, "apply_operator_noalloc: build the operator first");
  if (ctx->host_only) return fail(ctx, CPM_EDEVICE, "apply_operator_noalloc: host-only context");
  if (!x_dev || !y_dev) return fail(ctx, CPM_EINVAL, "apply_operator_noalloc: null vector");
  return cpm::dev_apply_operator_noalloc(ctx, x_dev, y_dev);
}

int cpm_apply_precond(cpm_ctx* ctx, const double* v_dev, double* z_dev) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 4) return fail(ctx, CPM_ESTATE, "apply_precond: factor first");
  if (!v_dev || !z_dev) return fail(ctx, CPM_EINVAL, "apply_precond: null vector");
  return cpm::dev_apply_precond(ctx, v_dev, z_dev);
}

int cpm_band_sizes(const cpm_ctx* ctx, int64_t* n_act, int64_t* n_ghost, int64_t shape[3]) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 1) return CPM_ESTATE;
  if (n_act) *n_act = ctx->band.n_act;
  if (n_ghost) *n_ghost = ctx->band.n_ghost;
  if (shape)
    for (int a = 0; a < 3; ++a) shape[a] = ctx->band.n[a];
  return CPM_OK;
}

int cpm_band_arrays(const cpm_ctx* ctx, int64_t* lin, double* cp, double* nrm, int32_t* nbr, int32_t* base,
                    double* wts) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 1) return CPM_ESTATE;
  const cpm::Band& b = ctx->band;
  if (lin) std::memcpy(lin, b.lin.data(), b.lin.size() * sizeof(int64_t));
  if (cp) std::memcpy(cp, b.cp.data(), b.cp.size() * sizeof(double));
  if (nrm) std::memcpy(nrm, b.nrm.data(), b.nrm.size() * sizeof(double));
  if (nbr) std::memcpy(nbr, b.nbr.data(), b.nbr.size() * sizeof(int32_t));
  if (base) std::memcpy(base, b.base.data(), b.base.size() * sizeof(int32_t));
  if (wts) std::memcpy(wts, b.wts.data(), b.wts.size() * sizeof(double));
  return CPM_OK;
}

int cpm_partition_info(const cpm_ctx* ctx, int* n_sub, int32_t* part, uint8_t* cross) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 3) return CPM_ESTATE;
  if (n_sub) *n_sub = ctx->dec.n_sub;
  if (part) std::memcpy(part, ctx->dec.part.data(), ctx->dec.part.size() * sizeof(int32_t));
  if (cross) std::memcpy(cross, ctx->dec.cross.data(), ctx->dec.cross.size());
  return CPM_OK;
}

int cpm_subdomain_sizes(const cpm_ctx* ctx, int j, int64_t sizes[5]) {
  if (!ctx || !sizes) return CPM_EINVAL;
  if (ctx->state < 3) return CPM_ESTATE;
  if (j < 0 || j >= ctx->dec.n_sub) return CPM_EINVAL;
  const cpm::Sub& s = ctx->dec.subs[j];
  sizes[0] = (int64_t)s.tilde.size();
  sizes[1] = (int64_t)s.sigma.size();
  sizes[2] = (int64_t)s.fin.size();
  sizes[3] = (int64_t)s.ghost.size();
  sizes[4] = (int64_t)s.bnd.size();
  return CPM_OK;
}

int cpm_subdomain_sets(const cpm_ctx* ctx, int j, int32_t* tilde, int32_t* sigma, int32_t* fin,
                       int32_t* ghost, int32_t* bnd, int32_t* xstar, double* s, double* alpha) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 3) return CPM_ESTATE;
  if (j < 0 || j >= ctx->dec.n_sub) return CPM_EINVAL;
  const cpm::Sub& d = ctx->dec.subs[j];
  auto cp32 = [](int32_t* dst, const std::vector<int32_t>& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(int32_t));
  };
  cp32(tilde, d.tilde);
  cp32(sigma, d.sigma);
  cp32(fin, d.fin);
  cp32(ghost, d.ghost);
  cp32(bnd, d.bnd);
  cp32(xstar, d.xstar);
  if (s && !d.s.empty()) std::memcpy(s, d.s.data(), d.s.size() * sizeof(double));
  if (alpha && !d.alpha.empty()) std::memcpy(alpha, d.alpha.data(), d.alpha.size() * sizeof(double));
  return CPM_OK;
}

int cpm_subdomain_order(const cpm_ctx* ctx, int j, int64_t* n_unk, int32_t* order) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 3) return CPM_ESTATE;
  if (j < 0 || j >= ctx->dec.n_sub) return CPM_EINVAL;
  const std::vector<int32_t>& o = ctx->dec.subs[j].order;
  if (n_unk) *n_unk = (int64_t)o.size();
  if (order && !o.empty()) std::memcpy(order, o.data(), o.size() * sizeof(int32_t));
  return CPM_OK;
}

int cpm_factor_export(cpm_ctx* ctx, int j, double* w) {
  if (!ctx || !w) return CPM_EINVAL;
  if (ctx->state < 4) return fail(ctx, CPM_ESTATE, "factor_export: factor first");
  if (j < 0 || j >= ctx->dec.n_sub) return fail(ctx, CPM_EINVAL, "factor_export: bad subdomain");
  return guarded(ctx, [&]() -> int { return cpm::dev_export_w(ctx, j, w); });
}

size_t cpm_footprint_bytes(const cpm_ctx* ctx) {
  if (!ctx) return 0;
  return ctx->dev.op_bytes + ctx->dev.w_bytes + ctx->dev.krylov_bytes;
}

int cpm_footprint_estimate(const cpm_ctx* ctx, int prec, int restart, size_t* resident, size_t* peak) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 3) return CPM_ESTATE;
  if (prec != CPM_FP64 && prec != CPM_FP32) return CPM_EINVAL;
  if (restart < 0 || restart > 64) return CPM_EINVAL;
  cpm::dev_estimate(ctx, prec, restart, resident, peak);
  return CPM_OK;
}

int cpm_set_workspace_cache(size_t bytes, size_t* idle_before) {
  const size_t before = cpm::pool_set_cap(bytes);
  if (idle_before) *idle_before = before;
  return CPM_OK;
}

int cpm_workspace_cache(int device, size_t* cap, size_t* idle, size_t* in_use) {
  if (device < 0) return CPM_EINVAL;
  cpm::pool_stats(device, cap, idle, in_use);
  return CPM_OK;
}

int cpm_set_factor_workspace(cpm_ctx* ctx, size_t bytes) {
  if (!ctx) return CPM_EINVAL;
  ctx->dev.ws_limit = bytes ? bytes : (size_t(64) << 30);
  return CPM_OK;
}

int cpm_factor_groups(const cpm_ctx* ctx) { return ctx ? ctx->dev.n_groups : 0; }

int cpm_set_precond_chunk(cpm_ctx* ctx, int columns) {
  if (!ctx) return CPM_EINVAL;
  if (columns < 0 || columns > 16384 || columns % 8 != 0)
    return fail(ctx, CPM_EINVAL, "set_precond_chunk: columns must be 0 or a multiple of 8 up to 16384");
  ctx->dev.chunk_req = columns;
  return CPM_OK;
}

int cpm_precond_chunk(const cpm_ctx* ctx) { return ctx ? ctx->dev.chunk : 0; }

int cpm_set_precond_tiling(cpm_ctx* ctx, int tiling) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 4) return fail(ctx, CPM_ESTATE, "set_precond_tiling: factor first");
  return guarded(ctx, [&]() -> int { return cpm::dev_set_tiling(ctx, tiling); });
}

int cpm_precond_tiling(const cpm_ctx* ctx) { return ctx ? ctx->dev.tiling : 0; }

int cpm_set_factor_tile(cpm_ctx* ctx, int rows) {
  if (!ctx) return CPM_EINVAL;
  if (rows != 0 && rows != 64 && rows != 128) return fail(ctx, CPM_EINVAL, "set_factor_tile: rows must be 0, 64 or 128");
  ctx->dev.factor_tile = rows;
  return CPM_OK;
}

int cpm_factor_tile(const cpm_ctx* ctx) { return ctx && ctx->state >= 4 ? ctx->dev.factor_tile_used : 0; }

int cpm_factor_flops(const cpm_ctx* ctx, double* flops) {
  if (!ctx || !flops) return CPM_EINVAL;
  if (ctx->state < 4) return CPM_ESTATE;
  *flops = ctx->dev.factor_flops;
  return CPM_OK;
}

int cpm_autotune_factor(cpm_ctx* ctx, int prec, int* best, double* ms) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 3) return fail(ctx, CPM_ESTATE, "autotune_factor: partition first");
  if (prec != CPM_FP64 && prec != CPM_FP32) return fail(ctx, CPM_EINVAL, "autotune_factor: precision must be FP64 or FP32");
  if (ctx->host_only) return fail(ctx, CPM_EDEVICE, "autotune_factor: host-only context");
  return guarded(ctx, [&]() -> int {
    const int rc = cpm::dev_autotune_factor(ctx, prec, best, ms);
    ctx->state = rc == CPM_OK ? 4 : 3;
    ctx->c_factor = rc == CPM_OK ? ctx->c : 0.0;
    return rc;
  });
}

int cpm_set_multi_tiling(cpm_ctx* ctx, int tiling) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 4) return fail(ctx, CPM_ESTATE, "set_multi_tiling: factor first");
  return guarded(ctx, [&]() -> int { return cpm::dev_set_multi_tiling(ctx, tiling); });
}

int cpm_multi_tiling(const cpm_ctx* ctx) { return ctx ? ctx->dev.multi_tiling : 0; }

int cpm_autotune_multi(cpm_ctx* ctx, int reps, int* best, double* ms) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 4) return fail(ctx, CPM_ESTATE, "autotune_multi: factor first");
  if (reps < 1) return fail(ctx, CPM_EINVAL, "autotune_multi: reps must be >= 1");
  return guarded(ctx, [&]() -> int { return cpm::dev_autotune_multi(ctx, reps, best, ms); });
}

int cpm_set_operator_kernel(cpm_ctx* ctx, int kernel) {
  if (!ctx) return CPM_EINVAL;
  return cpm::dev_set_operator_kernel(ctx, kernel);
}

int cpm_operator_kernel(const cpm_ctx* ctx) {
  if (!ctx) return -1;
  const cpm::Dev& d = ctx->dev;
  if (d.op_kernel == 1 && !(d.n_ext_groups > 0 && d.ext_lds <= 64 * 1024)) return 2;  // falls back to gathers
  if (d.op_kernel == 0 && !d.compact) return 2;
  return d.op_kernel;
}

int cpm_set_graphs(cpm_ctx* ctx, int on) {
  if (!ctx) return CPM_EINVAL;
  ctx->dev.use_graphs = on != 0;
  if (!ctx->host_only) cpm::drop_graphs(ctx->dev);
  return CPM_OK;
}

int cpm_autotune_precond(cpm_ctx* ctx, int reps, int* best, double* ms) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->state < 4) return fail(ctx, CPM_ESTATE, "autotune_precond: factor first");
  if (reps < 1) return fail(ctx, CPM_EINVAL, "autotune_precond: reps must be >= 1");
  return guarded(ctx, [&]() -> int { return cpm::dev_autotune(ctx, reps, best, ms); });
}

int cpm_set_timing(cpm_ctx* ctx, int on) {
  if (!ctx) return CPM_EINVAL;
  if (ctx->host_only) return fail(ctx, CPM_EDEVICE, "set_timing: host-only context");
  cpm::timer_harvest(ctx);
  ctx->timer.on = on != 0;
  for (int q = 0; q < cpm::N_TIMERS; ++q) {
    ctx->timer.ms[q] = 0;
    ctx->timer.count[q] = 0;
  }
  return CPM_OK;
}

int cpm_kernel_time(cpm_ctx* ctx, int which, double* total_ms, int64_t* launches) {
  if (!ctx) return CPM_EINVAL;
  if (which < 0 || which >= cpm::N_TIMERS) return fail(ctx, CPM_EINVAL, "kernel_time: unknown kernel");
  if (!ctx->host_only) cpm::timer_harvest(ctx);
  if (total_ms) *total_ms = ctx->timer.ms[which];
  if (launches) *launches = ctx->timer.count[which];
  return CPM_OK;
}

}  // extern "C"

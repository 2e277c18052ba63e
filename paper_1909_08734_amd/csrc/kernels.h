// HIP kernels for gfx950 (wave64). Included once, by device.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cpm_internal.h"

namespace cpm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One step of wave_sum_many (lane offset O, N values left), then the rest.
template <int N, int O, int K>
__device__ __forceinline__ void wave_sum_step(double (&v)[K], int lane) {
  if constexpr (O > 0) {
    if constexpr (N > 1) {
      const bool hi = (lane & O) != 0;
#pragma unroll
      for (int k = 0; k < N / 2; ++k) {
        const double send = hi ? v[k] : v[k + N / 2];
        const double keep = hi ? v[k + N / 2] : v[k];
        v[k] = keep + __shfl_xor(send, O, 64);
      }
      wave_sum_step<N / 2, O / 2, K>(v, lane);
    } else {
      v[0] += __shfl_xor(v[0], O, 64);
      wave_sum_step<1, O / 2, K>(v, lane);
    }
  }
}

// Wave sums of K values per lane (K a power of two up to 64) with wave_sum's
// pairing: at each step o = 32, 16, ..., 1 the partial sums of lanes l and
// l ^ o are added, so every result equals wave_sum of that value bit for bit
// (addition is commutative). Instead of reducing each value whole, a step
// while more than one value is left splits them between the two lanes of a
// pair (the lane with bit o set keeps the upper half), so the K sums take
// K - 1 + (6 - log2 K) exchanges instead of 6 K. On return lane l holds the
// sum of value l >> (6 - log2 K), as do the other lanes of its group of
// 2^(6 - log2 K). v is consumed.
template <int K>
__device__ __forceinline__ double wave_sum_many(double (&v)[K], int lane) {
  static_assert(K >= 1 && K <= 64 && (K & (K - 1)) == 0, "K: a power of two up to 64");
  wave_sum_step<K, 32, K>(v, lane);
  return v[0];
}

constexpr int ilog2(int k) { return k <= 1 ? 0 : 1 + ilog2(k / 2); }

// Sum of one value per thread over a 256-thread block (fixed order).
__device__ __forceinline__ double block_sum256(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// ---------------------------------------------------------------------------
// Operator apply (Section 2.1): e = E x over all band rows, then
// y = (c + 6/h^2) x - (1/h^2) sum_{6 neighbours} e.
// The extension rows are stored in apply order (grouped by the grid position
// of their interpolation stencil, see ExtGroup); perm[q] is the band row of
// apply position q, and e is written in band order.
//
// Blocks are mapped to work XCD by XCD: the hardware hands consecutive block
// indices to the eight XCDs in turn, so block b runs work item
// xcd_item(b, n), which gives each XCD one contiguous eighth of the items and
// keeps the x values its L2 serves to that eighth of the band.
// ---------------------------------------------------------------------------
constexpr int N_XCD = 8;
__device__ __forceinline__ int xcd_item(int b, int n) {
  const int q = n / N_XCD, r = n % N_XCD, x = b % N_XCD;
  return x * q + min(x, r) + b / N_XCD;
}

// One row's extension value from z-line starts s (P1 x P1) and its weights w
// (3 x P1: x, y, z), x read through rd(index). Sum order: per plane a,
// sum_b wy[b] (sum_c wz[c] x), then w[a] times that; planes (0,1) and (2,3)
// summed apart and added, as the two-lane form does.
template <int P, class RD>
__device__ __forceinline__ double ext_plane(const double* __restrict__ w, const int32_t* s, RD rd) {
  constexpr int P1 = P + 1;
  double pa = 0.0;
#pragma unroll
  for (int b = 0; b < P1; ++b) {
    double lz = 0.0;
#pragma unroll
    for (int c = 0; c < P1; ++c) lz += w[2 * P1 + c] * rd(s[b] + c);
    pa += w[P1 + b] * lz;
  }
  return pa;
}

// The same sum with each z-line's p+1 values read as 16-byte loads from its
// 8-byte aligned start (half the load instructions of single values).
typedef double d2u __attribute__((ext_vector_type(2))) __attribute__((aligned(8)));
template <int P>
__device__ __forceinline__ double ext_plane_vec(const double* __restrict__ w, const int32_t* s,
                                                const double* __restrict__ x) {
  constexpr int P1 = P + 1;
  double v[P1][P1];
#pragma unroll
  for (int b = 0; b < P1; ++b) {
    const d2u a0 = *reinterpret_cast<const d2u*>(x + s[b]);
    v[b][0] = a0.x;
    v[b][1] = a0.y;
    if constexpr (P1 == 4) {
      const d2u a1 = *reinterpret_cast<const d2u*>(x + s[b] + 2);
      v[b][2] = a1.x;
      v[b][3] = a1.y;
    } else {
      v[b][2] = x[s[b] + 2];
    }
  }
  double pa = 0.0;
#pragma unroll
  for (int b = 0; b < P1; ++b) {
    double lz = 0.0;
#pragma unroll
    for (int c = 0; c < P1; ++c) lz += w[2 * P1 + c] * v[b][c];
    pa += w[P1 + b] * lz;
  }
  return pa;
}

// Row data layout (apply order q, N_T rows): weights as structure of arrays,
// wts[c * n + q] for c < 3(p+1) (x, y, z weights), z-line starts
// lines[l * n + q] for l = a (p+1) + b < (p+1)^2, so that the lanes of a wave,
// one row each, read every component of their rows with one coalesced load.
// Extension by gathers from device memory, one lane per row.
template <int P>
__global__ __launch_bounds__(256) void k_extend(int64_t n_rows, const int32_t* __restrict__ lines,
                                                const double* __restrict__ wts, const int32_t* __restrict__ perm,
                                                const double* __restrict__ x, double* __restrict__ e,
                                                int64_t x_stride, int64_t e_stride) {
  constexpr int P1 = P + 1, NW = 3 * P1;
  x += blockIdx.y * x_stride;  // right-hand side blockIdx.y of a batch
  e += blockIdx.y * e_stride;
  const int64_t row = (int64_t)xcd_item(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (row >= n_rows) return;
  double wl[NW];
#pragma unroll
  for (int c = 0; c < NW; ++c) wl[c] = wts[c * n_rows + row];
  double half[2] = {0.0, 0.0};
#pragma unroll
  for (int a = 0; a < P1; ++a) {
    int32_t s[P1];
#pragma unroll
    for (int b = 0; b < P1; ++b) s[b] = lines[(a * P1 + b) * n_rows + row];
    half[a >> 1] += wl[a] * ext_plane_vec<P>(wl, s, x);
  }
  e[perm[row]] = half[0] + half[1];
}

// Lagrange basis on the nodes 0..P at s: l_m(s) = prod_{q != m} (s - q) /
// prod_{q != m} (m - q), the products formed in q order and the denominator
// exact, as the host set-up forms the stored weights (so both agree bit for
// bit).
// A denominator that is a power of two (+-1, +-2) divides exactly as a
// product with its reciprocal; the others (+-6 for p = 3) are divided.
constexpr int lagrange_den(int p, int m) {
  int d = 1;
  for (int q = 0; q <= p; ++q)
    if (q != m) d *= m - q;
  return d;
}
constexpr bool power_of_two(int v) { return v > 0 && (v & (v - 1)) == 0; }

template <int P>
__device__ __forceinline__ void lagrange_basis(double s, double* w) {
#pragma clang fp contract(off)
#pragma unroll
  for (int m = 0; m <= P; ++m) {
    double num = 1.0;
#pragma unroll
    for (int q = 0; q <= P; ++q) {
      if (q == m) continue;
      num *= (s - (double)q);
    }
    constexpr int dd[4] = {lagrange_den(P, 0), lagrange_den(P, 1), lagrange_den(P, 2), P >= 3 ? lagrange_den(P, 3) : 1};
    const int den = dd[m];
    if (power_of_two(den < 0 ? -den : den))
      w[m] = num * (1.0 / (double)den);
    else
      w[m] = num / (double)den;
  }
}

// Extension from the compact row form: per row the local stencil coordinates
// s (3 doubles; the weights are the Lagrange basis at s, formed here) and the
// z-line starts as the first start of each stencil plane (int32) plus the
// p increments to the next columns' starts (uint16): 64 bytes a row for
// p = 3 instead of 160. Same sums in the same order as k_extend.
template <int P>
__global__ __launch_bounds__(256) void k_extend_compact(int64_t n_rows, const double* __restrict__ sloc,
                                                        const int32_t* __restrict__ starts,
                                                        const uint16_t* __restrict__ steps,
                                                        const int32_t* __restrict__ perm,
                                                        const double* __restrict__ x, double* __restrict__ e,
                                                        int64_t x_stride, int64_t e_stride) {
  constexpr int P1 = P + 1, NW = 3 * P1;
  x += blockIdx.y * x_stride;
  e += blockIdx.y * e_stride;
  const int64_t row = (int64_t)xcd_item(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (row >= n_rows) return;
  double sl[3];
  int32_t st[P1];
  uint16_t dz[P1 * P];
#pragma unroll
  for (int a = 0; a < 3; ++a) sl[a] = sloc[a * n_rows + row];
#pragma unroll
  for (int a = 0; a < P1; ++a) st[a] = starts[a * n_rows + row];
#pragma unroll
  for (int q = 0; q < P1 * P; ++q) dz[q] = steps[q * n_rows + row];
  double wl[NW];
#pragma unroll
  for (int a = 0; a < 3; ++a) lagrange_basis<P>(sl[a], wl + a * P1);
  double half[2] = {0.0, 0.0};
#pragma unroll
  for (int a = 0; a < P1; ++a) {
    int32_t s[P1];
    s[0] = st[a];
#pragma unroll
    for (int b = 1; b < P1; ++b) s[b] = s[b - 1] + (int32_t)dz[a * P + b - 1];
    half[a >> 1] += wl[a] * ext_plane_vec<P>(wl, s, x);
  }
  e[perm[row]] = half[0] + half[1];
}

// Extension with x staged in LDS: block b serves ExtGroup xcd_item(b, n); the
// group's P+1 intervals of x (contiguous band indices, one per stencil plane)
// are copied to LDS with coalesced loads, then each row (one lane) reads its
// (P+1)^3 stencil values from LDS. Same sums in the same order as k_extend.
template <int P>
__global__ __launch_bounds__(256) void k_extend_lds(const ExtGroup* __restrict__ groups, int64_t n_rows,
                                                    const int32_t* __restrict__ lines,
                                                    const double* __restrict__ wts,
                                                    const int32_t* __restrict__ perm,
                                                    const double* __restrict__ x, double* __restrict__ e,
                                                    int64_t x_stride, int64_t e_stride) {
  constexpr int P1 = P + 1, NW = 3 * P1;
  extern __shared__ double xs[];
  x += blockIdx.y * x_stride;
  e += blockIdx.y * e_stride;
  const ExtGroup g = groups[xcd_item(blockIdx.x, gridDim.x)];
#pragma unroll
  for (int a = 0; a < P1; ++a) {
    const double* src = x + g.lo[a];
    double* dst = xs + g.off[a];
    const int len = g.off[a + 1] - g.off[a];
    for (int q = threadIdx.x; q < len; q += blockDim.x) dst[q] = src[q];
  }
  __syncthreads();
  for (int r = threadIdx.x; r < g.nrows; r += blockDim.x) {
    const int64_t row = (int64_t)g.row0 + r;
    double wl[NW];
#pragma unroll
    for (int c = 0; c < NW; ++c) wl[c] = wts[c * n_rows + row];
    double half[2] = {0.0, 0.0};
#pragma unroll
    for (int a = 0; a < P1; ++a) {
      int32_t s[P1];
#pragma unroll
      for (int b = 0; b < P1; ++b) s[b] = lines[(a * P1 + b) * n_rows + row] - g.lo[a] + g.off[a];
      half[a >> 1] += wl[a] * ext_plane<P>(wl, s, [&](int32_t i) { return xs[i]; });
    }
    e[perm[row]] = half[0] + half[1];
  }
}

// y = diag x - ih2 * sum_nb e[nb]           (f == nullptr)
// y = f - (diag x - ih2 * sum_nb e[nb])     (residual form)
__global__ __launch_bounds__(256) void k_stencil(int64_t na, double diag, double ih2,
                                                 const int32_t* __restrict__ nbr,
                                                 const double* __restrict__ x,
                                                 const double* __restrict__ e,
                                                 const double* __restrict__ f, double* __restrict__ y) {
  const int64_t i = (int64_t)xcd_item(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= na) return;
  const double s = (e[nbr[i]] + e[nbr[na + i]]) + (e[nbr[2 * na + i]] + e[nbr[3 * na + i]]) +
                   (e[nbr[4 * na + i]] + e[nbr[5 * na + i]]);
  const double v = diag * x[i] - ih2 * s;
  y[i] = f ? f[i] - v : v;
}

// ---------------------------------------------------------------------------
// Preconditioner apply (eq. algRAS): for every subdomain j and row q of
// Sigma~_j, z[tilde_j(q)] = sum_c W_j[q, c] v[sigma_j(c)]. One block per
// (subdomain, group of rows); v|Sigma_j is gathered into LDS once per block,
// W streams from HBM with 16-byte loads; each row is written once.
//
// Layout of W_j (ldw = |Sigma_j| rounded up to 8 columns, the padding zero):
// rows in tiles of W_TILE, the last tile padded; inside a tile the columns in
// chunks of W_CW<T> = 64 lanes x 16 bytes (128 FP64 / 256 FP32 values), each
// chunk stored as W_TILE rows of W_CW values one after another, the last
// chunk ragged (W_TILE rows of ldw mod W_CW). A block's waves, streaming the
// tile's rows chunk by chunk, then read one contiguous stretch of memory per
// step instead of one short piece of each of many rows.
// ---------------------------------------------------------------------------
template <typename T>
struct VecOf;
template <>
struct VecOf<double> {
  typedef d2v type;
  static constexpr int n = 2;
  static constexpr int unroll = 2;  // 16-byte chunks in flight per row and lane
};
template <>
struct VecOf<float> {
  typedef f4 type;
  static constexpr int n = 4;
  static constexpr int unroll = 2;
};

constexpr int PRECOND_THREADS = 512;  // 8 waves per block
constexpr int W_TILE = 8;             // rows per tile of W_j (a multiple of every tiling's rows per wave)
template <typename T>
constexpr int W_CW = 64 * VecOf<T>::n;  // columns per chunk

// Element offset of W_j[r, c] from the start of W_j (cw = W_CW<T>).
__host__ __device__ inline int64_t w_tile_index(int ldw, int cw, int r, int c) {
  const int R = r / W_TILE * W_TILE, i = r - R;
  const int nfull = ldw / cw, k = c / cw;
  const int64_t tile = (int64_t)R * ldw;
  if (k < nfull) return tile + (int64_t)k * W_TILE * cw + (int64_t)i * cw + (c - k * cw);
  const int wk = ldw - nfull * cw;
  return tile + (int64_t)nfull * W_TILE * cw + (int64_t)i * wk + (c - nfull * cw);
}
// Rows of W_j as stored (t rounded up to whole tiles).
__host__ __device__ inline int64_t w_rows_stored(int t) { return (int64_t)(t + W_TILE - 1) / W_TILE * W_TILE; }

// vs[c] = sc * v[sigma_j(c)] for c < m, 0 for m <= c < ldw. The index loads
// of PRECOND_GATHER columns are issued together, then their gathers (an index
// past m reads entry 0 of the list, whose value is discarded), so a block
// starts streaming W after two round trips to memory rather than two per
// column group.
constexpr int PRECOND_GATHER = 8;
// (si: the index list from the first staged column; m >= 1 entries of it are
// real, ncols columns are staged.)
__device__ __forceinline__ void gather_v(const int32_t* __restrict__ si, int m, int ncols,
                                         const double* __restrict__ v, double sc, double* __restrict__ vs) {
  for (int c0 = threadIdx.x; c0 < ncols; c0 += PRECOND_GATHER * PRECOND_THREADS) {
    int32_t g[PRECOND_GATHER];
    double x[PRECOND_GATHER];
#pragma unroll
    for (int u = 0; u < PRECOND_GATHER; ++u) {
      const int c = c0 + u * PRECOND_THREADS;
      g[u] = si[c < m ? c : 0];
    }
#pragma unroll
    for (int u = 0; u < PRECOND_GATHER; ++u) x[u] = v[g[u]];
#pragma unroll
    for (int u = 0; u < PRECOND_GATHER; ++u) {
      const int c = c0 + u * PRECOND_THREADS;
      if (c < ncols) vs[c] = c < m ? sc * x[u] : 0.0;
    }
  }
}

// Block b serves rows [(b - blk_off) rpb, ...) of subdomain blk_sub[b] (rpb a
// multiple of W_TILE); the host sizes rpb so that every block streams about
// the same number of bytes. RPW rows per wave and UNR chunks in flight per
// row are the tunable tiling; every tiling forms each row's sum over the same
// columns in the same order (lane l: columns l VN + k W_CW, k ascending, then
// the ragged chunk), so all give bit-identical results.
// Waves per SIMD a tiling is compiled for (its register budget, no spills):
// 4 rows per wave need more than the 64 registers of 8 waves, 8 loads in
// flight more than the 80 of 6, 16 more than the 128 of 4.
constexpr int precond_waves(int rpw, int unr) {
  return rpw * unr >= 16 ? 3 : rpw * unr >= 8 ? 4 : rpw >= 4 ? 6 : 8;
}

template <typename T, int RPW, int UNR>
__global__ __launch_bounds__(PRECOND_THREADS, precond_waves(RPW, UNR)) void k_precond(const SubDesc* __restrict__ desc,
                                                             const int32_t* __restrict__ blk_sub,
                                                             const int32_t* __restrict__ sig_idx,
                                                             const int32_t* __restrict__ tilde_idx,
                                                             const T* __restrict__ W,
                                                             const double* __restrict__ v,
                                                             const double* __restrict__ scale,
                                                             double* __restrict__ z) {
  extern __shared__ double vs[];
  typedef typename VecOf<T>::type VT;
  constexpr int VN = VecOf<T>::n;
  constexpr int CW = W_CW<T>;
  constexpr int64_t KS = (int64_t)W_TILE * CW;  // stride between chunks of one row
  constexpr int NWAVE = PRECOND_THREADS / 64;
  const int blk = blockIdx.x;
  const int j = blk_sub[blk];
  const SubDesc d = desc[j];
  const double sc = scale ? *scale : 1.0;  // z = sc * M^{-1} v (M^{-1} is linear)
  gather_v(sig_idx + d.u_off, d.m, d.ldw, v, sc, vs);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r_begin = (blk - d.blk_off) * d.rpb;
  const int r_end = min(r_begin + d.rpb, d.t);
  const int nfull = d.ldw / CW, wk = d.ldw - nfull * CW;
  const double* vl = vs + lane * VN;
  for (int r0 = r_begin + wave * RPW; r0 < r_end; r0 += NWAVE * RPW) {
    // rows r0 .. r0 + RPW - 1 (the last clamped to r_end - 1) lie in one tile
    const int R = r0 / W_TILE * W_TILE;
    const T* wf = W + d.w_off + (int64_t)R * d.ldw + (r0 - R) * CW + lane * VN;  // chunk 0, row r0
    int ro[RPW];                                                                   // row offsets in a chunk
    double acc[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      ro[i] = min(i, r_end - 1 - r0);
      acc[i] = 0.0;
    }
    int k = 0;
#pragma unroll 1
    for (; k + UNR <= nfull; k += UNR) {
      VT wv[UNR][RPW];
#pragma unroll
      for (int u = 0; u < UNR; ++u)
#pragma unroll
        for (int i = 0; i < RPW; ++i)
          wv[u][i] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(wf + (k + u) * KS + ro[i] * CW));
#pragma unroll
      for (int u = 0; u < UNR; ++u)
#pragma unroll
        for (int e = 0; e < VN; ++e) {
          const double xv = vl[(k + u) * CW + e];
#pragma unroll
          for (int i = 0; i < RPW; ++i) acc[i] += (double)wv[u][i][e] * xv;
        }
    }
#pragma unroll 1
    for (; k < nfull; ++k) {
      VT wv[RPW];
#pragma unroll
      for (int i = 0; i < RPW; ++i)
        wv[i] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(wf + k * KS + ro[i] * CW));
#pragma unroll
      for (int e = 0; e < VN; ++e) {
        const double xv = vl[k * CW + e];
#pragma unroll
        for (int i = 0; i < RPW; ++i) acc[i] += (double)wv[i][e] * xv;
      }
    }
    if (lane * VN < wk) {
      // ragged chunk: rows of wk values
      const T* wt = W + d.w_off + (int64_t)R * d.ldw + nfull * KS + (r0 - R) * wk + lane * VN;
      VT wv[RPW];
#pragma unroll
      for (int i = 0; i < RPW; ++i) wv[i] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(wt + ro[i] * wk));
#pragma unroll
      for (int e = 0; e < VN; ++e) {
        const double xv = vl[nfull * CW + e];
#pragma unroll
        for (int i = 0; i < RPW; ++i) acc[i] += (double)wv[i][e] * xv;
      }
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const double s = wave_sum(acc[i]);
      if (lane == 0 && r0 + i < r_end) z[tilde_idx[d.t_off + r0 + i]] = s;
    }
  }
}

// Chunked form, for subdomains whose v|Sigma_j does not fit in LDS: v is
// staged `chunk` columns at a time and each row's partial sums are kept in LDS
// (at most PRECOND_RPB_MAX rows per block), then the rows are written once.
constexpr int PRECOND_CHUNK = 4096;     // columns of v per pass (default)
constexpr int PRECOND_RPB_MAX = 1024;   // rows per block in the chunked form
constexpr int CHUNKED_RPW = 2;

template <typename T>
__global__ __launch_bounds__(PRECOND_THREADS, 8) void k_precond_chunked(const SubDesc* __restrict__ desc,
                                                                     const int32_t* __restrict__ blk_sub,
                                                                     const int32_t* __restrict__ sig_idx,
                                                                     const int32_t* __restrict__ tilde_idx,
                                                                     const T* __restrict__ W,
                                                                     const double* __restrict__ v,
                                                                     const double* __restrict__ scale,
                                                                     double* __restrict__ z, int chunk) {
  extern __shared__ double lds[];
  double* vs = lds;          // chunk columns of v|Sigma_j
  double* ps = lds + chunk;  // partial sums of the block's rows
  typedef typename VecOf<T>::type VT;
  constexpr int VN = VecOf<T>::n;
  constexpr int CW = W_CW<T>;
  constexpr int NWAVE = PRECOND_THREADS / 64;
  const int blk = blockIdx.x;
  const int j = blk_sub[blk];
  const SubDesc d = desc[j];
  const double sc = scale ? *scale : 1.0;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r_begin = (blk - d.blk_off) * d.rpb;
  const int r_end = min(r_begin + d.rpb, d.t);
  const T* Wj = W + d.w_off;
  for (int q = threadIdx.x; q < r_end - r_begin; q += PRECOND_THREADS) ps[q] = 0.0;
  for (int c0 = 0; c0 < d.ldw; c0 += chunk) {
    const int cw = min(chunk, d.ldw - c0);
    __syncthreads();  // the previous chunk is consumed
    gather_v(sig_idx + d.u_off + c0, d.m - c0, cw, v, sc, vs);  // c0 < m: ldw - m < 8 <= chunk
    __syncthreads();
    for (int r0 = r_begin + wave * CHUNKED_RPW; r0 < r_end; r0 += NWAVE * CHUNKED_RPW) {
      int rr[CHUNKED_RPW];
      double acc[CHUNKED_RPW];
#pragma unroll
      for (int i = 0; i < CHUNKED_RPW; ++i) {
        rr[i] = min(r0 + i, r_end - 1);
        acc[i] = 0.0;
      }
      for (int c = lane * VN; c < cw; c += 64 * VN) {
        VT wv[CHUNKED_RPW];
#pragma unroll
        for (int i = 0; i < CHUNKED_RPW; ++i)
          wv[i] = __builtin_nontemporal_load(
              reinterpret_cast<const VT*>(Wj + w_tile_index(d.ldw, CW, rr[i], c0 + c)));
#pragma unroll
        for (int e = 0; e < VN; ++e) {
          const double xv = vs[c + e];
#pragma unroll
          for (int i = 0; i < CHUNKED_RPW; ++i) acc[i] += (double)wv[i][e] * xv;
        }
      }
#pragma unroll
      for (int i = 0; i < CHUNKED_RPW; ++i) {
        const double s = wave_sum(acc[i]);
        if (lane == 0 && r0 + i < r_end) ps[r0 + i - r_begin] += s;
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < r_end - r_begin; q += PRECOND_THREADS) z[tilde_idx[d.t_off + r_begin + q]] = ps[q];
}

// Several right-hand sides per pass over W: v_q|Sigma_j (q < NB) staged in LDS
// one after the other (each read like the single apply's, without extra bank
// conflicts), each W element multiplied by all of them. For every
// right-hand side the sums are formed in the order of k_precond (the row sums
// by wave_sum_many, which pairs lanes as wave_sum does), so a batched apply
// equals NB single applies bit for bit. desc and blk_sub are the batched
// apply's own block plan (fewer, larger blocks than the single apply's).
// RPW rows per wave and UNR 16-byte chunks in flight per row are tunable as
// in k_precond (the sums do not depend on them). With PIPE the full chunks go
// through two register sets of UNR chunks instead: the loads of the next
// group are issued before the products of the current one (one more form
// for the autotuner; with few waves beside the staged vectors it measured
// about as fast as one register set).
// Register budget (waves per SIMD) without spills: accumulators, loads in
// flight and the v values of a chunk for every right-hand side.
// (Values from the compiler's register counts for each instance.)
constexpr int multi_waves(int nb, int vn, int rpw, int unr, bool pipe) {
  return pipe ? (nb >= 4 || unr >= 2 ? 2 : 3)
         : (rpw == 2 && unr == 2) ? (nb >= 4 ? (vn >= 4 ? 4 : 6) : (vn >= 4 ? 7 : 8))
         : vn >= 4 ? (rpw * unr <= 4 ? 4 : rpw == 8 ? 2 : 3)
                   : (rpw * unr <= 4 ? (nb >= 4 ? 4 : 5) : rpw == 8 ? (nb >= 4 ? 2 : 3) : 4);
}

template <typename T, int NB, int MULTI_RPW, int UNR, bool PIPE = false>
__global__ __launch_bounds__(PRECOND_THREADS, multi_waves(NB, VecOf<T>::n, MULTI_RPW, UNR, PIPE)) void k_precond_multi(const SubDesc* __restrict__ desc,
                                                                   const int32_t* __restrict__ blk_sub,
                                                                   const int32_t* __restrict__ sig_idx,
                                                                   const int32_t* __restrict__ tilde_idx,
                                                                   const T* __restrict__ W,
                                                                   const double* __restrict__ v, int64_t v_stride,
                                                                   const double* __restrict__ scale,
                                                                   int64_t scale_stride, double* __restrict__ z,
                                                                   int64_t z_stride) {
  extern __shared__ double vs[];  // vs[q * ldw + c]
  typedef typename VecOf<T>::type VT;
  constexpr int VN = VecOf<T>::n;
  constexpr int CW = W_CW<T>;
  constexpr int64_t KS = (int64_t)W_TILE * CW;
  constexpr int NWAVE = PRECOND_THREADS / 64;
  const int blk = blockIdx.x;
  const int j = blk_sub[blk];
  const SubDesc d = desc[j];
  double sc[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) sc[q] = scale ? scale[q * scale_stride] : 1.0;
  {  // gather as in gather_v, all NB vectors' loads of a column group together
    const int32_t* si = sig_idx + d.u_off;
    for (int c0 = threadIdx.x; c0 < d.ldw; c0 += PRECOND_GATHER * PRECOND_THREADS) {
      int32_t g[PRECOND_GATHER];
      double x[NB][PRECOND_GATHER];
#pragma unroll
      for (int u = 0; u < PRECOND_GATHER; ++u) {
        const int c = c0 + u * PRECOND_THREADS;
        g[u] = si[c < d.m ? c : 0];
      }
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int u = 0; u < PRECOND_GATHER; ++u) x[q][u] = v[q * v_stride + g[u]];
#pragma unroll
      for (int u = 0; u < PRECOND_GATHER; ++u) {
        const int c = c0 + u * PRECOND_THREADS;
        if (c < d.ldw)
#pragma unroll
          for (int q = 0; q < NB; ++q) vs[q * d.ldw + c] = c < d.m ? sc[q] * x[q][u] : 0.0;
      }
    }
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r_begin = (blk - d.blk_off) * d.rpb;
  const int r_end = min(r_begin + d.rpb, d.t);
  const int nfull = d.ldw / CW, wk = d.ldw - nfull * CW;
  const double* vl = vs + lane * VN;
  for (int r0 = r_begin + wave * MULTI_RPW; r0 < r_end; r0 += NWAVE * MULTI_RPW) {
    const int R = r0 / W_TILE * W_TILE;
    const T* wf = W + d.w_off + (int64_t)R * d.ldw + (r0 - R) * CW + lane * VN;
    int ro[MULTI_RPW];
    double acc[MULTI_RPW][NB];
#pragma unroll
    for (int i = 0; i < MULTI_RPW; ++i) {
      ro[i] = min(i, r_end - 1 - r0);
#pragma unroll
      for (int q = 0; q < NB; ++q) acc[i][q] = 0.0;
    }
    int k = 0;
    if constexpr (PIPE) {  // groups of UNR chunks, two groups held
      VT wa[UNR][MULTI_RPW], wb[UNR][MULTI_RPW];
      auto fetch = [&](VT(&w)[UNR][MULTI_RPW], int kk) {
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
          for (int i = 0; i < MULTI_RPW; ++i)
            w[u][i] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(wf + (kk + u) * KS + ro[i] * CW));
      };
      auto madd = [&](const VT(&w)[UNR][MULTI_RPW], int kk) {
#pragma unroll
        for (int u = 0; u < UNR; ++u)
#pragma unroll
          for (int e = 0; e < VN; ++e)
#pragma unroll
            for (int q = 0; q < NB; ++q) {
              const double xv = vl[q * d.ldw + (kk + u) * CW + e];
#pragma unroll
              for (int i = 0; i < MULTI_RPW; ++i) acc[i][q] += (double)w[u][i][e] * xv;
            }
      };
      const int kg = nfull / UNR * UNR;  // chunks in whole groups; the rest below
      if (kg > 0) fetch(wa, 0);
#pragma unroll 1
      for (; k + 2 * UNR <= kg; k += 2 * UNR) {  // wa holds the group at k
        fetch(wb, k + UNR);
        madd(wa, k);
        if (k + 2 * UNR < kg) fetch(wa, k + 2 * UNR);
        madd(wb, k + UNR);
      }
      if (k < kg) {  // odd number of groups: the last is in wa
        madd(wa, k);
        k += UNR;
      }
    }
#pragma unroll 1
    for (; !PIPE && k + UNR <= nfull; k += UNR) {
      VT wv[UNR][MULTI_RPW];
#pragma unroll
      for (int u = 0; u < UNR; ++u)
#pragma unroll
        for (int i = 0; i < MULTI_RPW; ++i)
          wv[u][i] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(wf + (k + u) * KS + ro[i] * CW));
#pragma unroll
      for (int u = 0; u < UNR; ++u)
#pragma unroll
        for (int e = 0; e < VN; ++e)
#pragma unroll
          for (int q = 0; q < NB; ++q) {
            const double xv = vl[q * d.ldw + (k + u) * CW + e];
#pragma unroll
            for (int i = 0; i < MULTI_RPW; ++i) acc[i][q] += (double)wv[u][i][e] * xv;
          }
    }
#pragma unroll 1
    for (; k < nfull; ++k) {
      VT wv[MULTI_RPW];
#pragma unroll
      for (int i = 0; i < MULTI_RPW; ++i)
        wv[i] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(wf + k * KS + ro[i] * CW));
#pragma unroll
      for (int e = 0; e < VN; ++e)
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          const double xv = vl[q * d.ldw + k * CW + e];
#pragma unroll
          for (int i = 0; i < MULTI_RPW; ++i) acc[i][q] += (double)wv[i][e] * xv;
        }
    }
    if (lane * VN < wk) {
      const T* wt = W + d.w_off + (int64_t)R * d.ldw + nfull * KS + (r0 - R) * wk + lane * VN;
      VT wv[MULTI_RPW];
#pragma unroll
      for (int i = 0; i < MULTI_RPW; ++i) wv[i] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(wt + ro[i] * wk));
#pragma unroll
      for (int e = 0; e < VN; ++e)
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          const double xv = vl[q * d.ldw + nfull * CW + e];
#pragma unroll
          for (int i = 0; i < MULTI_RPW; ++i) acc[i][q] += (double)wv[i][e] * xv;
        }
    }
    // the RPW x NB row sums, each as wave_sum forms it, in groups of up to 8
    // (beside the second register set 4, or one at a time for 4-byte W, so
    // that no exchange temporary spills); one lane writes each
    constexpr int K = MULTI_RPW * NB, G = K < 8 ? K : !PIPE ? 8 : VN >= 4 ? 1 : 4, LG = ilog2(G);
#pragma unroll
    for (int g = 0; g < K; g += G) {
      double red[G];
#pragma unroll
      for (int k = 0; k < G; ++k) red[k] = acc[(g + k) / NB][(g + k) % NB];
      const double s = wave_sum_many<G>(red, lane);
      const int kv = g + (lane >> (6 - LG)), i = kv / NB, q = kv % NB;
      if ((lane & ((1 << (6 - LG)) - 1)) == 0 && r0 + i < r_end) z[q * z_stride + tilde_idx[d.t_off + r0 + i]] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// Local operator assembly (Section 5, eq. localOP) into the augmented matrix
//   [ A_j        E_Sigma ]      E_Sigma: identity on the Sigma_j rows
//   [ R~_j          0    ]      R~_j: selects Sigma~_j
// stored row-major. Eliminating the first n_j columns leaves -W_j in the
// lower-right block. Interior rows: (c + 6/h^2) u_x - (1/h^2) sum over the FD
// neighbours of their extended value: the E row for Sigma_j and ghost
// neighbours, the Robin row T_b = E[x*(b)] / (1 + alpha_b s_b) (eq. robfo) for
// a neighbour in B_j (ORAS), 0 for RAS (T_j = [0 I] with u_b = 0). B rows
// (ORAS), where the local Laplacian has no row:
// (c + 6/h^2) u_b - (6/h^2) T_b u = 0.
// The unknowns sit in the subdomain's elimination order (reverse
// Cuthill-McKee); rcol marks the Sigma_j unknowns with their right-hand
// column (in order of position) and the B_j unknowns with -1; border row i
// selects the i-th Sigma~_j node in order of position (tilde_pos). A
// right-hand column then keeps its single unit entry until that row is chosen
// as a pivot, and a border row stays zero left of its unit entry, so the
// blocks the elimination has not reached yet are exactly zero.
// Column lookup: binary search of the band index in the sorted unknown list.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int local_pos(const int32_t* __restrict__ srt, const int32_t* __restrict__ pos,
                                         int n, int32_t key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (srt[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n && srt[lo] == key) ? pos[lo] : -1;
}

template <typename T, int P>
__global__ __launch_bounds__(256) void k_assemble(const SubDesc* __restrict__ desc, int64_t na, int64_t n_rows,
                                                  const int32_t* __restrict__ lines,
                                                  const double* __restrict__ wts,
                                                  const int32_t* __restrict__ nbr,
                                                  const int32_t* __restrict__ U,
                                                  const int32_t* __restrict__ usrt,
                                                  const int32_t* __restrict__ upos,
                                                  const int32_t* __restrict__ bx,
                                                  const double* __restrict__ bs,
                                                  const double* __restrict__ ba,
                                                  const int32_t* __restrict__ tilde_pos,
                                                  const int32_t* __restrict__ rcol,
                                                  const int32_t* __restrict__ ext_pos,
                                                  double diag, double ih2, int oras, T* __restrict__ A) {
  constexpr int P1 = P + 1;
  const int j = blockIdx.y;
  const SubDesc d = desc[j];
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= d.rows) return;
  T* row = A + d.a_off + (int64_t)r * d.lda;
  const int32_t* srt = usrt + d.u_off;
  const int32_t* ps = upos + d.u_off;
  auto add_ext = [&](int32_t node, double scale) {
    const int64_t at = ext_pos[node];  // the row's position in apply order (structure of arrays)
    auto w = [&](int c) { return wts[c * n_rows + at]; };
    for (int a = 0; a < P1; ++a)
      for (int b = 0; b < P1; ++b) {
        const int32_t s = lines[(a * P1 + b) * n_rows + at];
        const double wab = w(a) * w(P1 + b);
        for (int c = 0; c < P1; ++c) {
          const int q = local_pos(srt, ps, d.n, s + c);
          if (q >= 0) row[q] = (T)((double)row[q] - scale * (wab * w(2 * P1 + c)));
        }
      }
  };
  const int rc = r < d.n ? rcol[d.u_off + r] : -1;
  if (rc >= 0) {  // a Sigma_j unknown; its right-hand column is d.n + rc
    const int32_t x = U[d.u_off + r];
    row[r] = (T)((double)row[r] + diag);
    for (int e = 0; e < 6; ++e) {
      const int32_t y = nbr[e * na + x];
      if (y < na) {
        const int q = local_pos(srt, ps, d.n, y);
        if (q >= 0 && rcol[d.u_off + q] < 0) {  // ORAS transmission node: its Robin extension row
          const int32_t k = d.u_off + q;
          add_ext(bx[k], ih2 / (1.0 + ba[k] * bs[k]));
          continue;
        }
        if (q < 0) continue;  // RAS: u_b = 0
      }
      add_ext(y, ih2);
    }
    row[d.n + rc] = (T)1;
  } else if (r < d.n) {
    const int32_t k = d.u_off + r;
    row[r] = (T)((double)row[r] + diag);
    if (oras) add_ext(bx[k], 6.0 * ih2 / (1.0 + ba[k] * bs[k]));
  } else {
    row[tilde_pos[d.t_off + (r - d.n)]] = (T)1;
  }
}

// ---------------------------------------------------------------------------
// Batched right-looking LU with partial pivoting on the augmented matrices
// (pivots searched in the first n_j rows only), panel width NB.
// ---------------------------------------------------------------------------
constexpr int LU_NB = 32;  // panel width
constexpr int LU_KMAX = 128;  // outer block width (panels caught up left-looking inside it)
static_assert(LU_KMAX % LU_NB == 0, "whole panels per outer block");
constexpr int PANEL_THREADS = 1024;
constexpr int PANEL_TB = 4;     // 32-row tiles per round of the panel's gather and write-back

// (value, row) pairs are ordered by value, then by lower row: the maximum of
// that total order is the pivot, whatever order the pairs are combined in.
__device__ __forceinline__ bool argmax_takes(double ob, int oi, double b, int i) {
  return ob > b || (ob == b && oi < i);
}

// One exchange of the wave argmax by a data-parallel-primitives lane move
// (CTRL: a fixed pairing of lanes within each 16-lane row), no LDS traffic.
template <int CTRL>
__device__ __forceinline__ void argmax_dpp(double& best, int& bi) {
  const long long b = __double_as_longlong(best);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  const int oi = __builtin_amdgcn_update_dpp(0, bi, CTRL, 0xF, 0xF, false);
  const double ob = __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
  if (argmax_takes(ob, oi, best, bi)) {
    best = ob;
    bi = oi;
  }
}

// Wave argmax: within each 16-lane row by four lane moves (swap neighbours,
// swap pairs, mirror each half-row, mirror the row: each joins two groups
// that already agree), then the four rows' results read from lanes 0, 16, 32
// and 48; every lane returns the wave's result.
__device__ __forceinline__ void wave_argmax(double& best, int& bi) {
  argmax_dpp<0xB1>(best, bi);   // quad_perm [1,0,3,2]
  argmax_dpp<0x4E>(best, bi);   // quad_perm [2,3,0,1]
  argmax_dpp<0x141>(best, bi);  // row_half_mirror
  argmax_dpp<0x140>(best, bi);  // row_mirror
  const long long b = __double_as_longlong(best);
  const int blo = (int)b, bhi = (int)(b >> 32);
  auto at = [&](int lane, double& v, int& i) {
    const int lo = __builtin_amdgcn_readlane(blo, lane), hi = __builtin_amdgcn_readlane(bhi, lane);
    v = __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
    i = __builtin_amdgcn_readlane(bi, lane);
  };
  double rb;
  int ri;
  at(0, rb, ri);
#pragma unroll
  for (int r = 16; r < 64; r += 16) {
    double v;
    int i;
    at(r, v, i);
    if (argmax_takes(v, i, rb, ri)) {
      rb = v;
      ri = i;
    }
  }
  best = rb;
  bi = ri;
}

// (value, row) pair reduction over the block: largest |value|, lowest row on
// ties; -1 when every value is zero. One barrier: each wave posts its result,
// then every thread reduces the posted results itself. rv / ri are written
// again only by the next call, which callers reach through another barrier.
template <int NT = PANEL_THREADS>
__device__ __forceinline__ int block_argmax(double best, int bi, double* rv, int* ri) {
  constexpr int NW = NT / 64;
  wave_argmax(best, bi);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    rv[wave] = best;
    ri[wave] = bi;
  }
  __syncthreads();
  double b0 = rv[0];
  int i0 = ri[0];
#pragma unroll
  for (int w = 1; w < NW; ++w)
    if (argmax_takes(rv[w], ri[w], b0, i0)) {
      b0 = rv[w];
      i0 = ri[w];
    }
  return (i0 == INT32_MAX || b0 == 0.0) ? -1 : i0;
}

// Panel scratch layout: 64-row tiles, column-major inside a tile, so that a
// wave's 64 consecutive rows read a column as 64 consecutive values and one
// row's columns sit at fixed offsets (64 apart) from a single address.
__device__ __forceinline__ int64_t panel_index(int r, int c) {
  return (int64_t)(r >> 6) * (LU_NB * 64) + c * 64 + (r & 63);
}

// Fast form of the panel (k_lu_panel below) when its rows fit on the CU: rows
// [0, PANEL_FAST_THREADS) in registers (thread t holds row t's LU_NB values),
// rows [PANEL_FAST_THREADS, PANEL_FAST_THREADS + PanelLds<T>::ROWS) in LDS
// (column c of LDS row q at lds[c * LRP + q]), so the column steps touch no
// global memory.
// Same arithmetic in the same order as the scratch form: column jj: the
// interchange of rows jj and piv, l = a_jj / u_jj, a_c -= l u_c for c > jj,
// the pivot of column jj+1 from the updated values.
template <typename T>
struct PanelLds;
template <>
struct PanelLds<double> {
  static constexpr int LRP = 577;  // odd: a column's rows fall in consecutive banks
  static constexpr int ROWS = LRP - 1;
};
template <>
struct PanelLds<float> {
  static constexpr int LRP = 1153;
  static constexpr int ROWS = LRP - 1;
};
// dynamic LDS of the panel kernel: the LDS rows of the fast form, or the
// staging tiles of either form (they are used one after the other)
template <typename T>
constexpr size_t panel_lds_bytes() {
  return (size_t)PanelLds<T>::LRP * LU_NB * sizeof(T);
}
constexpr int PANEL_STAGE = 128;  // rows per staging round of the register rows

constexpr int PANEL_FAST_THREADS = 512;  // threads per block of the fast form
constexpr int PANEL_FAST_RR = 2;         // register rows per thread: rows t and t + PANEL_FAST_THREADS

// Used only when every panel of the launch is LU_NB wide and its rows that
// may be nonzero fit (host-checked from pbound).
template <typename T>
__global__ __launch_bounds__(PANEL_FAST_THREADS) void k_lu_panel_fast(const SubDesc* __restrict__ desc,
                                                                      T* __restrict__ A, int k,
                                                                      int32_t* __restrict__ ipiv,
                                                                      int32_t* __restrict__ info,
                                                                      const int32_t* __restrict__ pbound,
                                                                      int32_t* __restrict__ rowhi) {
  constexpr int NT = PANEL_FAST_THREADS;
  constexpr int RR = PANEL_FAST_RR;
  constexpr int NR = RR * NT;  // register rows; LDS rows follow
  constexpr int NW = NT / 64;
  constexpr int LRP = PanelLds<T>::LRP;
  extern __shared__ __align__(16) unsigned char panel_dyn[];  // panel_lds_bytes<T>()
  __shared__ T xa[LU_NB];
  __shared__ T xb[LU_NB];
  __shared__ double rv[NW];
  __shared__ int ri[NW];
  __shared__ int hi_s[NW];
  const int j = blockIdx.x;
  const SubDesc d = desc[j];
  if (k >= d.n) return;
  const int kb = LU_NB;
  T* a = A + d.a_off + (int64_t)k * d.lda + k;
  const int64_t lda = d.lda;
  const int32_t* pb = pbound + 2 * ((int64_t)d.pb_off + k / LU_NB);
  const int ga = min(pb[0] - k, d.n - k);
  const int32_t pb1 = pb[1];
  const int t = threadIdx.x;
  T* stage = reinterpret_cast<T*>(panel_dyn);  // PANEL_STAGE x 33
  T* L = reinterpret_cast<T*>(panel_dyn);      // LDS rows, after the register rows are in place
  T v[RR][LU_NB];  // register row t + s NT in v[s]
#pragma unroll
  for (int s2 = 0; s2 < RR; ++s2)
#pragma unroll
    for (int c = 0; c < LU_NB; ++c) v[s2][c] = (T)0;
  int hia = 0;
  double best = -1.0;
  int bi = INT32_MAX;
  // lanes cover RPL rows x 32 columns at a time; a round of PANEL_STAGE rows
  // is LAY such layers, their loads in flight together
  constexpr int RPL = NT / 32, LAY = PANEL_STAGE / RPL;
  const int rl = t >> 5, cl = t & 31;
  // register rows [0, gr): staged through LDS, coalesced loads
  const int gr = min(ga, NR);
  for (int R0 = 0; R0 < gr; R0 += PANEL_STAGE) {
    T g[LAY];
#pragma unroll
    for (int b = 0; b < LAY; ++b) {
      const int r = R0 + b * RPL + rl;
      g[b] = (r < gr && cl < kb) ? a[(int64_t)r * lda + cl] : (T)0;
    }
#pragma unroll
    for (int b = 0; b < LAY; ++b) {
      stage[(b * RPL + rl) * 33 + cl] = g[b];
      const int r = R0 + b * RPL + rl;
      if (g[b] != (T)0) {
        hia = r + 1;
        const double av = fabs((double)g[b]);
        if (cl == 0 && av > best) { best = av; bi = r; }
      }
    }
    __syncthreads();
#pragma unroll
    for (int s2 = 0; s2 < RR; ++s2) {
      const int r = t + s2 * NT;
      if (r >= R0 && r < R0 + PANEL_STAGE) {
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) v[s2][c] = stage[(r - R0) * 33 + c];
      }
    }
    __syncthreads();
  }
  // LDS rows [NR, ga)
  for (int r0 = NR; r0 < ga; r0 += PANEL_STAGE) {
    T g[LAY];
#pragma unroll
    for (int b = 0; b < LAY; ++b) {
      const int r = r0 + b * RPL + rl;
      g[b] = (r < ga && cl < kb) ? a[(int64_t)r * lda + cl] : (T)0;
    }
#pragma unroll
    for (int b = 0; b < LAY; ++b) {
      const int r = r0 + b * RPL + rl;
      if (r < ga) L[cl * LRP + (r - NR)] = g[b];
      if (g[b] != (T)0) {
        hia = r + 1;
        const double av = fabs((double)g[b]);
        if (cl == 0 && av > best) { best = av; bi = r; }
      }
    }
  }
  {
    const int lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) hia = max(hia, __shfl_xor(hia, o, 64));
    if (lane == 0) hi_s[wave] = hia;
  }
  int piv = block_argmax<NT>(best, bi, rv, ri);  // its barrier also publishes hi_s and the LDS rows
  int ea = kb;
  for (int w = 0; w < NW; ++w) ea = max(ea, hi_s[w]);
  if (t == 0) {
    int32_t* lv = rowhi + 2 * j;
    if (k % LU_KMAX == 0) {
      lv[0] = k + ea;
      lv[1] = pb1;
    } else {
      lv[0] = max(lv[0], k + ea);
      lv[1] = max(lv[1], pb1);
    }
  }
  constexpr int LM = (PanelLds<T>::ROWS + NT - 1) / NT;  // LDS rows per thread: q = t + m NT
  // The register row is rotated one place per column, so that at step jj
  // v[c] holds column jj + c (mod LU_NB): every access to v is at a fixed
  // index (a runtime index would put v in private memory) and after LU_NB
  // steps v is back in column order. The pivot row xa and the exchange
  // buffer xb are kept in column order.
  for (int jj = 0; jj < LU_NB; ++jj) {
    if (t == 0) {
      ipiv[d.u_off + k + jj] = k + (piv < 0 ? jj : piv);
      if (piv < 0 && info[j] == 0) info[j] = k + jj + 1;
    }
    // interchange rows jj (a register row) and piv: the pivot row to xa,
    // row jj to xb; each owner then takes the other
    const bool swap = piv >= 0 && piv != jj;
    if (swap) {
      if (piv < NR) {
        if (t == piv % NT) {
#pragma unroll
          for (int s2 = 0; s2 < RR; ++s2)
            if (s2 == piv / NT) {
#pragma unroll
              for (int c = 0; c < LU_NB; ++c) xa[(c + jj) & (LU_NB - 1)] = v[s2][c];
            }
        }
      } else if (t == (piv - NR) % NT) {
        const int q = piv - NR;
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) xa[c] = L[c * LRP + q];
      }
      if (t == jj) {
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) xb[(c + jj) & (LU_NB - 1)] = v[0][c];
      }
    } else if (t == jj) {
#pragma unroll
      for (int c = 0; c < LU_NB; ++c) xa[(c + jj) & (LU_NB - 1)] = v[0][c];
    }
    __syncthreads();
    if (swap) {
      if (t == jj) {
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) v[0][c] = xa[(c + jj) & (LU_NB - 1)];
      }
      if (piv < NR) {
        if (t == piv % NT) {
#pragma unroll
          for (int s2 = 0; s2 < RR; ++s2)
            if (s2 == piv / NT) {
#pragma unroll
              for (int c = 0; c < LU_NB; ++c) v[s2][c] = xb[(c + jj) & (LU_NB - 1)];
            }
        }
      } else if (t == (piv - NR) % NT) {
        const int q = piv - NR;
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) L[c * LRP + q] = xb[c];
      }
    }
    const T pv = xa[jj];
    best = -1.0;
    bi = INT32_MAX;
    if (piv >= 0) {
#pragma unroll
      for (int s2 = 0; s2 < RR; ++s2) {
        asm volatile("" ::: "memory");  // xa is read where it is used
        const int r = t + s2 * NT;
        if (r > jj && r < ea) {  // register row r: column jj at v[s2][0]
          const T l = v[s2][0] / pv;
          v[s2][0] = l;
#pragma unroll
          for (int c = 1; c < LU_NB; ++c)
            if (c < LU_NB - jj) v[s2][c] = v[s2][c] - l * xa[jj + c];
        }
      }
      asm volatile("" ::: "memory");
#pragma unroll
      for (int m = 0; m < LM; ++m) {
        const int q = t + m * NT;
        if (NR + q < ea) {  // LDS row NR + q (> jj)
          T* lr = L + q;
          const T l = lr[jj * LRP] / pv;
          lr[jj * LRP] = l;
          for (int c = jj + 1; c < LU_NB; ++c) lr[c * LRP] = lr[c * LRP] - l * xa[c];
          if (jj + 1 < LU_NB) {
            const double av = fabs((double)lr[(jj + 1) * LRP]);
            if (av > best) { best = av; bi = NR + q; }
          }
        }
      }
    } else if (jj + 1 < LU_NB) {  // singular column: nothing eliminated, search the next one
#pragma unroll
      for (int m = 0; m < LM; ++m) {
        const int q = t + m * NT;
        if (NR + q < ea) {
          const double av = fabs((double)L[(jj + 1) * LRP + q]);
          if (av > best) { best = av; bi = NR + q; }
        }
      }
    }
    // rotate: column jj + 1 to v[s][0]; pivot candidates of column jj + 1
    // among the register rows (in row order, after the LDS rows' candidates:
    // ties keep the lower row in block_argmax)
#pragma unroll
    for (int s2 = 0; s2 < RR; ++s2) {
      const T v0 = v[s2][0];
#pragma unroll
      for (int c = 0; c < LU_NB - 1; ++c) v[s2][c] = v[s2][c + 1];
      v[s2][LU_NB - 1] = v0;
      const int r = t + s2 * NT;
      if (jj + 1 < LU_NB && r > jj && r < ea) {
        const double av = fabs((double)v[s2][0]);
        if (av > best || (av == best && r < bi)) { best = av; bi = r; }
      }
    }
    if (jj + 1 < LU_NB) piv = block_argmax<NT>(best, bi, rv, ri);
    else __syncthreads();
  }
  // write back: the LDS rows, then the register rows through the staging tile
  for (int r0 = NR; r0 < ea; r0 += PANEL_STAGE) {
#pragma unroll
    for (int b = 0; b < LAY; ++b) {
      const int r = r0 + b * RPL + rl;
      if (r < ea && cl < kb) a[(int64_t)r * lda + cl] = L[cl * LRP + (r - NR)];
    }
  }
  __syncthreads();
  const int er = min(ea, NR);
  for (int R0 = 0; R0 < er; R0 += PANEL_STAGE) {
#pragma unroll
    for (int s2 = 0; s2 < RR; ++s2) {
      const int r = t + s2 * NT;
      if (r >= R0 && r < R0 + PANEL_STAGE) {
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) stage[(r - R0) * 33 + c] = v[s2][c];
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < LAY; ++b) {
      const int r = R0 + b * RPL + rl;
      if (r < er && cl < kb) a[(int64_t)r * lda + cl] = stage[(b * RPL + rl) * 33 + cl];
    }
    __syncthreads();
  }
}

// Unblocked LU with partial pivoting of the A_j rows of the panel
// A[k:n, k:k+kb] of every subdomain (one block each); the border rows, which
// never pivot, are eliminated afterwards by k_lu_border. Rows that are zero
// throughout the panel have zero multipliers, so eliminating them changes
// nothing: the panel reads only the rows the structure of A_j allows to be
// nonzero (pbound[0]), finds among them the last row that is nonzero, and
// eliminates only up to it. Those rows are moved to the scratch (transposed
// through LDS, PANEL_TB 32-row tiles per round with their loads in flight
// together), where a pass gives each thread one row with all its values
// loaded at once; the pass that eliminates column jj also finds the pivot of
// column jj+1. The last possibly nonzero rows (absolute; border rows: from
// pbound[1]) are kept in rowhi[2j], rowhi[2j+1], as maxima over the panels of
// the current outer block of LU_KMAX columns.
template <typename T>
__global__ __launch_bounds__(PANEL_THREADS) void k_lu_panel(const SubDesc* __restrict__ desc, T* __restrict__ A,
                                                            int k, int32_t* __restrict__ ipiv,
                                                            int32_t* __restrict__ info, T* __restrict__ scratch,
                                                            const int64_t* __restrict__ scr_off,
                                                            const int32_t* __restrict__ pbound,
                                                            int32_t* __restrict__ rowhi) {
  constexpr int NW = PANEL_THREADS / 64;
  extern __shared__ __align__(16) unsigned char panel_dyn[];  // panel_lds_bytes<T>()
  T (*tile)[33] = reinterpret_cast<T (*)[33]>(panel_dyn);      // PANEL_TB * 32 rows
  __shared__ T prow[LU_NB];
  __shared__ double rv[NW];
  __shared__ int ri[NW];
  __shared__ int hi_s[1][NW];
  const int j = blockIdx.x;
  const SubDesc d = desc[j];
  if (k >= d.n) return;
  const int kb = min(LU_NB, d.n - k);
  const int np = d.n - k;       // pivot-eligible rows
  T* a = A + d.a_off + (int64_t)k * d.lda + k;
  const int64_t lda = d.lda;
  T* P = scratch + scr_off[j];
  const int t = threadIdx.x;
  const int32_t* pb = pbound + 2 * ((int64_t)d.pb_off + k / LU_NB);
  const int ga = min(pb[0] - k, np);  // A_j rows [0, ga) may be nonzero
  // gather those rows, noting the last nonzero row and the pivot of column 0
  int hia = 0;
  double best = -1.0;
  int bi = INT32_MAX;
  {
    const int s1 = ga;
    for (int r0 = 0; r0 < s1; r0 += PANEL_TB * 32) {
      {
        const int rl = t >> 5, c = t & 31;
        T g[PANEL_TB];
#pragma unroll
        for (int b = 0; b < PANEL_TB; ++b) {
          const int r = r0 + b * 32 + rl;
          g[b] = (r < s1 && c < kb) ? a[(int64_t)r * lda + c] : (T)0;
        }
#pragma unroll
        for (int b = 0; b < PANEL_TB; ++b) {
          tile[b * 32 + rl][c] = g[b];
          const int r = r0 + b * 32 + rl;
          if (g[b] != (T)0) {
            hia = r + 1;
            const double av = fabs((double)g[b]);
            if (c == 0 && av > best) { best = av; bi = r; }
          }
        }
      }
      __syncthreads();
      {
        const int c = t >> 5, rl = t & 31;
#pragma unroll
        for (int b = 0; b < PANEL_TB; ++b) {
          const int r = r0 + b * 32 + rl;
          if (r < s1) P[panel_index(r, c)] = tile[b * 32 + rl][c];
        }
      }
      __syncthreads();
    }
  }
  {
    const int lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) hia = max(hia, __shfl_xor(hia, o, 64));
    if (lane == 0) hi_s[0][wave] = hia;
  }
  int piv = block_argmax(best, bi, rv, ri);  // its barrier also publishes hi_s
  // active rows [0, ea)
  int ea = kb;
  for (int w = 0; w < NW; ++w) ea = max(ea, hi_s[0][w]);
  if (t == 0) {
    int32_t* lv = rowhi + 2 * j;
    if (k % LU_KMAX == 0) {
      lv[0] = k + ea;
      lv[1] = pb[1];
    } else {
      lv[0] = max(lv[0], k + ea);
      lv[1] = max(lv[1], pb[1]);
    }
  }
  for (int jj = 0; jj < kb; ++jj) {
    if (t == 0) {
      ipiv[d.u_off + k + jj] = k + (piv < 0 ? jj : piv);
      if (piv < 0 && info[j] == 0) info[j] = k + jj + 1;
    }
    // interchange rows jj and piv (thread c: column c) and keep the new row jj
    if (t < kb) {
      T* pj = P + panel_index(jj, t);
      const T rj = *pj;
      if (piv >= 0 && piv != jj) {
        T* pp = P + panel_index(piv, t);
        const T rp = *pp;
        *pj = rp;
        *pp = rj;
        prow[t] = rp;
      } else {
        prow[t] = rj;
      }
    }
    __syncthreads();
    const T pv = prow[jj];
    best = -1.0;
    bi = INT32_MAX;
    if (piv >= 0) {
      for (int r = jj + 1 + t; r < ea; r += PANEL_THREADS) {
        // prow is read from LDS inside the loop (a compiler-only barrier keeps
        // its values from being held in registers next to the row's)
        asm volatile("" ::: "memory");
        T* row = P + panel_index(r, 0);  // column c at row[64 c]
        T v[LU_NB];
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) v[c] = row[64 * c];  // columns past kb are zeros, not used
        const T vj = row[64 * jj];
        const T vn = jj + 1 < kb ? row[64 * (jj + 1)] : (T)0;
        const T l = vj / pv;
#pragma unroll
        for (int c = 0; c < LU_NB; ++c)
          if (c > jj && c < kb) row[64 * c] = v[c] - l * prow[c];
        row[64 * jj] = l;
        if (jj + 1 < kb) {
          const double av = fabs((double)(vn - l * prow[jj + 1]));
          if (av > best) { best = av; bi = r; }
        }
      }
    } else if (jj + 1 < kb) {  // singular column: nothing eliminated, search the next one
      for (int r = jj + 1 + t; r < ea; r += PANEL_THREADS) {
        const double av = fabs((double)P[panel_index(r, jj + 1)]);
        if (av > best) { best = av; bi = r; }
      }
    }
    if (jj + 1 < kb) piv = block_argmax(best, bi, rv, ri);
    else __syncthreads();
  }
  // write the active rows of the factored panel back (same rounds)
  {
    const int s1 = ea;
    for (int r0 = 0; r0 < s1; r0 += PANEL_TB * 32) {
      {
        const int c = t >> 5, rl = t & 31;
        T g[PANEL_TB];
#pragma unroll
        for (int b = 0; b < PANEL_TB; ++b) {
          const int r = r0 + b * 32 + rl;
          g[b] = (r < s1 && c < kb) ? P[panel_index(r, c)] : (T)0;
        }
#pragma unroll
        for (int b = 0; b < PANEL_TB; ++b) tile[b * 32 + rl][c] = g[b];
      }
      __syncthreads();
      {
        const int rl = t >> 5, c = t & 31;
#pragma unroll
        for (int b = 0; b < PANEL_TB; ++b) {
          const int r = r0 + b * 32 + rl;
          if (r < s1 && c < kb) a[(int64_t)r * lda + c] = tile[b * 32 + rl][c];
        }
      }
      __syncthreads();
    }
  }
}

// The border rows of a panel (Section 5: the rows R~_j appended to A_j) take
// no part in pivoting, so their multipliers need not wait for the panel's
// column-by-column pivot searches: after the panel, each border row that may
// be nonzero in it (rows [n, pbound[1])) is eliminated against the panel's
// final upper triangle U11 by the same steps the panel applies to its own
// rows (column jj: l = a_jj / u_jj, then a_c -= l u_jc for c > jj; nothing
// where u_jj = 0, a column the panel found singular). One row per thread,
// U11 in LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_border(const SubDesc* __restrict__ desc, T* __restrict__ A, int k,
                                                   const int32_t* __restrict__ pbound) {
  __shared__ T U[LU_NB][LU_NB + 1];
  const int j = blockIdx.y;
  const SubDesc d = desc[j];
  if (k >= d.n) return;
  const int kb = min(LU_NB, d.n - k);
  const int n_b = pbound[2 * ((int64_t)d.pb_off + k / LU_NB) + 1] - d.n;
  if ((int)blockIdx.x * 256 >= n_b) return;  // the whole block
  const int64_t lda = d.lda;
  const T* u = A + d.a_off + (int64_t)k * lda + k;
  for (int e = threadIdx.x; e < LU_NB * LU_NB; e += 256) {
    const int r = e / LU_NB, c = e - (e / LU_NB) * LU_NB;
    U[r][c] = (r < kb && c < kb) ? u[(int64_t)r * lda + c] : (T)0;
  }
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_b) return;
  T* row = A + d.a_off + (int64_t)(d.n + i) * lda + k;
  T v[LU_NB];
#pragma unroll
  for (int c = 0; c < LU_NB; ++c) v[c] = c < kb ? row[c] : (T)0;
#pragma unroll
  for (int jj = 0; jj < LU_NB; ++jj) {
    if (jj < kb && U[jj][jj] != (T)0) {
      const T l = v[jj] / U[jj][jj];
      v[jj] = l;
#pragma unroll
      for (int c = jj + 1; c < LU_NB; ++c) v[c] = v[c] - l * U[jj][c];
    }
  }
#pragma unroll
  for (int c = 0; c < LU_NB; ++c)
    if (c < kb) row[c] = v[c];
}

__device__ __forceinline__ int find_job(const int32_t* __restrict__ prefix, int n_jobs, int blk) {
  int lo = 0, hi = n_jobs - 1;  // largest q with prefix[q] <= blk
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= blk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One unit of blocked-LU work on subdomain j: the L block is columns
// [kstart, kstart + kdim) (rows interchanged by ipiv[kstart .. kstart+kdim)),
// applied to rows >= r_lo and columns [c_lo, c_hi).
struct LuJob {
  int32_t j, kstart, kdim, r_lo, c_lo, c_hi;
};

constexpr int TRSM_COLS = 64;

// sum_{q < i} li[q] X[q][t] in four interleaved partial sums (q mod 4),
// combined as (s0 + s1) + (s2 + s3): a quarter of the dependent chain of one
// running sum, in a fixed order. Terms are fetched sixteen at a time, all
// loads before the products, so that their latencies overlap (each partial
// sum still adds its terms in q order).
template <typename T>
__device__ __forceinline__ T row_dot4(const T* __restrict__ li, const T (*X)[TRSM_COLS], int i, int t) {
  T s0 = (T)0, s1 = (T)0, s2 = (T)0, s3 = (T)0;
  int q = 0;
  for (; q + 16 <= i; q += 16) {
    T lv[16], xv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      lv[u] = li[q + u];
      xv[u] = X[q + u][t];
    }
#pragma unroll
    for (int u = 0; u < 16; u += 4) {
      s0 += lv[u] * xv[u];
      s1 += lv[u + 1] * xv[u + 1];
      s2 += lv[u + 2] * xv[u + 2];
      s3 += lv[u + 3] * xv[u + 3];
    }
  }
  for (; q + 4 <= i; q += 4) {
    s0 += li[q] * X[q][t];
    s1 += li[q + 1] * X[q + 1][t];
    s2 += li[q + 2] * X[q + 2][t];
    s3 += li[q + 3] * X[q + 3][t];
  }
  if (q < i) s0 += li[q] * X[q][t];
  if (q + 1 < i) s1 += li[q + 1] * X[q + 1][t];
  if (q + 2 < i) s2 += li[q + 2] * X[q + 2][t];
  return (s0 + s1) + (s2 + s3);
}

// Forward substitution of one column held in registers (KD rows, fixed at
// compile time): x_i -= sum_{q<i} l_iq x_q, each row's sum formed as in
// row_dot4 (partial sum q mod 4, terms in q order, combined (s0 + s1) +
// (s2 + s3)), so the results equal row_dot4's bit for bit; row i of L11 is
// read from LDS (the same entry for every lane), with no dependence on x, so
// its loads run ahead of the arithmetic.
template <typename T, int KD, int LDL>
__device__ __forceinline__ void solve_column_regs(const T (*Ls)[LDL], T* col, int64_t lda) {
  T x[KD];
#pragma unroll
  for (int i = 0; i < KD; ++i) x[i] = col[(int64_t)i * lda];
#pragma unroll
  for (int i = 1; i < KD; ++i) {
    T s0 = (T)0, s1 = (T)0, s2 = (T)0, s3 = (T)0;
#pragma unroll
    for (int q = 0; q < i; ++q) {
      if ((q & 3) == 0) s0 += Ls[i][q] * x[q];
      else if ((q & 3) == 1) s1 += Ls[i][q] * x[q];
      else if ((q & 3) == 2) s2 += Ls[i][q] * x[q];
      else s3 += Ls[i][q] * x[q];
    }
    x[i] = x[i] - ((s0 + s1) + (s2 + s3));
    col[(int64_t)i * lda] = x[i];
  }
}

// Row interchanges ipiv[kstart + q] (q < kdim, in order) applied to columns
// [c_lo, c_hi); with TRSM, then U = L11^{-1} A on rows [kstart, kstart+kdim)
// (L11 unit lower triangular), column values in LDS. One wave per 64 columns.
// The interchanges are loaded once, two per lane, and broadcast by shuffles;
// most are the identity, and a block whose interchanges all are skips them.
template <typename T, bool TRSM>
__global__ __launch_bounds__(TRSM_COLS) void k_lu_swap_trsm(const SubDesc* __restrict__ desc, T* __restrict__ A,
                                                            const int32_t* __restrict__ ipiv,
                                                            const LuJob* __restrict__ jobs,
                                                            const int32_t* __restrict__ prefix, int n_jobs) {
  static_assert(LU_KMAX <= 2 * TRSM_COLS, "two interchanges per lane");
  // The solve form serves the catch-up of a panel inside its outer block, so
  // kdim = k - K0 <= LU_KMAX - LU_NB (the host plan builds no other).
  constexpr int KT = LU_KMAX - LU_NB;
  __shared__ T X[TRSM ? KT : 1][TRSM_COLS];  // the interchange-only form needs no LDS
  __shared__ T Ls[TRSM ? KT : 1][TRSM ? KT : 1];  // strictly lower L11, staged once
  const int q = find_job(prefix, n_jobs, blockIdx.x);
  const LuJob jb = jobs[q];
  const SubDesc d = desc[jb.j];
  const int t = threadIdx.x;
  const int c = jb.c_lo + (blockIdx.x - prefix[q]) * TRSM_COLS + t;
  const bool live = c < jb.c_hi;  // every lane takes part in the shuffles
  T* a = A + d.a_off;
  const int64_t lda = d.lda;
  if (TRSM) {
    // L11 (columns [kstart, kstart + kdim), not touched by the interchanges
    // below, which act on columns >= kstart + kdim) read row by row with
    // coalesced loads, all issued before the interchanges' round trips, so
    // that the solve reads its rows from LDS instead of one global round trip
    // per row
    const T* l11 = a + (int64_t)jb.kstart * lda + jb.kstart;
    static_assert(KT <= 2 * TRSM_COLS, "two L11 columns per lane");
    for (int i0 = 1; i0 < jb.kdim; i0 += 16) {  // sixteen rows' loads in flight together
      T g[16][2];
#pragma unroll
      for (int u = 0; u < 16; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = i0 + u, qq = t + h * TRSM_COLS;
          g[u][h] = (i < jb.kdim && qq < i) ? l11[(int64_t)i * lda + qq] : (T)0;
        }
#pragma unroll
      for (int u = 0; u < 16; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = i0 + u, qq = t + h * TRSM_COLS;
          if (i < jb.kdim && qq < i) Ls[i][qq] = g[u][h];
        }
    }
  }
  const int32_t* pg = ipiv + d.u_off + jb.kstart;
  const int pv0 = t < jb.kdim ? pg[t] : jb.kstart + t;
  const int pv1 = t + TRSM_COLS < jb.kdim ? pg[t + TRSM_COLS] : jb.kstart + t + TRSM_COLS;
  // most interchanges are the identity: skip the loop when all of them are
  const bool any_swap = __any(pv0 != jb.kstart + t || pv1 != jb.kstart + t + TRSM_COLS);
  for (int i = 0; any_swap && i < jb.kdim; ++i) {
    const int p = __shfl(i < TRSM_COLS ? pv0 : pv1, i & (TRSM_COLS - 1), TRSM_COLS);
    const int r = jb.kstart + i;
    if (live && p != r) {
      const T tmp = a[r * lda + c];
      a[r * lda + c] = a[p * lda + c];
      a[p * lda + c] = tmp;
    }
  }
  if (!TRSM) return;
  __syncthreads();  // the staged L11 (one wave: orders the LDS writes before the reads)
  if (!live) return;
  // forward substitution by rows: X_i -= sum_{q<i} l_iq X_q, row i of L11
  // from LDS; the column in registers for the block sizes that occur (kdim
  // is a multiple of LU_NB), else in LDS
  if constexpr (TRSM) {
    T* col = a + (int64_t)jb.kstart * lda + c;
    if (jb.kdim == 32) {
      solve_column_regs<T, 32, KT>(Ls, col, lda);
    } else if (jb.kdim == 64) {
      solve_column_regs<T, 64, KT>(Ls, col, lda);
    } else if (jb.kdim == 96) {
      solve_column_regs<T, 96, KT>(Ls, col, lda);
    } else {
      for (int i = 0; i < jb.kdim; ++i) X[i][t] = col[(int64_t)i * lda];
      for (int i = 1; i < jb.kdim; ++i) {
        const T x = X[i][t] - row_dot4<T>(&Ls[i][0], X, i, t);
        X[i][t] = x;
        col[(int64_t)i * lda] = x;
      }
    }
  }
}

// Trailing update on matrix cores: C -= Lsrc * Usrc for one 64x64 tile of C,
// K = kdim in chunks of GEMM_KC staged through LDS; C is read and written once.
// 16x16x4 operand layout (wave64): A[i][k] in lane i + 16k, B[k][j] in lane
// j + 16k. Result D[i][j], j = lane % 16: for f32 element e of lane l holds
// row 4(l/16) + e; for f64 it holds row l/16 + 4e (measured on gfx950).
__device__ __forceinline__ d4 mfma_16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_16x16x4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T>
struct Acc4;
template <>
struct Acc4<double> {
  typedef d4 type;
  __device__ static int row(int lk, int e) { return lk + 4 * e; }
};
template <>
struct Acc4<float> {
  typedef f4 type;
  __device__ static int row(int lk, int e) { return 4 * lk + e; }
};

constexpr int GEMM_KC = 32;      // K chunk of the matrix-core updates staged through LDS
constexpr int GEMM_TILE = 64;
constexpr int GEMM_TILE_R = 128;  // rows of the trailing-update tile (columns: GEMM_TILE)

// TM x TN tile of C; four waves in a 2 x 2 arrangement, each (TM/2) x (TN/2)
// as (TM/32) x (TN/32) blocks of 16 x 16. Every C element accumulates the same
// MFMA steps in the same order whatever the tile shape, so all shapes give
// the same bits. Returns whether this thread wrote a nonzero.
template <typename T, int TM = GEMM_TILE, int TN = GEMM_TILE>
__device__ __forceinline__ bool tile_update(T* a, int64_t lda, int rows, int cols, int kdim,
                                            int r0, int c0, const T* __restrict__ lsrc, int64_t lld,
                                            const T* usrc, int64_t uld) {
  // C[r0.., c0..] -= Lsrc[r0.., 0..kdim) * Usrc[0..kdim, c0..]   (C = a, rows x cols in view).
  // Usrc may be C itself when one tile covers all kdim rows (TM >= kdim, r0 = 0):
  // every read of Usrc comes before the tile's only write of C, at the end.
  constexpr int NBR = TM / 32, NBC = TN / 32;  // 16 x 16 blocks per wave
  __shared__ T Ls[TM][GEMM_KC + 1];
  __shared__ T Us[GEMM_KC][TN + 1];
  typedef typename Acc4<T>::type AT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * (TM / 2), wc = (wave & 1) * (TN / 2);
  const int li = lane & 15, lk = lane >> 4;
  AT acc[NBR][NBC];
  bool nz = false;
  // C element (bi, bj, i) of a lane: a row base that is the same for the whole
  // wave plus one byte offset per lane, so that every load and store of the
  // tile takes the scalar-base address form with the same offset register
  // (no address register is rewritten between the stores). Tiles wholly
  // inside the view skip the bounds tests.
  const int wru = __builtin_amdgcn_readfirstlane(wr), wcu = __builtin_amdgcn_readfirstlane(wc);
  const uint32_t loff = (uint32_t)(((int64_t)Acc4<T>::row(lk, 0) * lda + li) * (int64_t)sizeof(T));
  auto cbase = [&](int bi, int bj, int i) {
    return reinterpret_cast<char*>(a + (int64_t)(r0 + wru + bi * 16 + Acc4<T>::row(0, i)) * lda +
                                   (c0 + wcu + bj * 16));
  };
  const bool full = r0 + TM <= rows && c0 + TN <= cols;
  if (full) {
#pragma unroll
    for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBC; ++bj)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[bi][bj][i] = *reinterpret_cast<const T*>(cbase(bi, bj, i) + loff);
  } else {
#pragma unroll
    for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBC; ++bj)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int rr = r0 + wr + bi * 16 + Acc4<T>::row(lk, i), cc = c0 + wc + bj * 16 + li;
          acc[bi][bj][i] = (rr < rows && cc < cols) ? *reinterpret_cast<const T*>(cbase(bi, bj, i) + loff) : (T)0;
        }
  }
  // K in chunks of GEMM_KC, staged through LDS; the next chunk's loads are issued
  // into registers before the current chunk's matrix-core steps, so their
  // latency overlaps the arithmetic (nothing reads the loaded registers until
  // they are staged). Each load brings V consecutive elements of a row (16
  // bytes); a vector is loaded when its first element is in the tile, and its
  // elements past the tile's edge are zeroed as it is staged. The row starts
  // are V-aligned except for U sources that begin at an unaligned column (the
  // last outer block's right-hand columns), hence the element-aligned vector
  // type. Every vector read stays inside its matrix row or the next one: rows
  // are padded to a multiple of 16 columns, the L columns start V-aligned,
  // and U rows are never the matrix's last row.
  constexpr int V = 16 / (int)sizeof(T);
  typedef T VT __attribute__((ext_vector_type(V), aligned(sizeof(T))));
  constexpr int PL = TM * GEMM_KC / (256 * V), PU = GEMM_KC * TN / (256 * V);
  VT lreg[PL], ureg[PU];
  auto fetch = [&](int kc) {
    const int kb = min(GEMM_KC, kdim - kc);
#pragma unroll
    for (int t = 0; t < PL; ++t) {
      const int idx = (threadIdx.x + t * 256) * V;
      const int i = idx / GEMM_KC, qq = idx - (idx / GEMM_KC) * GEMM_KC;
      lreg[t] = (r0 + i < rows && qq < kb) ? *reinterpret_cast<const VT*>(lsrc + (int64_t)(r0 + i) * lld + kc + qq)
                                           : (VT)(T)0;
    }
#pragma unroll
    for (int t = 0; t < PU; ++t) {
      const int idx = (threadIdx.x + t * 256) * V;
      const int qq = idx / TN, jx = idx - (idx / TN) * TN;
      ureg[t] = (qq < kb && c0 + jx < cols) ? *reinterpret_cast<const VT*>(usrc + (int64_t)(kc + qq) * uld + c0 + jx)
                                             : (VT)(T)0;
    }
  };
  if (kdim > 0) fetch(0);
  for (int kc = 0; kc < kdim; kc += GEMM_KC) {
    const int kb = min(GEMM_KC, kdim - kc);
    // L is staged negated, so that the steps below add products
#pragma unroll
    for (int t = 0; t < PL; ++t)
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int idx = (threadIdx.x + t * 256) * V + e;
        const int qq = idx - (idx / GEMM_KC) * GEMM_KC;
        Ls[idx / GEMM_KC][qq] = qq < kb ? -lreg[t][e] : (T)0;
      }
#pragma unroll
    for (int t = 0; t < PU; ++t)
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int idx = (threadIdx.x + t * 256) * V + e;
        const int jx = idx - (idx / TN) * TN;
        Us[idx / TN][jx] = c0 + jx < cols ? ureg[t][e] : (T)0;
      }
    __syncthreads();
    if (kc + GEMM_KC < kdim) fetch(kc + GEMM_KC);
    const int ksteps = (kb + 3) >> 2;
    for (int kk = 0; kk < ksteps; ++kk) {
      T av[NBR], bv[NBC];
#pragma unroll
      for (int bi = 0; bi < NBR; ++bi) av[bi] = Ls[wr + bi * 16 + li][kk * 4 + lk];
#pragma unroll
      for (int bj = 0; bj < NBC; ++bj) bv[bj] = Us[kk * 4 + lk][wc + bj * 16 + li];
#pragma unroll
      for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
        for (int bj = 0; bj < NBC; ++bj) acc[bi][bj] = mfma_16x16x4(av[bi], bv[bj], acc[bi][bj]);
    }
    __syncthreads();
  }
  if (full) {
#pragma unroll
    for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBC; ++bj)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          *reinterpret_cast<T*>(cbase(bi, bj, i) + loff) = acc[bi][bj][i];
          nz |= acc[bi][bj][i] != (T)0;
        }
  } else {
#pragma unroll
    for (int bi = 0; bi < NBR; ++bi)
#pragma unroll
      for (int bj = 0; bj < NBC; ++bj)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int rr = r0 + wr + bi * 16 + Acc4<T>::row(lk, i), cc = c0 + wc + bj * 16 + li;
          if (rr < rows && cc < cols) {
            *reinterpret_cast<T*>(cbase(bi, bj, i) + loff) = acc[bi][bj][i];
            nz |= acc[bi][bj][i] != (T)0;
          }
        }
  }
  return nz;
}

// Whether rows [r, r + rows_n) meet the rows whose multipliers in the current
// outer block may be nonzero: A_j rows below hi[0] and border rows below hi[1]
// (hi[1] == n: none).
__device__ __forceinline__ bool rows_live(const int32_t* hi, int n, int r, int rows_n) {
  return r < hi[0] || (r + rows_n > n && r < hi[1] && hi[1] > n);
}

// One tile of a job's update per block (jobs located through the prefix of
// their tile counts); TM x TN the tile shape the host planned the job with.
// Tiles whose rows carry only zero multipliers (rowhi, as left by the
// panels) leave C as it is and return at once.
template <typename T, int TM = GEMM_TILE, int TN = GEMM_TILE>
__global__ __launch_bounds__(256) void k_lu_gemm(const SubDesc* __restrict__ desc, T* __restrict__ A,
                                                 const LuJob* __restrict__ jobs, const int32_t* __restrict__ prefix,
                                                 int n_jobs, const int32_t* __restrict__ rowhi,
                                                 unsigned long long* __restrict__ flops) {
  const int q = find_job(prefix, n_jobs, blockIdx.x);
  const LuJob jb = jobs[q];
  const SubDesc d = desc[jb.j];
  const int ncol = jb.c_hi - jb.c_lo;
  const int ntc = (ncol + TN - 1) / TN;
  const int tile = blockIdx.x - prefix[q];
  const int tr = tile / ntc, tc = tile - (tile / ntc) * ntc;
  if (!rows_live(rowhi + 2 * jb.j, d.n, jb.r_lo + tr * TM, TM)) return;
  if (threadIdx.x == 0) atomicAdd(flops, 2ull * TM * TN * (unsigned long long)jb.kdim);
  T* a = A + d.a_off;
  const int64_t lda = d.lda;
  // view with origin (r_lo, c_lo)
  tile_update<T, TM, TN>(a + (int64_t)jb.r_lo * lda + jb.c_lo, lda, d.rows - jb.r_lo, ncol, jb.kdim, tr * TM,
                         tc * TN, a + (int64_t)jb.r_lo * lda + jb.kstart, lda,
                         a + (int64_t)jb.kstart * lda + jb.c_lo, lda);
}

// The unit-lower solve of a full outer block as a matrix-core product: first
// Lm = I - L11^{-1} (strictly lower; L11^{-1} by forward substitution on the
// identity, 64 columns per block), written row-major, LU_KMAX x LU_KMAX per
// subdomain; then U12 -= Lm U12 in place (k_lu_gemm_u), i.e. U12 = L11^{-1} U12.
// Columns col = BASE + t (t < TRSM_COLS) of L11^{-1}, the column in
// registers (rows [BASE, LU_KMAX); the rows above BASE are zero for these
// columns), row i's sum formed as in row_dot4 (partial sum q mod 4, terms in
// q order): the terms q < BASE it skips are zero, and adding a zero leaves a
// partial sum's bits unchanged, so the results equal the full solve's. Rows
// of L11 from LDS. Writes Lm = I - L11^{-1} (strictly lower) as k_lu_linv.
template <typename T, int BASE>
__device__ __forceinline__ void linv_columns(const T (*Ls)[LU_KMAX], int col, int kd, T* __restrict__ out) {
  constexpr int KD = LU_KMAX - BASE;
  T x[KD];
#pragma unroll
  for (int i = BASE; i < LU_KMAX; ++i) {
    T s0 = (T)0, s1 = (T)0, s2 = (T)0, s3 = (T)0;
#pragma unroll
    for (int q = BASE; q < i; ++q) {
      if ((q & 3) == 0) s0 += Ls[i][q] * x[q - BASE];
      else if ((q & 3) == 1) s1 += Ls[i][q] * x[q - BASE];
      else if ((q & 3) == 2) s2 += Ls[i][q] * x[q - BASE];
      else s3 += Ls[i][q] * x[q - BASE];
    }
    x[i - BASE] = (i == col ? (T)1 : (T)0) - ((s0 + s1) + (s2 + s3));
  }
#pragma unroll
  for (int i = 0; i < LU_KMAX; ++i)
    out[(int64_t)i * LU_KMAX + col] = (i >= BASE && i < kd && col < kd && i > col) ? -x[i >= BASE ? i - BASE : 0] : (T)0;
}

template <typename T>
__global__ __launch_bounds__(TRSM_COLS) void k_lu_linv(const SubDesc* __restrict__ desc, const T* __restrict__ A,
                                                       const LuJob* __restrict__ jobs,
                                                       const int32_t* __restrict__ prefix, int n_jobs,
                                                       T* __restrict__ lm, int32_t* __restrict__ n_tiles) {
  static_assert(LU_KMAX == 2 * TRSM_COLS, "two column blocks per L11");
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_tiles = 0;  // the trailing-tile list of this outer block starts empty
  const int q = find_job(prefix, n_jobs, blockIdx.x);
  const LuJob jb = jobs[q];
  const SubDesc d = desc[jb.j];
  const int t = threadIdx.x;
  const int cb = blockIdx.x - prefix[q];  // column block: 0 or 1
  const int col = cb * TRSM_COLS + t;     // < LU_KMAX
  const int kd = jb.kdim;
  const int64_t lda = d.lda;
  const T* l = A + d.a_off + (int64_t)jb.kstart * lda + jb.kstart;
  T* out = lm + (int64_t)jb.j * LU_KMAX * LU_KMAX;
  if constexpr (sizeof(T) == 4) {
    // FP32: L11 staged (sixteen rows' coalesced loads in flight together),
    // the column in registers (2x faster; in FP64 the 128-value column needs
    // more registers than a wave has and the form below is faster)
    __shared__ T Ls[LU_KMAX][LU_KMAX];  // strictly lower L11 (rows past kdim zero)
    for (int i0 = 0; i0 < LU_KMAX; i0 += 16) {
      T g[16][2];
#pragma unroll
      for (int u = 0; u < 16; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i = i0 + u, qq = t + h * TRSM_COLS;
          g[u][h] = (i < kd && qq < i) ? l[(int64_t)i * lda + qq] : (T)0;
        }
#pragma unroll
      for (int u = 0; u < 16; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) Ls[i0 + u][t + h * TRSM_COLS] = g[u][h];
    }
    __syncthreads();
    if (cb == 0)
      linv_columns<T, 0>(Ls, col, kd, out);
    else
      linv_columns<T, TRSM_COLS>(Ls, col, kd, out);
  } else {
    // forward substitution by rows on the identity column, reading row i of
    // L11 contiguously, the column in LDS
    __shared__ T X[LU_KMAX][TRSM_COLS];
    for (int i = 0; i < kd; ++i) {
      const T x = (i == col ? (T)1 : (T)0) - row_dot4<T>(l + (int64_t)i * lda, X, i, t);
      X[i][t] = x;
    }
    for (int i = 0; i < LU_KMAX; ++i)
      out[(int64_t)i * LU_KMAX + col] = (i < kd && col < kd && i > col) ? -X[i][t] : (T)0;
  }
}

// U12 = L11^{-1} U12 for one GEMM_TILE-column tile. When the tile is not all
// zero, the tiles of the trailing update below it whose rows may carry nonzero
// multipliers (rowhi) are appended to `list` as (job, tile) pairs: tile =
// tr * ntc + tc for TR-row tiles. The trailing update of a tile with a zero
// U12 or zero multipliers changes nothing, so only listed tiles are computed.
template <typename T>
__global__ __launch_bounds__(256) void k_lu_gemm_u(const SubDesc* __restrict__ desc, T* __restrict__ A,
                                                   const LuJob* __restrict__ jobs,
                                                   const int32_t* __restrict__ prefix, int n_jobs,
                                                   const T* __restrict__ lm, const int32_t* __restrict__ rowhi,
                                                   int TR, int2* __restrict__ list, int32_t* __restrict__ n_tiles,
                                                   unsigned long long* __restrict__ flops) {
  __shared__ int base_s;
  const int q = find_job(prefix, n_jobs, blockIdx.x);
  const LuJob jb = jobs[q];
  const SubDesc d = desc[jb.j];
  const int ncol = jb.c_hi - jb.c_lo;
  const int tc = blockIdx.x - prefix[q];
  T* u = A + d.a_off + (int64_t)jb.kstart * d.lda + jb.c_lo;  // the U12 block, rows [kstart, kstart + kdim)
  const bool nz = tile_update<T, LU_KMAX, GEMM_TILE>(u, d.lda, jb.kdim, ncol, jb.kdim, 0, tc * GEMM_TILE,
                                                     lm + (int64_t)jb.j * LU_KMAX * LU_KMAX, LU_KMAX, u, d.lda);
  if (!__syncthreads_or(nz)) return;
  // trailing rows [K1, rows), K1 = c_lo, in TR-row tiles: A_j rows below
  // rowhi[0] and border rows below rowhi[1]
  const int K1 = jb.c_lo;
  const int ntr = (d.rows - K1 + TR - 1) / TR;
  const int ntc = (ncol + GEMM_TILE - 1) / GEMM_TILE;
  const int hia = rowhi[2 * jb.j], hib = rowhi[2 * jb.j + 1];
  const int a_hi = hia > K1 ? min(ntr, (hia - K1 + TR - 1) / TR) : 0;
  const int b_lo = max(a_hi, (d.n - K1) / TR);
  const int b_hi = hib > d.n ? min(ntr, (hib - K1 + TR - 1) / TR) : 0;
  const int cnt = a_hi + max(0, b_hi - b_lo);
  if (threadIdx.x == 0) {
    base_s = atomicAdd(n_tiles, cnt);
    // matrix-core work of the listed tiles (whole tiles, as computed)
    atomicAdd(flops, (unsigned long long)cnt * 2ull * TR * GEMM_TILE * (unsigned long long)jb.kdim);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
    const int tr = e < a_hi ? e : b_lo + (e - a_hi);
    list[base_s + e] = make_int2(q, tr * ntc + tc);
  }
}

// Trailing update A22 -= L21 U12 of an outer block over the listed tiles
// (k_lu_gemm_u), a persistent grid (gridDim.x a multiple of 8); `jobs` are
// the U12 jobs (rows of the trailing update start at K1 = c_lo). Workgroups go
// to the 8 XCDs in turn, so XCD x = blockIdx.x % 8 takes the x-th contiguous
// eighth of the list: the tiles of a U12 column tile (listed together) and of
// neighbouring column tiles share their L2.
template <typename T, int TM, int TN>
__global__ __launch_bounds__(256, 2) void k_lu_gemm_list(const SubDesc* __restrict__ desc, T* __restrict__ A,
                                                      const LuJob* __restrict__ jobs,
                                                      const int2* __restrict__ list,
                                                      const int32_t* __restrict__ n_tiles) {
  const int nt = *n_tiles;
  const int x = blockIdx.x & 7, per = gridDim.x >> 3;
  const int q = (nt + 7) >> 3;  // entries per XCD
  for (int v = blockIdx.x >> 3; v < q; v += per) {
    const int e = x * q + v;
    if (e >= nt) break;
    const int2 it = list[e];
    const LuJob jb = jobs[it.x];
    const SubDesc d = desc[jb.j];
    const int K1 = jb.c_lo;
    const int ncol = jb.c_hi - K1;
    const int ntc = (ncol + TN - 1) / TN;
    const int tr = it.y / ntc, tc = it.y - (it.y / ntc) * ntc;
    T* a = A + d.a_off;
    const int64_t lda = d.lda;
    tile_update<T, TM, TN>(a + (int64_t)K1 * lda + K1, lda, d.rows - K1, ncol, jb.kdim, tr * TM, tc * TN,
                           a + (int64_t)K1 * lda + jb.kstart, lda, a + (int64_t)jb.kstart * lda + K1, lda);
  }
}

// Self-test of the matrix-core tile: C (64x64) -= A (64 x kdim) B (kdim x 64), row-major.
template <typename T>
__global__ __launch_bounds__(256) void k_tile_selftest(T* C, const T* Am, const T* Bm, int kdim) {
  tile_update<T>(C, GEMM_TILE, GEMM_TILE, GEMM_TILE, kdim, 0, 0, Am, LU_KMAX, Bm, GEMM_TILE);
}

// W_j = -(lower-right block) of the eliminated augmented matrix, written in the
// tiled layout of the apply kernels (w_tile_index).
// Row q of W_j (Sigma~_j in band order) is border row wrow[q]; column c
// (Sigma_j in band order) is right-hand column wcol[c].
template <typename T>
__global__ __launch_bounds__(256) void k_extract_w(const SubDesc* __restrict__ desc, const T* __restrict__ A,
                                                   const int32_t* __restrict__ wrow, const int32_t* __restrict__ wcol,
                                                   T* __restrict__ W) {
  const int j = blockIdx.y;
  const SubDesc d = desc[j];
  const int q = blockIdx.x;
  if (q >= d.t) return;
  const T* src = A + d.a_off + (int64_t)(d.n + wrow[d.t_off + q]) * d.lda + d.n;
  const int32_t* wc = wcol + d.u_off;
  T* dst = W + d.w_off;
  for (int c = threadIdx.x; c < d.ldw; c += 256)
    dst[w_tile_index(d.ldw, W_CW<T>, q, c)] = c < d.m ? -src[wc[c]] : (T)0;
}

// ---------------------------------------------------------------------------
// Krylov kernels (FGMRES with classical Gram-Schmidt applied twice). Every
// reduction is two-stage with a fixed order: a pass kernel writes one partial
// sum per block and column, a reduction kernel (one block per column) adds
// them in block order, so results are reproducible run to run. Each thread
// owns one row and keeps that row of the basis in registers, so the fused
// "w -= V h, then V^T w" pass reads V once.
// ---------------------------------------------------------------------------
// Per-right-hand-side strides of the batched Krylov kernels (blockIdx.y = the
// right-hand side; all zero with a one-row grid for a single solve).
struct BatchStrides {
  int64_t v = 0;      // basis V (and w, a column of it)
  int64_t z = 0;      // preconditioned basis Z
  int64_t e = 0;      // extension scratch
  int64_t part = 0;   // partial sums
  int64_t small = 0;  // small buffer (H, rotations, scalars)
  int64_t slot = 0;   // host slots
};

constexpr int RED_THREADS = 256;
constexpr int MAX_BASIS = 64;       // restart length limit (columns of V per pass)
constexpr int RED_MAX_BLOCKS = 4096;
constexpr int PART_LD = MAX_BASIS;  // partial-sum stride per block

inline int red_blocks(int64_t n) {
  const int64_t b = (n + RED_THREADS - 1) / RED_THREADS;
  return (int)(b < RED_MAX_BLOCKS ? (b < 1 ? 1 : b) : RED_MAX_BLOCKS);
}

// Layout of the small device buffer (doubles).
struct SmallLayout {
  int m;
  __host__ __device__ int H() const { return 0; }                    // (m+1) x m, column-major
  __host__ __device__ int cs() const { return (m + 1) * m; }
  __host__ __device__ int sn() const { return cs() + m; }
  __host__ __device__ int g() const { return sn() + m; }             // m+1
  __host__ __device__ int y() const { return g() + m + 1; }          // m
  __host__ __device__ int h1() const { return y() + m; }             // m+1
  __host__ __device__ int h2() const { return h1() + m + 1; }        // m+1
  __host__ __device__ int scal() const { return h2() + m + 1; }      // 8 scalars
  __host__ __device__ int size() const { return scal() + 8; }
};
// scal[]: residual estimate, ||w||, 1/||w|| (scale of the newest basis vector), ||r|| at the cycle start
enum { S_EST = 0, S_HK1 = 1, S_INV = 2, S_BETA = 3, S_NSCAL = 8 };

// Scalars handed to the host through mapped pinned memory: the values, then
// (after a system-scope fence) the ticket the host waits for.
struct HostSlot {
  double v[8];
  unsigned long long ticket;
  unsigned long long pad[7];
};

__device__ __forceinline__ void publish(HostSlot* slot, unsigned long long ticket, const double* scal) {
  if (!slot) return;
#pragma unroll
  for (int q = 0; q < 8; ++q) slot->v[q] = scal[q];
  __threadfence_system();
  *(volatile unsigned long long*)&slot->ticket = ticket;
}

// Block partial sums of acc[0..nc) (one value per thread and column) into part[blk][j0 + j].
template <int NC>
__device__ __forceinline__ void block_partials(const double (&acc)[NC], int j0, int nc, double* __restrict__ part) {
  __shared__ double red[RED_THREADS / 64][NC];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    if (u < nc) {
      const double t = wave_sum(acc[u]);
      if (lane == 0) red[wave][u] = t;
    }
  }
  __syncthreads();
  for (int u = threadIdx.x; u < nc; u += RED_THREADS) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < RED_THREADS / 64; ++q) s += red[q][u];
    part[(int64_t)blockIdx.x * PART_LD + j0 + u] = s;
  }
  __syncthreads();
}

// block_partials for 32 accumulators per thread (acc is consumed).
__device__ __forceinline__ void block_partials32(double (&acc)[32], int j0, int nc, double* __restrict__ part) {
  if (nc <= 2) {
    block_partials<2>(reinterpret_cast<const double(&)[2]>(acc), j0, nc, part);
    return;
  }
  __shared__ double red[RED_THREADS / 64][32];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double t = wave_sum_many<32>(acc, lane);  // lanes 2c and 2c + 1: column c
  if ((lane & 1) == 0) red[wave][lane >> 1] = t;
  __syncthreads();
  if (threadIdx.x < nc) {
    const int u = threadIdx.x;
    part[(int64_t)blockIdx.x * PART_LD + j0 + u] = (red[0][u] + red[1][u]) + (red[2][u] + red[3][u]);
  }
  __syncthreads();
}

// acc[u] += X[j0 + u][r] wr for u < nc (nc <= 32), the column scale_col (when
// in [j0, j0 + nc)) first multiplied by sc and written back. Columns are read
// eight at a time with all eight loads issued before any use (a group's last
// columns past nc repeat its first and feed accumulators that are never
// reported), and the one write comes after the reads, so the loads of a row
// are in flight together instead of one round trip per column.
__device__ __forceinline__ void row_dots(double (&acc)[32], double* __restrict__ X, int64_t ldx, int64_t r, int j0,
                                         int nc, double wr, int scale_col, double sc) {
  double xs = 0.0;
#pragma unroll
  for (int g = 0; g < 32; g += 8) {
    if (g < nc) {
      double xv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) xv[q] = X[(int64_t)(j0 + (g + q < nc ? g + q : g)) * ldx + r];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        double x = xv[q];
        if (j0 + g + q == scale_col) {
          x *= sc;
          xs = x;
        }
        acc[g + q] += x * wr;
      }
    }
  }
  if (scale_col >= j0 && scale_col < j0 + nc) X[(int64_t)scale_col * ldx + r] = xs;
}

// part[blk][j] = sum over the block's rows of X_j[r] w[r], j < ncols. With
// `scale_col` >= 0 that column of X is first scaled in place by *scale.
__global__ __launch_bounds__(RED_THREADS) void k_dots(int64_t n, double* __restrict__ X, int64_t ldx, int ncols,
                                                      const double* __restrict__ w, double* __restrict__ part,
                                                      int scale_col, const double* __restrict__ scale) {
  constexpr int NC = 32;
  const double sc = scale_col >= 0 ? *scale : 1.0;
  for (int j0 = 0; j0 < ncols; j0 += NC) {
    const int nc = min(NC, ncols - j0);
    double acc[NC];
#pragma unroll
    for (int u = 0; u < NC; ++u) acc[u] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; r < n; r += (int64_t)gridDim.x * RED_THREADS)
      row_dots(acc, X, ldx, r, j0, nc, w[r], scale_col, sc);
    block_partials32(acc, j0, nc, part);
  }
}

// Operator apply fused with the first Gram-Schmidt pass: w = diag z - ih2 sum_nb e[nb]
// (the stencil of k_stencil, same arithmetic), then part = X^T w as in k_dots.
__global__ __launch_bounds__(RED_THREADS) void k_stencil_dots(int64_t n, double diag, double ih2,
                                                              const int32_t* __restrict__ nbr,
                                                              const double* __restrict__ z,
                                                              const double* __restrict__ e, double* __restrict__ w,
                                                              double* __restrict__ X, int64_t ldx, int ncols,
                                                              double* __restrict__ part, int scale_col,
                                                              const double* __restrict__ scale, BatchStrides bs) {
  constexpr int NC = 32;
  const int64_t b = blockIdx.y;  // right-hand side of a batch
  z += b * bs.z;
  e += b * bs.e;
  w += b * bs.v;
  X += b * bs.v;
  part += b * bs.part;
  const double sc = scale_col >= 0 ? scale[b * bs.small] : 1.0;
  for (int j0 = 0; j0 < ncols; j0 += NC) {
    const int nc = min(NC, ncols - j0);
    double acc[NC];
#pragma unroll
    for (int u = 0; u < NC; ++u) acc[u] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; r < n; r += (int64_t)gridDim.x * RED_THREADS) {
      double wr;
      if (j0 == 0) {
        const double s = (e[nbr[r]] + e[nbr[n + r]]) + (e[nbr[2 * n + r]] + e[nbr[3 * n + r]]) +
                         (e[nbr[4 * n + r]] + e[nbr[5 * n + r]]);
        wr = diag * z[r] - ih2 * s;
        w[r] = wr;
      } else {
        wr = w[r];
      }
      row_dots(acc, X, ldx, r, j0, nc, wr, scale_col, sc);
    }
    block_partials32(acc, j0, nc, part);
  }
}

// w -= V[0..k] h (h: k+1 values), then part = V^T w (mode 0) or ||w||^2 (mode 1).
__global__ __launch_bounds__(RED_THREADS) void k_axpy_dots(int64_t n, const double* __restrict__ V, int64_t ld, int k,
                                                           const double* __restrict__ h, double* __restrict__ w,
                                                           double* __restrict__ part, int mode, BatchStrides bs) {
  constexpr int NC = 32;
  const int64_t b = blockIdx.y;  // right-hand side of a batch
  V += b * bs.v;
  w += b * bs.v;
  h += b * bs.small;
  part += b * bs.part;
  __shared__ double hs[MAX_BASIS];
  for (int q = threadIdx.x; q <= k; q += RED_THREADS) hs[q] = h[q];
  __syncthreads();
  const int ncols = k + 1;
  if (ncols <= NC) {
    double acc[NC];
#pragma unroll
    for (int u = 0; u < NC; ++u) acc[u] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; r < n; r += (int64_t)gridDim.x * RED_THREADS) {
      // s = sum_u V[u][r] h[u] in u order, the row read eight columns at a
      // time with the group's loads issued before any use (as in row_dots)
      double s = 0.0;
#pragma unroll
      for (int g = 0; g < NC; g += 8) {
        if (g < ncols) {
          double xv[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) xv[q] = V[(int64_t)(g + q < ncols ? g + q : g) * ld + r];
#pragma unroll
          for (int q = 0; q < 8; ++q)
            if (g + q < ncols) s += xv[q] * hs[g + q];
        }
      }
      const double wn = w[r] - s;
      w[r] = wn;
      if (mode == 0) {
        // The row of V is read again (from cache) rather than kept in 32 more
        // registers: the kernel then fits 4 waves per SIMD, so the whole grid
        // is resident in one round. The compiler barrier keeps the two reads
        // apart.
        asm volatile("" ::: "memory");
        row_dots(acc, const_cast<double*>(V), ld, r, 0, ncols, wn, -1, 1.0);  // no column is written
      } else {
        acc[0] += wn * wn;
      }
    }
    block_partials32(acc, 0, mode == 0 ? ncols : 1, part);
    return;
  }
  // long bases: two sweeps over V
  for (int64_t r = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; r < n; r += (int64_t)gridDim.x * RED_THREADS) {
    double s = 0.0;
    for (int q = 0; q < ncols; ++q) s += V[(int64_t)q * ld + r] * hs[q];
    w[r] -= s;
  }
  if (mode == 0) {
    for (int j0 = 0; j0 < ncols; j0 += NC) {
      const int nc = min(NC, ncols - j0);
      double acc[NC];
#pragma unroll
      for (int u = 0; u < NC; ++u) acc[u] = 0.0;
      for (int64_t r = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; r < n;
           r += (int64_t)gridDim.x * RED_THREADS)
        row_dots(acc, const_cast<double*>(V), ld, r, j0, nc, w[r], -1, 1.0);  // no column is written
      block_partials32(acc, j0, nc, part);
    }
  } else {
    double acc[1] = {0.0};
    for (int64_t r = (int64_t)blockIdx.x * RED_THREADS + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * RED_THREADS)
      acc[0] += w[r] * w[r];
    block_partials<1>(acc, 0, 1, part);
  }
}

// out[j] = sum_b part[b][j], one block per column, fixed order.
__device__ __forceinline__ double column_total(const double* __restrict__ part, int nblocks, int j) {
  __shared__ double red[RED_THREADS / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) s += part[(int64_t)b * PART_LD + j];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(RED_THREADS) void k_reduce_cols(const double* __restrict__ part, int nblocks,
                                                             double* __restrict__ out, BatchStrides bs) {
  part += blockIdx.y * bs.part;  // right-hand side of a batch
  out += blockIdx.y * bs.small;
  const double t = column_total(part, nblocks, blockIdx.x);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// ||x|| from partials: scal[S_BETA] = ||x||, scal[S_INV] = 1/||x|| (0 if zero),
// g = (||x||, 0, ..., 0); published to the host.
__global__ __launch_bounds__(RED_THREADS) void k_norm_finish(const double* __restrict__ part, int nblocks,
                                                             SmallLayout L, double* __restrict__ sm,
                                                             HostSlot* slot, unsigned long long ticket) {
  const double nr = sqrt(column_total(part, nblocks, 0));
  double* scal = sm + L.scal();
  for (int i = threadIdx.x; i <= L.m; i += RED_THREADS) sm[L.g() + i] = i == 0 ? nr : 0.0;
  if (threadIdx.x == 0) {
    scal[S_BETA] = nr;
    scal[S_INV] = nr > 0.0 ? 1.0 / nr : 0.0;
    publish(slot, ticket, scal);
  }
}

// Arnoldi column k: H[:,k] = h1 + h2, H[k+1,k] = ||w|| (from partials), the
// Givens update of the least-squares problem and the residual estimate
// |g[k+1]|; published to the host. The column and the rotations are staged in
// LDS so that the serial rotation sweep does not wait on device memory.
__global__ __launch_bounds__(RED_THREADS) void k_arnoldi(const double* __restrict__ part, int nblocks, int k,
                                                         SmallLayout L, double* __restrict__ sm, HostSlot* slot,
                                                         unsigned long long ticket, BatchStrides bs) {
  __shared__ double hc[MAX_BASIS + 2], csl[MAX_BASIS], snl[MAX_BASIS];
  part += blockIdx.y * bs.part;  // right-hand side of a batch
  sm += blockIdx.y * bs.small;
  if (slot) slot += blockIdx.y * bs.slot;
  const double tot = column_total(part, nblocks, 0);
  const int ldh = L.m + 1;
  double* H = sm + L.H() + (int64_t)k * ldh;
  double* cs = sm + L.cs();
  double* sn = sm + L.sn();
  double* g = sm + L.g();
  double* scal = sm + L.scal();
  for (int i = threadIdx.x; i <= k; i += RED_THREADS) hc[i] = sm[L.h1() + i] + sm[L.h2() + i];
  for (int i = threadIdx.x; i < k; i += RED_THREADS) {
    csl[i] = cs[i];
    snl[i] = sn[i];
  }
  __syncthreads();
  const double hk1 = sqrt(tot);
  if (threadIdx.x == 0) {
    double a = hc[0];  // rotated H[i] carried down the column
    for (int i = 0; i < k; ++i) {
      const double b = hc[i + 1];
      hc[i] = csl[i] * a + snl[i] * b;
      a = -snl[i] * a + csl[i] * b;
    }
    const double den = hypot(a, hk1);
    const double c = a / den, sr = hk1 / den;
    cs[k] = c;
    sn[k] = sr;
    hc[k] = den;
    hc[k + 1] = 0.0;
    const double gk = g[k];
    g[k + 1] = -sr * gk;
    g[k] = c * gk;
    scal[S_EST] = fabs(-sr * gk);
    scal[S_HK1] = hk1;
    scal[S_INV] = hk1 > 0.0 ? 1.0 / hk1 : 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= k + 1; i += RED_THREADS) H[i] = hc[i];
  __syncthreads();
  if (threadIdx.x == 0) publish(slot, ticket, scal);
}

// y = H[0:kk, 0:kk]^{-1} g[0:kk] (upper triangular after the rotations)
__global__ void k_backsolve(int kk, SmallLayout L, double* __restrict__ sm) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int ld = L.m + 1;
  const double* H = sm + L.H();
  double* y = sm + L.y();
  const double* g = sm + L.g();
  for (int i = kk - 1; i >= 0; --i) {
    double s = g[i];
    for (int q = i + 1; q < kk; ++q) s -= H[i + q * ld] * y[q];
    y[i] = s / H[i + i * ld];
  }
}

__global__ __launch_bounds__(256) void k_update_x(int64_t n, const double* __restrict__ Z, int64_t ldz, int kk,
                                                  const double* __restrict__ y, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int q = 0; q < kk; ++q) s += Z[q * ldz + i] * y[q];
  x[i] += s;
}

__global__ __launch_bounds__(256) void k_axpy(int64_t n, const double* __restrict__ z, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += z[i];
}

__global__ __launch_bounds__(256) void k_scale(int64_t n, double a, const double* __restrict__ x,
                                               double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

__global__ __launch_bounds__(256) void k_fill(int64_t n, double* __restrict__ x, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ __launch_bounds__(256) void k_copy(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

}  // namespace cpm

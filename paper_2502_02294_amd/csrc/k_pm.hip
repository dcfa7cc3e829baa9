// Particle-mesh kernels (Sec. 2.2): cell keys, a stable counting sort of the particles by
// their CIC base cell, the deterministic CIC deposit as a per-cell gather over the bins
// that can reach a cell, the mesh acceleration g = -grad(phi) (two-point central
// difference) and its CIC read-out, kick and drift (eq. dm_hamil: dx/dt = p/a^2,
// dp/dt = g), and the adjoints of all of them.
//
// CIC on cell centres: with s = x - 1/2, i0 = floor(s), w1 = s - i0, a particle puts
// weight (1-w1) in cell i0 and w1 in i0+1 per axis.  Cell c receives from particles whose
// base cell is c - o, o in {0,1}^3.  After the sort, the positions are gathered into bin
// order (float4 per particle); the deposit sums each bin's 8 corner weights in LDS and each
// cell adds its 8 corners, in a fixed order and with ascending particle id inside a bin:
// every sum is reproducible bit for bit without float atomics.
#include "dh_kernels.h"

namespace dh {

namespace {

constexpr int kScanThreads = 256;
constexpr int kLargeSortBlocks = 1024;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanThreads * kScanPer;

__device__ __forceinline__ int wrapi(int j, int n) { return j & (n - 1); }

struct Cic {
  int i0[3];
  float w1[3];
};

__device__ __forceinline__ Cic cic_of(float x, float y, float z, int n) {
  Cic c;
  const float v[3] = {x, y, z};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float s = v[d] - 0.5f;
    const float f = floorf(s);
    c.w1[d] = s - f;
    c.i0[d] = wrapi(static_cast<int>(f), n);
  }
  return c;
}

__device__ __forceinline__ float w1_of(float x) {
  const float s = x - 0.5f;
  return s - floorf(s);
}

__device__ __forceinline__ float wsel(float w1, int o) { return o ? w1 : 1.0f - w1; }

// acc[o] += val prod_d (o_d ? w1_d : 1 - w1_d), o = ox + 2 oy + 4 oz: the products are formed
// from z outwards, wx_o (wy_o (wz_o val)), so the 8 corners share their y-z factors (the
// vector deposit; the density deposit keeps its products (wx wy) wz, for which the compiler
// already shares the x-y factors: the shared form issues no fewer instructions there).
__device__ __forceinline__ void add_corners(float wx, float wy, float wz, float val,
                                            float (&acc)[8]) {
  const float z0 = (1.0f - wz) * val, z1 = wz * val;
  const float yz[4] = {(1.0f - wy) * z0, wy * z0, (1.0f - wy) * z1, wy * z1};
#pragma unroll
  for (int o = 0; o < 8; ++o) acc[o] = fmaf(wsel(wx, o & 1), yz[o >> 1], acc[o]);
}

// bin of particle i of sample s: s n^3 + CIC base cell
__device__ __forceinline__ uint32_t bin_of(const Cic& c, int n, int smp, long long nc) {
  return static_cast<uint32_t>(smp * nc + (c.i0[2] * n + c.i0[1]) * n + c.i0[0]);
}

__global__ void keys_kernel(const float* __restrict__ pos, uint32_t* __restrict__ key, int n,
                            long long np) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= np) return;
  pos += blockIdx.y * 3 * np;
  const Cic c = cic_of(pos[i], pos[np + i], pos[2 * np + i], n);
  key[blockIdx.y * np + i] = bin_of(c, n, blockIdx.y, np);
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, long long count) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ void hist_kernel(const uint32_t* __restrict__ key, uint32_t* count,
                            uint32_t* __restrict__ rank, long long np) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= np) return;
  rank[i] = atomicAdd(&count[key[i]], 1u);
}

// Scans of the bin counts: 32-bit integer sums, so the grouping does not change a result.
static_assert(kScanThreads == 256, "the block scans below assume four waves");

// inclusive scan over the 64 lanes of a wave
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

// Block-wide exclusive scan over kScanThreads values; sh holds the four wave totals.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
  const uint32_t inc = wave_inclusive_scan(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) sh[w] = inc;
  __syncthreads();
  uint32_t below = 0;
  total = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t t = sh[k];
    below += k < w ? t : 0u;
    total += t;
  }
  __syncthreads();   // sh is free again on return
  return below + inc - v;
}

// tile element e lives at LDS word e + e / kScanPer (padding breaks the 16-word stride)
__device__ __forceinline__ int tile_slot(int e) { return e + e / kScanPer; }

__global__ void __launch_bounds__(kScanThreads) scan_reduce_kernel(
    const uint32_t* __restrict__ in, uint32_t* __restrict__ block_sums, long long count) {
  __shared__ uint32_t sh[4];
  const long long base = static_cast<long long>(blockIdx.x) * kScanTile;
  uint32_t s = 0;
  if (base + kScanTile <= count) {
    // whole tile: 16-byte loads, consecutive threads on consecutive vectors
    const uint4* in4 = reinterpret_cast<const uint4*>(in + base);
#pragma unroll
    for (int k = 0; k < kScanPer / 4; ++k) {
      const uint4 v = in4[k * kScanThreads + threadIdx.x];
      s += v.x + v.y + v.z + v.w;
    }
  } else {
    for (int k = 0; k < kScanPer; ++k) {
      const long long e = base + k * kScanThreads + threadIdx.x;
      if (e < count) s += in[e];
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) block_sums[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Exclusive scan of the nb block sums in place, one workgroup: each thread takes kScanPer
// consecutive sums per round of kScanTile.
__global__ void __launch_bounds__(kScanThreads) scan_block_sums_kernel(uint32_t* sums, int nb) {
  __shared__ uint32_t sh[4];
  uint32_t carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kScanTile) {
    const int i0 = b0 + threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      v[k] = i0 + k < nb ? sums[i0 + k] : 0u;
      s += v[k];
    }
    uint32_t total;
    uint32_t run = carry + block_exclusive_scan(s, sh, total);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      if (i0 + k < nb) sums[i0 + k] = run;
      run += v[k];
    }
    carry += total;
  }
}

__global__ void __launch_bounds__(kScanThreads) scan_final_kernel(
    const uint32_t* __restrict__ in, const uint32_t* __restrict__ block_off,
    uint32_t* __restrict__ out, long long count) {
  __shared__ uint32_t tile[kScanTile + kScanTile / kScanPer];
  __shared__ uint32_t sh[4];
  const long long base = static_cast<long long>(blockIdx.x) * kScanTile;
  for (int k = 0; k < kScanPer; ++k) {
    const int e = k * kScanThreads + threadIdx.x;
    tile[tile_slot(e)] = base + e < count ? in[base + e] : 0u;
  }
  __syncthreads();
  uint32_t s = 0;
  for (int k = 0; k < kScanPer; ++k) s += tile[tile_slot(threadIdx.x * kScanPer + k)];
  uint32_t total;
  uint32_t run = block_exclusive_scan(s, sh, total) + block_off[blockIdx.x];
  for (int k = 0; k < kScanPer; ++k) {
    const int sl = tile_slot(threadIdx.x * kScanPer + k);
    const uint32_t v = tile[sl];
    tile[sl] = run;
    run += v;
  }
  __syncthreads();
  for (int k = 0; k < kScanPer; ++k) {
    const int e = k * kScanThreads + threadIdx.x;
    if (base + e < count) out[base + e] = tile[tile_slot(e)];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[count] = block_off[blockIdx.x] + total;
}

__global__ void scatter_kernel(const uint32_t* __restrict__ key, const uint32_t* __restrict__ rank,
                               const uint32_t* __restrict__ start, uint32_t* __restrict__ sorted,
                               long long np) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= np) return;
  sorted[start[key[i]] + rank[i]] = static_cast<uint32_t>(i);
}

// The atomics above fix each bin's size but not the order inside it; sorting each bin's ids
// ascending makes the layout a pure function of the keys.  A thread sorts a bin of up to 8
// ids with a sorting network in registers, of up to kSmallBin ids by insertion; larger bins (dense halos gather thousands of particles in a
// cell) go to a list that bin_sort_large_kernel sorts one workgroup per bin.  (Moving the
// positions along with the ids, in place of the gather pass after the sort, was slower: the
// scattered 16-byte writes cost more than the gather's scattered reads.)
constexpr uint32_t kSmallBin = 32;
constexpr int kLdsSort = 16384;   // ids a workgroup sorts in LDS (64 KB)

// Batcher's odd-even merge network for 8 keys (19 compare-exchanges)
__device__ __forceinline__ void sort8(uint32_t (&v)[8]) {
  constexpr int kNet[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6},
                               {5, 7}, {1, 2}, {5, 6}, {0, 4}, {1, 5}, {2, 6}, {3, 7},
                               {2, 4}, {3, 5}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
  for (int k = 0; k < 19; ++k) {
    const uint32_t a = v[kNet[k][0]], b = v[kNet[k][1]];
    v[kNet[k][0]] = min(a, b);
    v[kNet[k][1]] = max(a, b);
  }
}

__global__ void bin_sort_kernel(const uint32_t* __restrict__ start, uint32_t* sorted,
                                long long nbins, uint32_t* __restrict__ large) {
  const long long b = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  const uint32_t lo = start[b], hi = start[b + 1];
  const uint32_t cnt = hi - lo;
  if (cnt > kSmallBin) {
    // large[0] counts the entries large[1..]; the list order does not affect the result
    large[1 + atomicAdd(&large[0], 1u)] = static_cast<uint32_t>(b);
    return;
  }
  if (cnt < 2) return;
  if (cnt <= 8) {
    // independent loads, a sorting network in registers (the padding sorts last)
    uint32_t v[8];
#pragma unroll
    for (uint32_t i = 0; i < 8; ++i) v[i] = i < cnt ? sorted[lo + i] : 0xFFFFFFFFu;
    sort8(v);
#pragma unroll
    for (uint32_t i = 0; i < 8; ++i)
      if (i < cnt) sorted[lo + i] = v[i];
    return;
  }
  for (uint32_t i = lo + 1; i < hi; ++i) {
    const uint32_t v = sorted[i];
    uint32_t j = i;
    while (j > lo && sorted[j - 1] > v) {
      sorted[j] = sorted[j - 1];
      --j;
    }
    sorted[j] = v;
  }
}

// Ascending bitonic network over p = 2^m slots of which the first k hold data and the rest
// count as +infinity: every compare-exchange orders a lower index before a higher one (the
// first stage of each merge pairs i with its mirror), so a slot >= k is never written.
template <typename Get, typename Put>
__device__ void bitonic_ascending(uint32_t k, uint32_t p, Get get, Put put) {
  for (uint32_t size = 2; size <= p; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < p; i += blockDim.x) {
        const uint32_t j = stride == (size >> 1) ? (i ^ (size - 1)) : (i ^ stride);
        if (j > i && j < k) {
          const uint32_t a = get(i), c = get(j);
          if (a > c) {
            put(i, c);
            put(j, a);
          }
        }
      }
      __syncthreads();
    }
  }
}

__global__ void __launch_bounds__(256) bin_sort_large_kernel(const uint32_t* __restrict__ start,
                                                             uint32_t* sorted,
                                                             const uint32_t* __restrict__ large) {
  __shared__ uint32_t sh[kLdsSort];
  const uint32_t count = large[0];
  for (uint32_t e = blockIdx.x; e < count; e += gridDim.x) {
    const uint32_t b = large[1 + e];
    const uint32_t lo = start[b], k = start[b + 1] - lo;
    uint32_t p = 1;
    while (p < k) p <<= 1;
    uint32_t* g = sorted + lo;
    if (k <= static_cast<uint32_t>(kLdsSort)) {
      for (uint32_t i = threadIdx.x; i < k; i += blockDim.x) sh[i] = g[i];
      __syncthreads();
      bitonic_ascending(k, p, [&](uint32_t i) { return sh[i]; },
                        [&](uint32_t i, uint32_t v) { sh[i] = v; });
      for (uint32_t i = threadIdx.x; i < k; i += blockDim.x) g[i] = sh[i];
    } else {
      bitonic_ascending(k, p, [&](uint32_t i) { return g[i]; },
                        [&](uint32_t i, uint32_t v) { g[i] = v; });
    }
    __syncthreads();
  }
}

// out[j] = (v[0][id], v[1][id], v[2][id], 0) for id = sorted[j] (global particle index: sample
// id >> lnp, particle id & (np - 1) of a per-sample [3][np] array)
__global__ void gather_sorted_kernel(const uint32_t* __restrict__ sorted,
                                     const float* __restrict__ v, float4* __restrict__ out,
                                     long long total, int lnp) {
  const long long j = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= total) return;
  const uint32_t id = sorted[j];
  const long long np = 1LL << lnp;
  const long long smp = id >> lnp, loc = id & (np - 1);
  const float* vs = v + smp * 3 * np;
  out[j] = make_float4(vs[loc], vs[np + loc], vs[2 * np + loc], 0.0f);
}

// ---------------------------------------------------------------------------- deposit
// A block owns a tile of TX x TY x TZ cells.  Pass 1: for every bin of the tile and of its
// low halo (the bins that reach the tile), one thread sums over the bin's particles, in
// ascending order, the 8 CIC corner weights (times one component of the particle's vector
// for the vector deposit) into LDS:
//   W[o][b] = sum_{p in b} prod_d (o_d ? w1_d : 1 - w1_d),  o in {0,1}^3.
// Pass 2: cell c adds W[o][c - o] over o in a fixed order.  Each particle's weights are
// formed once per tile that sees its bin (about 1.5 times) instead of once per cell, and the
// sums are reproducible bit for bit.
template <int TX, int TY, int TZ>
struct DepTile {
  static constexpr int BX = TX + 1, BY = TY + 1, BZ = TZ + 1;
  static constexpr int NB = BX * BY * BZ;           // bins read by a tile
  static constexpr int NC = TX * TY * TZ;           // cells of a tile
  static constexpr int PER = (NB + 255) / 256;      // bins per thread
};

// Bins of more than kCrowded particles (dense halos gather hundreds or thousands of
// particles in a cell) are summed by whole waves instead of one thread: the block lists them
// in LDS during pass 1 and its waves take them one each, every lane over a strided share of
// the bin's particles in ascending order, then a fixed butterfly across the wave, so the sums
// stay reproducible bit for bit and no thread loops over a crowded bin alone.
constexpr uint32_t kCrowded = 16;

// sum of v over the 64 lanes of the wave, every lane receiving it (fixed order)
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// cell of tile bin b (the tile at x0, y0, z0 and its low halo)
template <int BX, int BY>
__device__ __forceinline__ int tile_bin_cell(int b, int x0, int y0, int z0, int n) {
  const int bx = b % BX, by = (b / BX) % BY, bz = b / (BX * BY);
  return (wrapi(z0 - 1 + bz, n) * n + wrapi(y0 - 1 + by, n)) * n + wrapi(x0 - 1 + bx, n);
}

// W[o][b] (or the weights times one component v of sval, VEC) of the crowded bins listed in
// list[0..count): wave w of the block takes entries w, w + waves, ...
template <int TX, int TY, int TZ, bool VEC>
__device__ __forceinline__ void crowded_bin_sums(const uint32_t* __restrict__ start,
                                                 const float4* __restrict__ spos,
                                                 const float4* __restrict__ sval, int v,
                                                 const uint16_t* list, int count, int x0, int y0,
                                                 int z0, int n, float* W) {
  using T = DepTile<TX, TY, TZ>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  for (int e = wave; e < count; e += waves) {
    const int b = list[e];
    const int cell = tile_bin_cell<T::BX, T::BY>(b, x0, y0, z0, n);
    const uint32_t lo = start[cell], hi = start[cell + 1];
    float acc[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) acc[o] = 0.0f;
    for (uint32_t j = lo + lane; j < hi; j += 64) {
      const float4 p = spos[j];
      float val = 1.0f;
      if (VEC) {
        const float4 q = sval[j];
        val = v == 0 ? q.x : (v == 1 ? q.y : q.z);
      }
      const float wx = w1_of(p.x), wy = w1_of(p.y), wz = w1_of(p.z);
#pragma unroll
      for (int o = 0; o < 8; ++o) {
        const float w = wsel(wx, o & 1) * wsel(wy, (o >> 1) & 1) * wsel(wz, o >> 2);
        acc[o] += VEC ? w * val : w;
      }
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const float t = wave_sum(acc[o]);
      if (lane == 0) W[o * T::NB + b] = t;
    }
  }
}

// Pass 1 of the density deposit: W[o][b] for the bins of the tile and its halo.
template <int TX, int TY, int TZ>
__device__ __forceinline__ void deposit_tile(const uint32_t* __restrict__ start,
                                             const float4* __restrict__ spos, int n, int x0,
                                             int y0, int z0, float* W) {
  using T = DepTile<TX, TY, TZ>;
  __shared__ int ncrowd;
  __shared__ uint16_t crowd[T::NB];
  if (threadIdx.x == 0) ncrowd = 0;
  __syncthreads();
  // bounds of this thread's bins first (independent loads), then their particles
  uint32_t lo[T::PER], hi[T::PER];
#pragma unroll
  for (int k = 0; k < T::PER; ++k) {
    const int b = threadIdx.x + 256 * k;
    lo[k] = hi[k] = 0;
    if (b < T::NB) {
      const int bx = b % T::BX, by = (b / T::BX) % T::BY, bz = b / (T::BX * T::BY);
      const long long cell = (static_cast<long long>(wrapi(z0 - 1 + bz, n)) * n +
                              wrapi(y0 - 1 + by, n)) * n + wrapi(x0 - 1 + bx, n);
      lo[k] = start[cell];
      hi[k] = start[cell + 1];
    }
  }
  // the first particle of every bin of this thread (one round of independent loads; bins
  // seldom hold more than one particle before clustering)
  float4 p0[T::PER];
#pragma unroll
  for (int k = 0; k < T::PER; ++k) p0[k] = spos[lo[k] < hi[k] ? lo[k] : 0u];
#pragma unroll
  for (int k = 0; k < T::PER; ++k) {
    const int b = threadIdx.x + 256 * k;
    if (b >= T::NB) continue;
    if (hi[k] - lo[k] > kCrowded) {
      // the list order only decides which wave sums the bin
      crowd[atomicAdd(&ncrowd, 1)] = static_cast<uint16_t>(b);
      continue;
    }
    float acc[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) acc[o] = 0.0f;
    for (uint32_t j = lo[k]; j < hi[k]; ++j) {
      const float4 p = j == lo[k] ? p0[k] : spos[j];
      const float wx = w1_of(p.x), wy = w1_of(p.y), wz = w1_of(p.z);
#pragma unroll
      for (int o = 0; o < 8; ++o)
        acc[o] += wsel(wx, o & 1) * wsel(wy, (o >> 1) & 1) * wsel(wz, o >> 2);
    }
#pragma unroll
    for (int o = 0; o < 8; ++o) W[o * T::NB + b] = acc[o];
  }
  __syncthreads();
  crowded_bin_sums<TX, TY, TZ, false>(start, spos, nullptr, 0, crowd, ncrowd, x0, y0, z0, n, W);
}

// sum over the 8 corners of cell (cx, cy, cz) of the tile
template <int TX, int TY, int TZ>
__device__ __forceinline__ float tile_cell_sum(const float* W, int cx, int cy, int cz) {
  using T = DepTile<TX, TY, TZ>;
  float s = 0.0f;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const int b = ((cz + 1 - (o >> 2)) * T::BY + (cy + 1 - ((o >> 1) & 1))) * T::BX +
                  (cx + 1 - (o & 1));
    s += W[o * T::NB + b];
  }
  return s;
}

// tile t of a sample: x fastest
template <int TX, int TY, int TZ>
__device__ __forceinline__ void tile_origin(int n, int& x0, int& y0, int& z0) {
  const int tx = n / TX, ty = n / TY;
  const int t = blockIdx.x;
  x0 = (t % tx) * TX;
  y0 = ((t / tx) % ty) * TY;
  z0 = (t / (tx * ty)) * TZ;
}

template <int TX, int TY, int TZ>
__global__ void __launch_bounds__(256) deposit_kernel(const uint32_t* __restrict__ start,
                                                      const float4* __restrict__ spos,
                                                      const float* __restrict__ rho_gas,
                                                      long long rho_stride, float m_dm,
                                                      float offset, float* __restrict__ out,
                                                      int n, const StepScal* __restrict__ tab) {
  using T = DepTile<TX, TY, TZ>;
  __shared__ float W[8 * T::NB];
  if (!sample_active(tab, blockIdx.y)) return;
  const long long nc = static_cast<long long>(n) * n * n;
  start += blockIdx.y * nc;
  if (rho_gas) rho_gas += blockIdx.y * rho_stride;
  out += blockIdx.y * nc;
  int x0, y0, z0;
  tile_origin<TX, TY, TZ>(n, x0, y0, z0);
  deposit_tile<TX, TY, TZ>(start, spos, n, x0, y0, z0, W);
  __syncthreads();
  for (int t = threadIdx.x; t < T::NC; t += 256) {
    const int cx = t % TX, cy = (t / TX) % TY, cz = t / (TX * TY);
    const long long c = (static_cast<long long>(z0 + cz) * n + (y0 + cy)) * n + (x0 + cx);
    const float g = rho_gas ? rho_gas[c] : 0.0f;
    out[c] = g + m_dm * tile_cell_sum<TX, TY, TZ>(W, cx, cy, cz) + offset;
  }
}

// Vector deposit: the three components go through the same 8-corner LDS table one after the
// other (a third of the LDS of a 24-sum table, so twice as many blocks per CU); the CIC
// weights of the first particle of each bin stay in registers across the three passes.
// (Reading the vector field through the bins' particle ids, one component per pass, instead
// of gathering it into bin order first, took 660 us against 432 + 104 us at 256^3: the
// dependent loads of every pass and halo bin cost more than the gather.)
template <int TX, int TY, int TZ>
__global__ void __launch_bounds__(256) deposit_vec_kernel(const uint32_t* __restrict__ start,
                                                          const float4* __restrict__ spos,
                                                          const float4* __restrict__ sval,
                                                          bool merged, float* __restrict__ out,
                                                          int n, const StepScal* __restrict__ tab) {
  using T = DepTile<TX, TY, TZ>;
  constexpr int CPT = (T::NC + 255) / 256;   // cells per thread
  __shared__ float W[8 * T::NB];
  __shared__ int ncrowd;
  __shared__ uint16_t crowd[T::NB];
  const StepScal& sc = tab[blockIdx.y];
  if (!sc.active) return;
  if (threadIdx.x == 0) ncrowd = 0;
  __syncthreads();
  const float scale = merged ? sc.h_dm : sc.h_open;
  const long long nc = static_cast<long long>(n) * n * n;
  start += blockIdx.y * nc;
  out += blockIdx.y * 3 * nc;
  int x0, y0, z0;
  tile_origin<TX, TY, TZ>(n, x0, y0, z0);
  uint32_t lo[T::PER], hi[T::PER];
#pragma unroll
  for (int k = 0; k < T::PER; ++k) {
    const int b = threadIdx.x + 256 * k;
    lo[k] = hi[k] = 0;
    if (b < T::NB) {
      const int bx = b % T::BX, by = (b / T::BX) % T::BY, bz = b / (T::BX * T::BY);
      const long long cell = (static_cast<long long>(wrapi(z0 - 1 + bz, n)) * n +
                              wrapi(y0 - 1 + by, n)) * n + wrapi(x0 - 1 + bx, n);
      lo[k] = start[cell];
      hi[k] = start[cell + 1];
    }
  }
  // crowded bins: listed once, summed by waves for each component
  bool crowded[T::PER];
#pragma unroll
  for (int k = 0; k < T::PER; ++k) {
    const int b = threadIdx.x + 256 * k;
    crowded[k] = b < T::NB && hi[k] - lo[k] > kCrowded;
    if (crowded[k]) crowd[atomicAdd(&ncrowd, 1)] = static_cast<uint16_t>(b);
  }
  float w0[T::PER][3];   // CIC weights of the first particle of each bin
  float4 v0[T::PER];
#pragma unroll
  for (int k = 0; k < T::PER; ++k) {
    const uint32_t j = lo[k] < hi[k] ? lo[k] : 0u;
    const float4 p = spos[j];
    w0[k][0] = w1_of(p.x);
    w0[k][1] = w1_of(p.y);
    w0[k][2] = w1_of(p.z);
    v0[k] = sval[j];
  }
  __syncthreads();
  float sum[3][CPT];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    crowded_bin_sums<TX, TY, TZ, true>(start, spos, sval, v, crowd, ncrowd, x0, y0, z0, n, W);
#pragma unroll
    for (int k = 0; k < T::PER; ++k) {
      const int b = threadIdx.x + 256 * k;
      if (b >= T::NB) continue;
      if (crowded[k]) continue;   // summed by a wave
      float acc[8];
#pragma unroll
      for (int o = 0; o < 8; ++o) acc[o] = 0.0f;
      if (lo[k] < hi[k]) {
        const float val = v == 0 ? v0[k].x : (v == 1 ? v0[k].y : v0[k].z);
        add_corners(w0[k][0], w0[k][1], w0[k][2], val, acc);
      }
      for (uint32_t j = lo[k] + 1; j < hi[k]; ++j) {
        const float4 p = spos[j];
        const float4 q = sval[j];
        const float val = v == 0 ? q.x : (v == 1 ? q.y : q.z);
        add_corners(w1_of(p.x), w1_of(p.y), w1_of(p.z), val, acc);
      }
#pragma unroll
      for (int o = 0; o < 8; ++o) W[o * T::NB + b] = acc[o];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int t = threadIdx.x + 256 * i;
      sum[v][i] = 0.0f;
      if (t < T::NC) {
        const int cx = t % TX, cy = (t / TX) % TY, cz = t / (TX * TY);
        sum[v][i] = tile_cell_sum<TX, TY, TZ>(W, cx, cy, cz);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < CPT; ++i) {
    const int t = threadIdx.x + 256 * i;
    if (t >= T::NC) continue;
    const int cx = t % TX, cy = (t / TX) % TY, cz = t / (TX * TY);
    const long long c = (static_cast<long long>(z0 + cz) * n + (y0 + cy)) * n + (x0 + cx);
#pragma unroll
    for (int v = 0; v < 3; ++v) out[v * nc + c] += scale * sum[v][i];
  }
}

// Cell c of one sample (at most 256^3, so 32-bit) from its x, y, z: n is a power of two.
struct GridIdx {
  unsigned n1, lg;   // n - 1, log2 n
  __device__ __forceinline__ unsigned at(unsigned x, unsigned y, unsigned z) const {
    return (((z & n1) << lg | (y & n1)) << lg) | (x & n1);
  }
};

// g4[c] = (g_x, g_y, g_z, 0),  g_d = -(phi[c + e_d] - phi[c - e_d]) / 2
__global__ void __launch_bounds__(256) grad_kernel(const float* __restrict__ phi,
                                                   float4* __restrict__ g4, int n, int lgn,
                                                   const StepScal* __restrict__ tab) {
  const unsigned c = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned nc = 1u << (3 * lgn);
  if (c >= nc || !sample_active(tab, blockIdx.y)) return;
  phi += static_cast<long long>(blockIdx.y) * nc;
  g4 += static_cast<long long>(blockIdx.y) * nc;
  const GridIdx gi{static_cast<unsigned>(n - 1), static_cast<unsigned>(lgn)};
  const unsigned ix = c & gi.n1, iy = (c >> lgn) & gi.n1, iz = c >> (2 * lgn);
  const float gx = -0.5f * (phi[gi.at(ix + 1, iy, iz)] - phi[gi.at(ix - 1, iy, iz)]);
  const float gy = -0.5f * (phi[gi.at(ix, iy + 1, iz)] - phi[gi.at(ix, iy - 1, iz)]);
  const float gz = -0.5f * (phi[gi.at(ix, iy, iz + 1)] - phi[gi.at(ix, iy, iz - 1)]);
  g4[c] = make_float4(gx, gy, gz, 0.0f);
}

__device__ __forceinline__ long long corner(const Cic& w, int ox, int oy, int oz, int n) {
  return (static_cast<long long>(wrapi(w.i0[2] + oz, n)) * n + wrapi(w.i0[1] + oy, n)) * n +
         wrapi(w.i0[0] + ox, n);
}

// CIC read-out of g at a particle
__device__ __forceinline__ void readout_g(const float4* __restrict__ g4, const Cic& w, int n,
                                          float out[3]) {
  out[0] = out[1] = out[2] = 0.0f;
#pragma unroll
  for (int oz = 0; oz < 2; ++oz)
#pragma unroll
    for (int oy = 0; oy < 2; ++oy)
#pragma unroll
      for (int ox = 0; ox < 2; ++ox) {
        const float4 g = g4[corner(w, ox, oy, oz, n)];
        const float ww = wsel(w.w1[0], ox) * wsel(w.w1[1], oy) * wsel(w.w1[2], oz);
        out[0] = fmaf(ww, g.x, out[0]);
        out[1] = fmaf(ww, g.y, out[1]);
        out[2] = fmaf(ww, g.z, out[2]);
      }
}

__global__ void __launch_bounds__(256) readout_g_kernel(const float4* __restrict__ g4,
                                                        const float* __restrict__ pos,
                                                        float* __restrict__ out, int n,
                                                        long long np) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= np) return;
  g4 += blockIdx.y * np;
  pos += blockIdx.y * 3 * np;
  out += blockIdx.y * 3 * np;
  const Cic w = cic_of(pos[i], pos[np + i], pos[2 * np + i], n);
  float g[3];
  readout_g(g4, w, n, g);
  out[i] = g[0];
  out[np + i] = g[1];
  out[2 * np + i] = g[2];
}

// Stars formed in a step, associated with the dark matter (Sec. 2.4.1): each particle's
// auxiliary field gains the CIC read-out of the step's new stars znew at its position.
// Particles in bin order (spos, sorted: global ids, sample in the high bits), so that
// neighbouring threads read neighbouring cells; samples that sit the step out are skipped.
__global__ void __launch_bounds__(256) star_readout_kernel(const float* __restrict__ znew,
                                                           const float4* __restrict__ spos,
                                                           const uint32_t* __restrict__ sorted,
                                                           float* __restrict__ aux, int n,
                                                           long long total, int lnp,
                                                           const StepScal* __restrict__ tab) {
  const long long j = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= total) return;
  const uint32_t id = sorted[j];
  const long long smp = id >> lnp;
  if (!sample_active(tab, static_cast<int>(smp))) return;
  const float* zs = znew + (smp << lnp);   // n^3 cells = n^3 particles per sample
  const float4 x = spos[j];
  const Cic w = cic_of(x.x, x.y, x.z, n);
  float v = 0.0f;
#pragma unroll
  for (int oz = 0; oz < 2; ++oz)
#pragma unroll
    for (int oy = 0; oy < 2; ++oy)
#pragma unroll
      for (int ox = 0; ox < 2; ++ox)
        v = fmaf(wsel(w.w1[0], ox) * wsel(w.w1[1], oy) * wsel(w.w1[2], oz),
                 zs[corner(w, ox, oy, oz, n)], v);
  aux[id] += v;
}

__device__ __forceinline__ float wrap_pos(float x, float fn) {
  x -= fn * floorf(x / fn);
  if (x >= fn) x -= fn;
  return x;
}

// Opening half kick and drift of the dark matter, with the keys of the new positions.  With
// `prev`, the closing half kick of the sample's previous step (factor h_prev, same field and
// positions) is applied first: the two kicks are the separate roundings of kick_kernel
// followed by this kernel, fused into one pass over the particles.
// pos_in and pos may be the same array (in place): no __restrict__ on them
__global__ void __launch_bounds__(256) kick_drift_kernel(const float4* __restrict__ g4,
                                                         const float* pos_in, float* pos,
                                                         float* __restrict__ mom,
                                                         uint32_t* __restrict__ key,
                                                         float* __restrict__ mom_copy,
                                                         float* __restrict__ pos_copy, int n,
                                                         long long np, int prev,
                                                         const StepScal* __restrict__ tab,
                                                         uint32_t* count,
                                                         uint32_t* __restrict__ rank) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const StepScal& sc = tab[blockIdx.y];
  if (i >= np) return;
  const int smp = blockIdx.y;
  g4 += smp * np;
  pos_in += smp * 3 * np;
  pos += smp * 3 * np;
  mom += smp * 3 * np;
  key += smp * np;
  if (mom_copy) mom_copy += smp * 3 * np;
  if (pos_copy) pos_copy += smp * 3 * np;
  if (count) rank += smp * np;
  if (!sc.active) {
    // the sort's histogram counts the sample's particles under the keys they have
    if (count) rank[i] = atomicAdd(&count[key[i]], 1u);
    // a sample that sits the step out keeps its particles; the copies (the tape of the
    // reverse pass, which sorts them again) receive them unchanged
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float xd = pos_in[d * np + i];
      if (pos != pos_in) pos[d * np + i] = xd;
      if (mom_copy) mom_copy[d * np + i] = mom[d * np + i];
      if (pos_copy) pos_copy[d * np + i] = xd;
    }
    return;
  }
  const float h = sc.h_open, drift_fac = sc.drift, hp = prev ? sc.h_prev : 0.0f;
  float x[3] = {pos_in[i], pos_in[np + i], pos_in[2 * np + i]};
  const Cic w = cic_of(x[0], x[1], x[2], n);
  float g[3];
  readout_g(g4, w, n, g);
  const float fn = static_cast<float>(n);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float p = mom[d * np + i];
    if (prev) p = fmaf(hp, g[d], p);
    p = fmaf(h, g[d], p);
    mom[d * np + i] = p;
    x[d] = wrap_pos(x[d] + p * drift_fac, fn);
    pos[d * np + i] = x[d];
    if (mom_copy) mom_copy[d * np + i] = p;
    if (pos_copy) pos_copy[d * np + i] = x[d];
  }
  const Cic w2 = cic_of(x[0], x[1], x[2], n);
  const uint32_t k = bin_of(w2, n, smp, np);
  key[i] = k;
  // the sort's histogram (count zeroed beforehand): the arrival rank of the particle in its bin
  if (count) rank[i] = atomicAdd(&count[k], 1u);
}

__global__ void __launch_bounds__(256) kick_kernel(const float4* __restrict__ g4,
                                                   const float* __restrict__ pos,
                                                   float* __restrict__ mom, int n, long long np,
                                                   const StepScal* __restrict__ tab) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const StepScal& sc = tab[blockIdx.y];
  if (i >= np || !sc.active) return;
  const float h = sc.h_close;
  g4 += blockIdx.y * np;
  pos += blockIdx.y * 3 * np;
  mom += blockIdx.y * 3 * np;
  const Cic w = cic_of(pos[i], pos[np + i], pos[2 * np + i], n);
  float g[3];
  readout_g(g4, w, n, g);
#pragma unroll
  for (int d = 0; d < 3; ++d) mom[d * np + i] = fmaf(h, g[d], mom[d * np + i]);
}

// acc = sum_corners (dw/dx) (g_corner . lp): the kick's adjoint with respect to the position
__device__ __forceinline__ void kick_pos_acc(const float4* __restrict__ g4, const Cic& w,
                                             const float lp[3], int n, float acc[3]) {
  acc[0] = acc[1] = acc[2] = 0.0f;
#pragma unroll
  for (int oz = 0; oz < 2; ++oz)
#pragma unroll
    for (int oy = 0; oy < 2; ++oy)
#pragma unroll
      for (int ox = 0; ox < 2; ++ox) {
        const float4 g = g4[corner(w, ox, oy, oz, n)];
        const float gl = g.x * lp[0] + g.y * lp[1] + g.z * lp[2];
        const float wx = wsel(w.w1[0], ox), wy = wsel(w.w1[1], oy), wz = wsel(w.w1[2], oz);
        acc[0] += (ox ? 1.0f : -1.0f) * wy * wz * gl;
        acc[1] += wx * (oy ? 1.0f : -1.0f) * wz * gl;
        acc[2] += wx * wy * (oz ? 1.0f : -1.0f) * gl;
      }
}

// lam_x += h * sum_corners (dw/dx) (g_corner . lam_p)
__global__ void __launch_bounds__(256) kick_vjp_pos_kernel(const float4* __restrict__ g4,
                                                           const float* __restrict__ pos,
                                                           const float* __restrict__ lam_p,
                                                           bool merged, float* __restrict__ lam_x,
                                                           int n, long long np,
                                                           const StepScal* __restrict__ tab) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const StepScal& sc = tab[blockIdx.y];
  if (i >= np || !sc.active) return;
  const float h = merged ? sc.h_dm : sc.h_open;
  g4 += blockIdx.y * np;
  pos += blockIdx.y * 3 * np;
  lam_p += blockIdx.y * 3 * np;
  lam_x += blockIdx.y * 3 * np;
  const Cic w = cic_of(pos[i], pos[np + i], pos[2 * np + i], n);
  const float lp[3] = {lam_p[i], lam_p[np + i], lam_p[2 * np + i]};
  float acc[3];
  kick_pos_acc(g4, w, lp, n, acc);
#pragma unroll
  for (int d = 0; d < 3; ++d) lam_x[d * np + i] = fmaf(h, acc[d], lam_x[d * np + i]);
}

// lam_x += mass * sum_corners lam_delta[corner] dw/dx
// With lam_p: first, with g4, the merged dark-matter kicks' adjoint with respect to the
// position (kick_vjp_pos_kernel, factor h_dm); last, lam_p += drift lam_x (the drift's
// adjoint, x1 = x0 + drift p).  One pass, the roundings of the separate kernels.
__global__ void __launch_bounds__(256) deposit_vjp_pos_kernel(const float* __restrict__ lam_delta,
                                                              const float* __restrict__ pos,
                                                              float mass, float* __restrict__ lam_x,
                                                              float* __restrict__ lam_p,
                                                              const float4* __restrict__ g4,
                                                              int n, long long np,
                                                              const StepScal* __restrict__ tab) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= np || !sample_active(tab, blockIdx.y)) return;
  lam_delta += blockIdx.y * np;
  pos += blockIdx.y * 3 * np;
  lam_x += blockIdx.y * 3 * np;
  if (lam_p) lam_p += blockIdx.y * 3 * np;
  if (g4) g4 += blockIdx.y * np;
  const Cic w = cic_of(pos[i], pos[np + i], pos[2 * np + i], n);
  float lx0[3] = {lam_x[i], lam_x[np + i], lam_x[2 * np + i]};
  float lp[3] = {0.0f, 0.0f, 0.0f};
  if (lam_p) {
#pragma unroll
    for (int d = 0; d < 3; ++d) lp[d] = lam_p[d * np + i];
  }
  if (g4) {
    float ka[3];
    kick_pos_acc(g4, w, lp, n, ka);
    const float h = tab[blockIdx.y].h_dm;
#pragma unroll
    for (int d = 0; d < 3; ++d) lx0[d] = fmaf(h, ka[d], lx0[d]);
  }
  float acc[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int oz = 0; oz < 2; ++oz)
#pragma unroll
    for (int oy = 0; oy < 2; ++oy)
#pragma unroll
      for (int ox = 0; ox < 2; ++ox) {
        const float l = lam_delta[corner(w, ox, oy, oz, n)];
        const float wx = wsel(w.w1[0], ox), wy = wsel(w.w1[1], oy), wz = wsel(w.w1[2], oz);
        acc[0] += (ox ? 1.0f : -1.0f) * wy * wz * l;
        acc[1] += wx * (oy ? 1.0f : -1.0f) * wz * l;
        acc[2] += wx * wy * (oz ? 1.0f : -1.0f) * l;
      }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float lx = fmaf(mass, acc[d], lx0[d]);
    lam_x[d * np + i] = lx;
    if (lam_p) lam_p[d * np + i] = fmaf(tab[blockIdx.y].drift, lx, lp[d]);
  }
}

__global__ void axpy_kernel(float* __restrict__ y, const float* __restrict__ x, float a,
                            long long count, long long ys, long long xs, bool by_drift,
                            const StepScal* __restrict__ tab) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count || !sample_active(tab, blockIdx.y)) return;
  const float f = by_drift ? a * tab[blockIdx.y].drift : a;
  y[blockIdx.y * ys + i] = fmaf(f, x[blockIdx.y * xs + i], y[blockIdx.y * ys + i]);
}

// lam_phi[c] = lam_phi_in[c] + sum_d (lam_g_d[c + e_d] - lam_g_d[c - e_d]) / 2.
// FIRST: the terms of a first field lam_g0 come before those of lam_g, starting from 0 (the
// value the launch for lam_g0 alone would have passed in as lam_phi_in, rounded alike).
template <bool FIRST>
__global__ void __launch_bounds__(256) grad_vjp_kernel(const float* __restrict__ lam_g,
                                                       const float* __restrict__ lam_phi_in,
                                                       float* __restrict__ lam_phi, int n, int lgn,
                                                       const StepScal* __restrict__ tab,
                                                       const float* __restrict__ lam_g0) {
  const unsigned c = blockIdx.x * blockDim.x + threadIdx.x;
  const unsigned nc = 1u << (3 * lgn);
  if (c >= nc || !sample_active(tab, blockIdx.y)) return;
  lam_g += static_cast<long long>(blockIdx.y) * 3 * nc;
  if (lam_phi_in) lam_phi_in += static_cast<long long>(blockIdx.y) * nc;
  lam_phi += static_cast<long long>(blockIdx.y) * nc;
  const GridIdx gi{static_cast<unsigned>(n - 1), static_cast<unsigned>(lgn)};
  const unsigned ix = c & gi.n1, iy = (c >> lgn) & gi.n1, iz = c >> (2 * lgn);
  const float* lx = lam_g;
  const float* ly = lam_g + nc;
  const float* lz = lam_g + 2 * static_cast<long long>(nc);
  float v = lam_phi_in ? lam_phi_in[c] : 0.0f;
  if (FIRST) {
    lam_g0 += static_cast<long long>(blockIdx.y) * 3 * nc;
    const float* mx = lam_g0;
    const float* my = lam_g0 + nc;
    const float* mz = lam_g0 + 2 * static_cast<long long>(nc);
    v += 0.5f * (mx[gi.at(ix + 1, iy, iz)] - mx[gi.at(ix - 1, iy, iz)]);
    v += 0.5f * (my[gi.at(ix, iy + 1, iz)] - my[gi.at(ix, iy - 1, iz)]);
    v += 0.5f * (mz[gi.at(ix, iy, iz + 1)] - mz[gi.at(ix, iy, iz - 1)]);
  }
  v += 0.5f * (lx[gi.at(ix + 1, iy, iz)] - lx[gi.at(ix - 1, iy, iz)]);
  v += 0.5f * (ly[gi.at(ix, iy + 1, iz)] - ly[gi.at(ix, iy - 1, iz)]);
  v += 0.5f * (lz[gi.at(ix, iy, iz + 1)] - lz[gi.at(ix, iy, iz - 1)]);
  lam_phi[c] = v;
}

}  // namespace

long long large_bin_capacity(long long total) { return total / (kSmallBin + 1) + 1; }

size_t scan_block_count(long long nbins) {
  return static_cast<size_t>((nbins + kScanTile - 1) / kScanTile);
}

namespace {
int log2_ll(long long v) {
  int l = 0;
  while ((1LL << l) < v) ++l;
  return l;
}
dim3 per_sample(long long work, const Batch& b) { return dim3(blocks_for(work, 256), b.S); }
}  // namespace

void launch_keys(hipStream_t st, const float* pos, uint32_t* key, const Batch& b) {
  const long long np = b.nc();
  hipLaunchKernelGGL(keys_kernel, per_sample(np, b), dim3(256), 0, st, pos, key, b.n, np);
  DH_LAUNCH_CHECK();
}

void launch_sort(hipStream_t st, const Bins& bins, const float* pos, const Batch& b,
                 bool counted) {
  const long long nbins = b.nc() * b.S, total = nbins;
  if (!counted) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(nbins, 256)), dim3(256), 0, st,
                       bins.count, 0u, nbins);
    DH_LAUNCH_CHECK();
    hipLaunchKernelGGL(hist_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, st, bins.key,
                       bins.count, bins.rank, total);
    DH_LAUNCH_CHECK();
  }
  const int nb = static_cast<int>(scan_block_count(nbins));
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(nb), dim3(kScanThreads), 0, st, bins.count,
                     bins.block_sums, nbins);
  DH_LAUNCH_CHECK();
  hipLaunchKernelGGL(scan_block_sums_kernel, dim3(1), dim3(kScanThreads), 0, st, bins.block_sums,
                     nb);
  DH_LAUNCH_CHECK();
  hipLaunchKernelGGL(scan_final_kernel, dim3(nb), dim3(kScanThreads), 0, st, bins.count,
                     bins.block_sums, bins.start, nbins);
  DH_LAUNCH_CHECK();
  hipLaunchKernelGGL(scatter_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, st, bins.key,
                     bins.rank, bins.start, bins.sorted, total);
  DH_LAUNCH_CHECK();
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, st, bins.large, 0u, 1LL);
  DH_LAUNCH_CHECK();
  hipLaunchKernelGGL(bin_sort_kernel, dim3(blocks_for(nbins, 256)), dim3(256), 0, st, bins.start,
                     bins.sorted, nbins, bins.large);
  DH_LAUNCH_CHECK();
  hipLaunchKernelGGL(bin_sort_large_kernel, dim3(kLargeSortBlocks), dim3(256), 0, st, bins.start,
                     bins.sorted, bins.large);
  DH_LAUNCH_CHECK();
  hipLaunchKernelGGL(gather_sorted_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, st,
                     bins.sorted, pos, bins.spos, total, log2_ll(b.nc()));
  DH_LAUNCH_CHECK();
}

void launch_gather_sorted(hipStream_t st, const Bins& bins, const float* v, const Batch& b) {
  const long long total = b.nc() * b.S;
  hipLaunchKernelGGL(gather_sorted_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, st,
                     bins.sorted, v, bins.sval, total, log2_ll(b.nc()));
  DH_LAUNCH_CHECK();
}

void launch_deposit(hipStream_t st, const Bins& bins, const float* rho_gas,
                    long long rho_stride, float m_dm, float offset, float* out, const Batch& b) {
  // tiles of 32 x 4 x 4 cells (16 x 4 x 4 at n = 16): 26 KB of LDS, six blocks per CU
  if (b.n >= 32) {
    const unsigned tiles = static_cast<unsigned>(b.nc() / (32 * 4 * 4));
    hipLaunchKernelGGL((deposit_kernel<32, 4, 4>), dim3(tiles, b.S), dim3(256), 0, st,
                       bins.start, bins.spos, rho_gas, rho_stride, m_dm, offset, out, b.n, b.tab);
  } else {
    const unsigned tiles = static_cast<unsigned>(b.nc() / (16 * 4 * 4));
    hipLaunchKernelGGL((deposit_kernel<16, 4, 4>), dim3(tiles, b.S), dim3(256), 0, st,
                       bins.start, bins.spos, rho_gas, rho_stride, m_dm, offset, out, b.n, b.tab);
  }
  DH_LAUNCH_CHECK();
}

void launch_deposit_vec(hipStream_t st, const Bins& bins, bool merged, float* out_accum,
                        const Batch& b) {
  if (!b.tab) throw ArgError("deposit_vec: step table required");
  // tiles of 32 x 4 x 4 cells (16 x 4 x 4 at n = 16)
  if (b.n >= 32) {
    const unsigned tiles = static_cast<unsigned>(b.nc() / (32 * 4 * 4));
    hipLaunchKernelGGL((deposit_vec_kernel<32, 4, 4>), dim3(tiles, b.S), dim3(256), 0, st,
                       bins.start, bins.spos, bins.sval, merged, out_accum, b.n, b.tab);
  } else {
    const unsigned tiles = static_cast<unsigned>(b.nc() / (16 * 4 * 4));
    hipLaunchKernelGGL((deposit_vec_kernel<16, 4, 4>), dim3(tiles, b.S), dim3(256), 0, st,
                       bins.start, bins.spos, bins.sval, merged, out_accum, b.n, b.tab);
  }
  DH_LAUNCH_CHECK();
}

void launch_grad(hipStream_t st, const float* phi, float4* g4, const Batch& b) {
  hipLaunchKernelGGL(grad_kernel, per_sample(b.nc(), b), dim3(256), 0, st, phi, g4, b.n,
                     log2_ll(b.n), b.tab);
  DH_LAUNCH_CHECK();
}

void launch_readout_g(hipStream_t st, const float4* g4, const float* pos, float* out,
                      const Batch& b) {
  hipLaunchKernelGGL(readout_g_kernel, per_sample(b.nc(), b), dim3(256), 0, st, g4, pos, out, b.n,
                     b.nc());
  DH_LAUNCH_CHECK();
}

void launch_star_readout(hipStream_t st, const float* znew, const float4* spos,
                         const uint32_t* sorted, float* aux, const Batch& b) {
  if (!b.tab) throw ArgError("star read-out: step table required");
  const long long total = b.nc() * b.S;
  hipLaunchKernelGGL(star_readout_kernel, dim3(blocks_for(total, 256)), dim3(256), 0, st, znew,
                     spos, sorted, aux, b.n, total, log2_ll(b.nc()), b.tab);
  DH_LAUNCH_CHECK();
}

void launch_kick_drift(hipStream_t st, const float4* g4, const float* pos_in, float* pos,
                       float* mom, uint32_t* key, float* mom_copy, float* pos_copy, bool prev,
                       const Batch& b, const Bins* count_into) {
  if (!b.tab) throw ArgError("kick_drift: step table required");
  if (count_into && key != count_into->key) throw ArgError("kick_drift: keys of another sort");
  uint32_t* count = count_into ? count_into->count : nullptr;
  uint32_t* rank = count_into ? count_into->rank : nullptr;
  if (count) {
    const long long nbins = b.nc() * b.S;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(nbins, 256)), dim3(256), 0, st, count, 0u,
                       nbins);
    DH_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(kick_drift_kernel, per_sample(b.nc(), b), dim3(256), 0, st, g4, pos_in, pos,
                     mom, key, mom_copy, pos_copy, b.n, b.nc(), prev ? 1 : 0, b.tab, count, rank);
  DH_LAUNCH_CHECK();
}

void launch_kick(hipStream_t st, const float4* g4, const float* pos, float* mom, const Batch& b) {
  if (!b.tab) throw ArgError("kick: step table required");
  hipLaunchKernelGGL(kick_kernel, per_sample(b.nc(), b), dim3(256), 0, st, g4, pos, mom, b.n,
                     b.nc(), b.tab);
  DH_LAUNCH_CHECK();
}

void launch_kick_vjp_pos(hipStream_t st, const float4* g4, const float* pos, const float* lam_p,
                         bool merged, float* lam_x, const Batch& b) {
  if (!b.tab) throw ArgError("kick adjoint: step table required");
  hipLaunchKernelGGL(kick_vjp_pos_kernel, per_sample(b.nc(), b), dim3(256), 0, st, g4, pos, lam_p,
                     merged, lam_x, b.n, b.nc(), b.tab);
  DH_LAUNCH_CHECK();
}

void launch_deposit_vjp_pos(hipStream_t st, const float* lam_delta, const float* pos, float mass,
                            float* lam_x, float* lam_p, const float4* g4, const Batch& b) {
  if (lam_p && !b.tab) throw ArgError("deposit adjoint: step table required for the drift");
  if (g4 && !lam_p) throw ArgError("deposit adjoint: the kick term needs lam_p");
  hipLaunchKernelGGL(deposit_vjp_pos_kernel, per_sample(b.nc(), b), dim3(256), 0, st, lam_delta,
                     pos, mass, lam_x, lam_p, g4, b.n, b.nc(), b.tab);
  DH_LAUNCH_CHECK();
}

void launch_axpy(hipStream_t st, float* y, const float* x, float a, long long count, long long ys,
                 long long xs, bool by_drift, const Batch& b) {
  if (by_drift && !b.tab) throw ArgError("axpy: step table required");
  hipLaunchKernelGGL(axpy_kernel, per_sample(count, b), dim3(256), 0, st, y, x, a, count, ys, xs,
                     by_drift, b.tab);
  DH_LAUNCH_CHECK();
}

void launch_grad_vjp(hipStream_t st, const float* lam_g, const float* lam_phi_in, float* lam_phi,
                     const Batch& b) {
  hipLaunchKernelGGL(grad_vjp_kernel<false>, per_sample(b.nc(), b), dim3(256), 0, st, lam_g,
                     lam_phi_in, lam_phi, b.n, log2_ll(b.n), b.tab, nullptr);
  DH_LAUNCH_CHECK();
}

void launch_grad_vjp2(hipStream_t st, const float* lam_g0, const float* lam_g, float* lam_phi,
                      const Batch& b) {
  hipLaunchKernelGGL(grad_vjp_kernel<true>, per_sample(b.nc(), b), dim3(256), 0, st, lam_g,
                     nullptr, lam_phi, b.n, log2_ll(b.n), b.tab, lam_g0);
  DH_LAUNCH_CHECK();
}

}  // namespace dh

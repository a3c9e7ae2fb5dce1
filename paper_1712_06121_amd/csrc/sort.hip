// Stable sort of (key, value) pairs by key and a stable selection, for the load and export paths.
//
// The sort is a least-significant-digit radix sort over 8-bit digits. Each pass: (1) every tile of
// 4096 keys counts its digits; (2) one workgroup per digit turns the counts of all tiles into
// exclusive prefixes (tile order) and the digit's total; (3) every tile ranks its keys by digit in
// input order (wavefronts take contiguous quarters of the tile, lanes match equal digits with one
// ballot per digit bit) and writes each pair to digit start + tile prefix + rank. Ranks follow
// input order within a tile and tiles follow each other, so every pass is stable and the result
// is the stable order by key.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "cube_internal.h"

namespace cube {
namespace {

constexpr int RS_BLOCK = 256;                          // threads per tile
constexpr int RS_WAVES = RS_BLOCK / 64;
constexpr int RS_CHUNKS = 16;                          // chunks of 64 keys per wavefront
constexpr int RS_TILE = RS_BLOCK * RS_CHUNKS;          // keys per tile
constexpr int RS_RADIX = 256;

__device__ __forceinline__ uint32_t digit_of(uint32_t k, int shift) { return (k >> shift) & 0xFFu; }

// (1) digit counts of every tile: hist[d * ntile + t]
__global__ __launch_bounds__(RS_BLOCK) void k_rs_hist(const uint32_t* __restrict__ key, int64_t n, int shift,
                                                      uint32_t* __restrict__ hist, int64_t ntile) {
  __shared__ uint32_t cnt[RS_RADIX];
  cnt[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * RS_TILE;
  for (int k = 0; k < RS_CHUNKS; ++k) {
    const int64_t i = t0 + (int64_t)k * RS_BLOCK + threadIdx.x;
    if (i < n) atomicAdd(&cnt[digit_of(key[i], shift)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntile + blockIdx.x] = cnt[threadIdx.x];
}

// (2) one workgroup per digit: exclusive prefix of its tile counts, in place, and its total
__global__ __launch_bounds__(1024) void k_rs_digit_scan(uint32_t* __restrict__ hist, int64_t ntile,
                                                        uint32_t* __restrict__ total) {
  __shared__ uint32_t part[1024 / 64];
  __shared__ uint32_t carry;
  uint32_t* row = hist + (int64_t)blockIdx.x * ntile;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry = 0u;
  __syncthreads();
  for (int64_t b = 0; b < ntile; b += 1024) {
    const int64_t i = b + threadIdx.x;
    const uint32_t v = i < ntile ? row[i] : 0u;
    // inclusive scan over the wavefront, then over the wavefront totals
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) part[wave] = x;
    __syncthreads();
    uint32_t before = carry;
    for (int w = 0; w < wave; ++w) before += part[w];
    if (i < ntile) row[i] = before + x - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = before + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) total[blockIdx.x] = carry;
}

// (3) stable scatter of a tile's pairs by digit
__global__ __launch_bounds__(RS_BLOCK) void k_rs_scatter(const uint32_t* __restrict__ key, const uint32_t* __restrict__ val,
                                                         int64_t n, int shift, const uint32_t* __restrict__ hist,
                                                         const uint32_t* __restrict__ total, int64_t ntile,
                                                         uint32_t* __restrict__ key_out, uint32_t* __restrict__ val_out) {
  __shared__ uint32_t wcnt[RS_WAVES][RS_RADIX];  // per wavefront: keys of each digit so far
  __shared__ uint64_t base[RS_RADIX];            // digit start + this tile's prefix
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int w = 0; w < RS_WAVES; ++w) wcnt[w][threadIdx.x] = 0u;
  {
    // exclusive prefix of the digit totals (one digit per thread), plus this tile's prefix
    __shared__ uint32_t tot[RS_RADIX];
    tot[threadIdx.x] = total[threadIdx.x];
    __syncthreads();
    uint64_t s = 0;
    for (int d = 0; d < (int)threadIdx.x; ++d) s += tot[d];
    base[threadIdx.x] = s + hist[(int64_t)threadIdx.x * ntile + blockIdx.x];
  }
  __syncthreads();
  const unsigned long long lt = (1ull << lane) - 1ull;
  // wavefront w ranks a contiguous quarter of the tile, 64 keys at a time, in order
  constexpr int PER_WAVE = RS_TILE / RS_WAVES;
  const int64_t w0 = (int64_t)blockIdx.x * RS_TILE + (int64_t)wave * PER_WAVE;
  uint32_t kk[PER_WAVE / 64], vv[PER_WAVE / 64], rk[PER_WAVE / 64];
#pragma unroll
  for (int c = 0; c < PER_WAVE / 64; ++c) {
    const int64_t i = w0 + c * 64 + lane;
    const bool active = i < n;
    kk[c] = active ? key[i] : 0u;
    vv[c] = active ? val[i] : 0u;
    const uint32_t d = digit_of(kk[c], shift);
    unsigned long long peers = __ballot(active);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bb = __ballot(active && bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t before = wcnt[wave][d];  // same-address reads broadcast
    rk[c] = before + (uint32_t)__popcll(peers & lt);
    if (active && (peers & lt) == 0ull) wcnt[wave][d] = before + (uint32_t)__popcll(peers);
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < PER_WAVE / 64; ++c) {
    const int64_t i = w0 + c * 64 + lane;
    if (i >= n) continue;
    const uint32_t d = digit_of(kk[c], shift);
    uint32_t off = 0;
    for (int w = 0; w < wave; ++w) off += wcnt[w][d];
    const uint64_t dst = base[d] + off + rk[c];
    key_out[dst] = kk[c];
    val_out[dst] = vv[c];
  }
}

// ---- stable selection of the counts of at least 255 ------------------------------------------
constexpr int SEL_BLOCK = 256;
constexpr int SEL_TILE = 4096;

__global__ __launch_bounds__(SEL_BLOCK) void k_sel_count(const uint32_t* __restrict__ cnt, int64_t n,
                                                         uint32_t* __restrict__ part) {
  __shared__ uint32_t c;
  if (threadIdx.x == 0) c = 0u;
  __syncthreads();
  uint32_t m = 0;
  for (int k = 0; k < SEL_TILE / SEL_BLOCK; ++k) {
    const int64_t i = (int64_t)blockIdx.x * SEL_TILE + (int64_t)k * SEL_BLOCK + threadIdx.x;
    if (i < n && cnt[i] >= 255u) ++m;
  }
  if (m) atomicAdd(&c, m);
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = c;
}

// the selected values of each tile, in order, at the tile's exclusive prefix (one workgroup per tile)
__global__ __launch_bounds__(SEL_BLOCK) void k_sel_scatter(const uint32_t* __restrict__ cnt, int64_t n,
                                                           const uint32_t* __restrict__ prefix, uint32_t* __restrict__ out) {
  __shared__ uint32_t wsum[SEL_BLOCK / 64];
  __shared__ uint32_t run;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) run = 0u;
  __syncthreads();
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (int k = 0; k < SEL_TILE / SEL_BLOCK; ++k) {
    const int64_t i = (int64_t)blockIdx.x * SEL_TILE + (int64_t)k * SEL_BLOCK + threadIdx.x;
    const uint32_t v = i < n ? cnt[i] : 0u;
    const bool sel = i < n && v >= 255u;
    const unsigned long long m = __ballot(sel);
    if (lane == 0) wsum[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = run;
    for (int w = 0; w < wave; ++w) before += wsum[w];
    if (sel) out[prefix[blockIdx.x] + before + (uint32_t)__popcll(m & lt)] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int w = 0; w < SEL_BLOCK / 64; ++w) t += wsum[w];
      run += t;
    }
    __syncthreads();
  }
}

}  // namespace

void sort_pairs_by_key(Sim& s, uint32_t* key, uint32_t* val, uint32_t* key_alt, uint32_t* val_alt, int64_t n,
                       uint32_t max_key, hipStream_t st, uint32_t** key_sorted, uint32_t** val_sorted) {
  *key_sorted = key;
  *val_sorted = val;
  if (n <= 0) return;
  int bits = 1;
  while (bits < 32 && (max_key >> bits) != 0u) ++bits;
  const int64_t ntile = (n + RS_TILE - 1) / RS_TILE;
  uint32_t* hist = static_cast<uint32_t*>(s.dmalloc(sizeof(uint32_t) * ((size_t)RS_RADIX * ntile + RS_RADIX)));
  uint32_t* total = hist + (size_t)RS_RADIX * ntile;
  uint32_t *ki = key, *vi = val, *ko = key_alt, *vo = val_alt;
  for (int shift = 0; shift < bits; shift += 8) {
    k_rs_hist<<<(unsigned)ntile, RS_BLOCK, 0, st>>>(ki, n, shift, hist, ntile);
    k_rs_digit_scan<<<RS_RADIX, 1024, 0, st>>>(hist, ntile, total);
    k_rs_scatter<<<(unsigned)ntile, RS_BLOCK, 0, st>>>(ki, vi, n, shift, hist, total, ntile, ko, vo);
    CUBE_HIP(hipGetLastError());
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  CUBE_HIP(hipStreamSynchronize(st));
  s.dfree(hist);
  *key_sorted = ki;
  *val_sorted = vi;
}

int64_t select_at_least_255(Sim& s, const uint32_t* cnt, int64_t n, uint32_t* out, hipStream_t st) {
  if (n <= 0) return 0;
  const int64_t ntile = (n + SEL_TILE - 1) / SEL_TILE;
  uint32_t* part = static_cast<uint32_t*>(s.dmalloc(sizeof(uint32_t) * (size_t)(ntile + 1)));
  k_sel_count<<<(unsigned)ntile, SEL_BLOCK, 0, st>>>(cnt, n, part);
  CUBE_HIP(hipGetLastError());
  // the tile prefixes on the host: at most a few thousand tiles
  std::vector<uint32_t> h((size_t)ntile);
  CUBE_HIP(hipMemcpyAsync(h.data(), part, sizeof(uint32_t) * (size_t)ntile, hipMemcpyDeviceToHost, st));
  CUBE_HIP(hipStreamSynchronize(st));
  uint64_t run = 0;
  for (auto& v : h) {
    const uint32_t c = v;
    v = (uint32_t)run;
    run += c;
  }
  CUBE_HIP(hipMemcpyAsync(part, h.data(), sizeof(uint32_t) * (size_t)ntile, hipMemcpyHostToDevice, st));
  k_sel_scatter<<<(unsigned)ntile, SEL_BLOCK, 0, st>>>(cnt, n, part, out);
  CUBE_HIP(hipGetLastError());
  CUBE_HIP(hipStreamSynchronize(st));
  s.dfree(part);
  return (int64_t)run;
}

}  // namespace cube

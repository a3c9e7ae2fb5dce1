// Particle kernels of the compressed PM step for gfx950: integer CIC deposit, the two move passes
// (count, then encode + scatter), the per-cell link/scan/statistics kernels, the initial-condition
// lattice move and the load path.
//
// Storage (Sec. 2.1-2.2): particles are cell ordered; position codes chi (Eq. (chi)) and velocity
// codes nu (Eq. (nu)) are structure-of-arrays byte planes; per coarse cell the count, the storage
// offset, the mean velocity v_c and the decode scale sigma sqrt(2/pi) of Eq. (v).
//
// All kernels work on tiles of T^3 coarse cells (one workgroup per tile). Deposit gathers: the
// workgroup that owns a tile of fine cells reads the particles of its tile and of the ring of
// neighbouring coarse cells and accumulates exact integer CIC weights in LDS (no float atomics,
// no global atomics), so the density is bit-reproducible. The move passes scatter: each particle
// is handled by the workgroup that owns its coarse cell; the potential tile with a 3-cell halo
// sits in LDS for the 4-point gradient.
//
// The arithmetic follows one fixed sequence of IEEE operations so that the encoding, cell counts
// and order are reproducible bit for bit from identical inputs: the compiler forms no fused
// multiply-adds of its own (-ffp-contract=off), and the fused ones the sequence names -- velocity
// decode, the interpolation lerps, kick and drift -- are written out as fmaf.
#include <cstring>
#include <type_traits>


#include "cube_internal.h"

namespace cube {
namespace {

constexpr int T = 4;            // coarse cells per tile side
// tile offsets (x, y, z) of own cell s (x fastest), by shifts: s is never negative
__device__ __forceinline__ void tile_xyz(int s, int& ox, int& oy, int& oz) {
  static_assert(T == 4, "shifts assume four cells per side");
  const unsigned u = (unsigned)s;
  ox = (int)(u & 3u);
  oy = (int)((u >> 2) & 3u);
  oz = (int)(u >> 4);
}
constexpr int TC = T * T * T;   // own cells per tile
constexpr int F = 4 * T;        // fine cells per tile side
constexpr int PH = F + 6;       // potential tile side (3-cell halo)
constexpr int RG = T + 2;       // new-cell region side (tile + ring)
constexpr int RC = RG * RG * RG;
constexpr int SRC = RC;         // deposit source cells (tile + ring)
constexpr int BLK = 256;
constexpr int LINK_BLK = 256;

template <int NCHI>
using chi_t = std::conditional_t<NCHI == 1, uint8_t, uint16_t>;
template <int NNU>
using nu_t = std::conditional_t<NNU == 1, int8_t, int16_t>;

__device__ __forceinline__ int wrapi(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

__device__ __forceinline__ void set_flag(uint32_t* flags, uint32_t f) { atomicOr(flags, f); }

// number of lanes below this one in the wave mask m
__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// A step whose error flags are set is not applied: the kernels that write the next state (link,
// scan, cell statistics, scatter) return at once, so the state stays the one before the failing
// step, and so it does through every later step enqueued behind it. The flag word is read once per
// workgroup (through LDS), so all of a workgroup's waves take the same branch even when another
// workgroup raises a flag meanwhile.
__device__ __forceinline__ bool workgroup_step_failed(const uint32_t* flags) {
  __shared__ uint32_t failed;
  if (threadIdx.x == 0) failed = __atomic_load_n(flags, __ATOMIC_RELAXED);
  __syncthreads();
  return failed != 0u;
}

// exclusive prefix of up to 256 uint32 values held one per thread; returns the total
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* out, int n, uint32_t* wsum) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t x = (tid < n) ? v : 0u;
  uint32_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t wbase = 0, total = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
    if (w < wave) wbase += wsum[w];
    total += wsum[w];
  }
  if (tid < n) out[tid] = wbase + inc - x;
  if (tid == 0) out[n] = total;
  __syncthreads();
  return total;
}

template <unsigned CTRL, unsigned ROWS = 0xF>
__device__ __forceinline__ unsigned long long dpp_add_u64(unsigned long long v) {
  const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  uint32_t l2, h2;
  if constexpr (ROWS == 0xF) {
    // every row written: lanes without a source read 0 (bound control), no old value needed
    l2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo, CTRL, 0xF, 0xF, true);
    h2 = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi, CTRL, 0xF, 0xF, true);
  } else {
    l2 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lo, CTRL, ROWS, 0xF, false);
    h2 = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)hi, CTRL, ROWS, 0xF, false);
  }
  unsigned int carry;
  const unsigned int rl = __builtin_addc(lo, l2, 0u, &carry);
  const unsigned int rh = __builtin_addc(hi, h2, carry, &carry);
  return ((unsigned long long)rh << 32) | rl;
}

// One step of the 64-bit inclusive scan: v += (v of the lane DPP selects, 0 where there is none;
// rows outside the row mask unchanged), as a carry-propagating add whose first operand is read
// through DPP. The s_nop before each step covers the two wait states a DPP read needs after a VALU
// write of the same register; the one after the block keeps later DPP reads of lo / hi safe.
#define CUBE_DPP_ADD64(lo, hi, CTRL, RMASK)                                                        \
  asm volatile("s_nop 1\n\t"                                                                     \
               "v_add_co_u32_dpp %0, vcc, %0, %0 " CTRL " row_mask:" RMASK                        \
               " bank_mask:0xf bound_ctrl:1\n\t"                                                 \
               "v_addc_co_u32_dpp %1, vcc, %1, %1, vcc " CTRL " row_mask:" RMASK                  \
               " bank_mask:0xf bound_ctrl:1\n\t"                                                 \
               "s_nop 1"                                                                          \
               : "+v"(lo), "+v"(hi)                                                               \
               :                                                                                  \
               : "vcc")

// inclusive prefix sum over the 64 lanes (every lane active): shifts by 1, 2, 4, 8 inside each
// row of 16 lanes, then the totals of rows 0 and 2 into rows 1 and 3, then that of rows 0-1 into
// rows 2 and 3
__device__ __forceinline__ unsigned long long wave_scan_u64(unsigned long long v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  CUBE_DPP_ADD64(lo, hi, "row_shr:1", "0xf");
  CUBE_DPP_ADD64(lo, hi, "row_shr:2", "0xf");
  CUBE_DPP_ADD64(lo, hi, "row_shr:4", "0xf");
  CUBE_DPP_ADD64(lo, hi, "row_shr:8", "0xf");
  CUBE_DPP_ADD64(lo, hi, "row_bcast:15", "0xa");
  CUBE_DPP_ADD64(lo, hi, "row_bcast:31", "0xc");
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long read_lane_u64(unsigned long long v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}

// sum over the 64 lanes (every lane active), returned to all lanes
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  v = dpp_add_u64<0xB1>(v);   // quad_perm [1,0,3,2]
  v = dpp_add_u64<0x4E>(v);   // quad_perm [2,3,0,1]
  v = dpp_add_u64<0x141>(v);  // row_half_mirror
  v = dpp_add_u64<0x140>(v);  // row_mirror: every lane holds its 16-lane row sum
  const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  unsigned long long t = 0;
#pragma unroll
  for (int r = 15; r < 64; r += 16)
    t += ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)hi, r) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)lo, r);
  return t;
}

__device__ __forceinline__ int find_cell(const uint32_t* pre, int ncell, uint32_t i) {
  int lo = 0, hi = ncell;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

struct TileGeom {
  int cx0, cy0, cz0;
};
__device__ __forceinline__ TileGeom tile_of(int b, int nt) {
  TileGeom g;
  g.cx0 = (b % nt) * T;
  g.cy0 = ((b / nt) % nt) * T;
  g.cz0 = (b / (nt * nt)) * T;
  return g;
}

// ---------------------------------------------------------------------------------------------
// CIC deposit (Sec. 3 "CIC"; cell centres at i + 1/2), exact integer weights, gather by tile.
// ---------------------------------------------------------------------------------------------
struct DepArgs {
  const void* chi;
  const uint32_t* cnt;
  const uint64_t* off;
  int64_t cap;
  float* mesh;
  int64_t pitch_f;
  int nm, nc, nt;
  int zc;  // coarse layers per z chunk
  double inv_mean;
  int interleave;  // visit a layer's particles with a stride (fewer lanes adding to one cell at once)
};

constexpr int DTX = 8;            // coarse cells per column side
constexpr int DF = 4 * DTX;       // fine cells per column side
constexpr int DR = DTX + 2;       // source cells per side (column + ring)
constexpr int DRC = DR * DR;      // source cells per coarse layer
constexpr int NSLOT = 6;          // fine planes a coarse layer can touch

__device__ __forceinline__ int slot_of(int p) { return ((p % NSLOT) + NSLOT) % NSLOT; }

// Streaming gather: the workgroup owns a DF x DF column of fine cells over the fine planes of
// coarse layers [cz0, cz1). It walks the source coarse layers cz0-1 .. cz1 in order, each time
// reading the particles of the DR x DR cells (column + ring), and adds exact integer CIC weights
// to a rolling set of NSLOT fine planes in LDS. After layer sz, planes up to 4 sz + 2 receive no
// more mass: they are converted once to FP32 delta, written, and their slots reused.
template <int NCHI, int BLK>
__device__ __forceinline__ void deposit_column(const DepArgs& a, const unsigned lb) {
  using CT = chi_t<NCHI>;
  constexpr int SH = 8 * NCHI - 1;
  __shared__ unsigned long long rho[NSLOT * DF * DF];
  __shared__ uint32_t pre[DRC + 1];
  __shared__ uint64_t start[DRC];
  __shared__ uint32_t wsum[BLK / 64];
  // owner[k]: the source cell holding layer particle k << osh (a sparse index into pre, so that a
  // particle's cell is found by a short forward scan instead of a binary search)
  constexpr int NOWN = 1024;
  static_assert(DRC < 256, "cell indices fit a byte");
  __shared__ uint8_t owner[NOWN];
  const unsigned cols = (unsigned)(a.nt * a.nt);
  const unsigned bxy = lb % cols, bz = lb / cols;
  const int cx0 = (bxy % a.nt) * DTX, cy0 = (bxy / a.nt) * DTX;
  const int cz0 = bz * a.zc;
  const int cz1 = min(cz0 + a.zc, a.nc);
  const int pz0 = 4 * cz0, pz1 = 4 * cz1;  // owned fine planes [pz0, pz1)
  for (int i = threadIdx.x; i < NSLOT * DF * DF; i += BLK) rho[i] = 0ull;
  // 32-bit accumulators: a fine cell receives mass only from particles of the (at most 8) coarse
  // cells around it, each weighing 2^(3 SH) in total; with 1-byte codes and at most 255 particles
  // in every source cell of this workgroup the sum stays below 8 * 255 * 2^21 < 2^32
  __shared__ uint32_t smax;
  if (threadIdx.x == 0) smax = 0u;
  __syncthreads();
  if constexpr (NCHI == 1) {
    uint32_t m = 0u;
    const int ncell = DRC * (cz1 - cz0 + 2);
    for (int i = threadIdx.x; i < ncell; i += BLK) {
      const int t = i % DRC, sz = cz0 - 1 + i / DRC;
      const int sx = t % DR - 1, sy = t / DR - 1;
      const uint32_t c = a.cnt[wrapi(cx0 + sx, a.nc) + (int64_t)a.nc * (wrapi(cy0 + sy, a.nc) + (int64_t)a.nc * wrapi(sz, a.nc))];
      m = c > m ? c : m;
    }
    atomicMax(&smax, m);
  }
  __syncthreads();
  const bool narrow = NCHI == 1 && smax <= 255u;
  uint32_t* rho32 = reinterpret_cast<uint32_t*>(rho);
  const CT* cx = static_cast<const CT*>(a.chi);
  const CT* cy = cx + a.cap;
  const CT* cz = cy + a.cap;
  for (int sz = cz0 - 1; sz <= cz1; ++sz) {
    uint32_t cntv = 0;
    if (threadIdx.x < DRC) {
      const int sx = threadIdx.x % DR - 1, sy = threadIdx.x / DR - 1;
      const int64_t c = wrapi(cx0 + sx, a.nc) + (int64_t)a.nc * (wrapi(cy0 + sy, a.nc) + (int64_t)a.nc * wrapi(sz, a.nc));
      cntv = a.cnt[c];
      start[threadIdx.x] = a.off[c];
    }
    const uint32_t total = block_exclusive_scan(cntv, pre, DRC, wsum);
    const uint32_t q64 = total / 64;
    int osh = 4;
    while ((total >> osh) >= (uint32_t)NOWN) ++osh;
    if (threadIdx.x < DRC) {
      const uint32_t lo = pre[threadIdx.x], hi = pre[threadIdx.x + 1];
      for (uint32_t k = (lo + (1u << osh) - 1) >> osh; (k << osh) < hi; ++k) owner[k] = (uint8_t)threadIdx.x;
    }
    __syncthreads();
    auto deposit_layer = [&](auto* acc) {
    using A = typename std::remove_pointer<decltype(acc)>::type;
    // source cell and codes of the layer's it-th particle
    auto fetch = [&](uint32_t it, int& s, int* ch) {
      // interleaved: lane l of the w-th group of 64 takes particle l * (total / 64) + w, so the lanes
      // of one wavefront hold particles of different cells (a bijection on [0, 64 * (total / 64)))
      const uint32_t i = (a.interleave && it < 64 * q64) ? (it % 64) * q64 + it / 64 : it;
      s = owner[i >> osh];
      while (pre[s + 1] <= i) ++s;
      const int64_t p = (int64_t)start[s] + (i - pre[s]);
      ch[0] = (int)cx[p];
      ch[1] = (int)cy[p];
      ch[2] = (int)cz[p];
    };
    // CIC of one particle with source cell s and codes ch
    auto deposit_one = [&](const int s, const int* ch) {
      // the three codes are needed here on every path: without this the compiler may move their
      // uses into the conditional corners and then wait conservatively for later loads as well
      asm volatile("" ::"v"(ch[0]), "v"(ch[1]), "v"(ch[2]));
      const int sl[3] = {s % DR - 1, s / DR - 1, sz};
      int i0[3], w1[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int pl = sl[d] * (1 << (SH + 2)) + 2 * ch[d] + 1 - (1 << (SH - 1));
        i0[d] = pl >> SH;
        w1[d] = pl & ((1 << SH) - 1);
      }
      // weight products: < 2^(3 SH) -- 32-bit arithmetic for 1-byte codes, one 64-bit product else
      const uint32_t wz2[2] = {(uint32_t)((1 << SH) - w1[2]), (uint32_t)w1[2]};
      const uint32_t wy2[2] = {(uint32_t)((1 << SH) - w1[1]), (uint32_t)w1[1]};
      const uint32_t wx2[2] = {(uint32_t)((1 << SH) - w1[0]), (uint32_t)w1[0]};
#pragma unroll
      for (int dz = 0; dz < 2; ++dz) {
        const int pz = i0[2] + dz;
        if (pz < pz0 || pz >= pz1) continue;
        const int sb = slot_of(pz) * DF * DF;
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
          const int y = i0[1] + dy;
          if (y < 0 || y >= DF) continue;
          const uint32_t wzy = wz2[dz] * wy2[dy];
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const int x = i0[0] + dx;
            if (x < 0 || x >= DF) continue;
            const A w = NCHI == 1 ? (A)(wzy * wx2[dx]) : (A)((unsigned long long)wzy * (unsigned long long)wx2[dx]);
            atomicAdd(&acc[sb + y * DF + x], w);
          }
        }
      }
    };
    // software pipeline, unrolled twice so that the two particles' registers alternate: a thread
    // requests the codes of its next particle before it computes the weights and issues the LDS
    // atomics of the current one, so the global-memory latency overlaps them. The requests are
    // unconditional (past the end they repeat the layer's last particle, whose codes go unused) so
    // that the wait for the current codes never waits for the next ones.
    if (total > 0) {
      const uint32_t last = total - 1;
      int s0, s1, ch0[3], ch1[3];
      fetch(min((uint32_t)threadIdx.x, last), s0, ch0);
      for (uint32_t it = threadIdx.x; it < total; it += 2 * BLK) {
        fetch(min(it + BLK, last), s1, ch1);
        deposit_one(s0, ch0);
        if (it + BLK >= total) break;
        fetch(min(it + 2 * BLK, last), s0, ch0);
        deposit_one(s1, ch1);
      }
    }
    };
    if (narrow) deposit_layer(rho32);
    else deposit_layer(rho);
    __syncthreads();
    // planes completed by this layer
    const int f0 = max(4 * sz - 1, pz0), f1 = min(4 * sz + 2, pz1 - 1);
    const int nplanes = f1 - f0 + 1;
    for (int i = threadIdx.x; i < nplanes * DF * DF; i += BLK) {
      const int pz = f0 + i / (DF * DF), e = i % (DF * DF);
      const int y = e / DF, x = e - y * DF;
      const int idx = slot_of(pz) * DF * DF + e;
      double r;
      if (narrow) {
        r = (double)rho32[idx];
        rho32[idx] = 0u;
      } else {
        r = (double)rho[idx];
        rho[idx] = 0ull;
      }
      a.mesh[((int64_t)pz * a.nm + (4 * cy0 + y)) * a.pitch_f + (4 * cx0 + x)] = (float)(r * a.inv_mean - 1.0);
    }
    __syncthreads();
  }
}

template <int NCHI, int BLK>
__global__ __launch_bounds__(BLK) void k_deposit(DepArgs a) {
  deposit_column<NCHI, BLK>(a, xcd_block(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y));
}

// every box of an ensemble in one launch (a box's workgroups: its columns times its z chunks)
template <int NCHI, int BLK>
__global__ __launch_bounds__(BLK) void k_deposit_boxes(BoxTable<DepArgs> t) {
  const unsigned l = xcd_block(blockIdx.x, gridDim.x);
  const int b = box_of(t.first, t.nbox, l);
  deposit_column<NCHI, BLK>(t.args[b], l - t.first[b]);
}

// ---------------------------------------------------------------------------------------------
// Move passes. MODE 0: kick with the potential in the mesh + drift; MODE 1: drift only;
// MODE 2: initial conditions (lattice + Zel'dovich displacement).
// ---------------------------------------------------------------------------------------------
struct MoveArgs {
  const void* chi;
  const void* nu;
  const uint32_t* cnt;
  const uint64_t* off;
  const float* vc;
  const float* vs;
  void* chi_n;
  void* nu_n;
  const uint64_t* off_n;
  const float* vc_n;
  const float* vinv;
  int64_t cap;
  const float* mesh;
  int64_t pitch_f;
  int nm, nc, nt;
  int64_t nc3;
  float kf, df;
  const float* tdec;
  const float* tedge;  // edge table with -inf / +inf sentinels (M + 1 entries)
  const int16_t* tbucket;
  int nbucket;
  int vhalf;
  uint32_t* mig;
  const uint32_t* slot;
  int64_t* mom;
  uint32_t* flags;
  // initial conditions
  const float* psi0;
  const float* psi1;
  const float* psi2;
  int64_t lat_pitch_f;
  int np, q;
  float vfac, lunit;
  // device-side schedule (replayable step graphs): when kd is set, the kick and drift factors of
  // step j = *kstep are kd[2 j] and kd[2 j + 1] instead of kf and df
  const float* kd;
  const int* kstep;
  // particle IDs (Sec. 2.1): pid_bytes 0 (none), 4 or 8; stored in the order of chi and nu
  const void* pid;
  void* pid_n;
  int pid_bytes;
  // adaptive time steps: when set, the count pass raises amax[0] to the largest |v|^2 after the
  // kick and amax[1] to the largest |t|^2 of the interpolated gradient (FP32 bit patterns)
  uint32_t* amax;
  // gradient-tile scatter: polls of the LDS turn word after which a chunk stops waiting for its
  // turn and raises the count error (the wait then ends whatever the other wavefronts do)
  uint32_t turn_limit;
};


__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
  return x;
}

__global__ void k_clear_u32(uint32_t* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// the wave's largest |v|^2 and |t|^2 into the step maxima (non-negative floats order as their bits)
__device__ __forceinline__ void raise_maxima(uint32_t* amax, float vv, float tq) {
  vv = wave_max(vv);
  tq = wave_max(tq);
  if ((threadIdx.x & 63) == 0) {
    if (vv > 0.0f) atomicMax(&amax[0], __float_as_uint(vv));
    if (tq > 0.0f) atomicMax(&amax[1], __float_as_uint(tq));
  }
}

// the ID of the particle at storage index p (steps), or of lattice particle li of tile cell s
// (initial conditions: the lattice index x + N_p (y + N_p z))
template <int MODE>
__device__ __forceinline__ uint64_t particle_id(const MoveArgs& a, const TileGeom& g, int s, int64_t p, uint32_t li) {
  if constexpr (MODE == 2) {
    const int64_t gx = (int64_t)(g.cx0 + s % T) * a.q + li % a.q;
    const int64_t gy = (int64_t)(g.cy0 + (s / T) % T) * a.q + (li / a.q) % a.q;
    const int64_t gz = (int64_t)(g.cz0 + s / (T * T)) * a.q + li / (a.q * a.q);
    return (uint64_t)(gx + a.np * (gy + a.np * gz));
  } else {
    return a.pid_bytes == 8 ? static_cast<const uint64_t*>(a.pid)[p] : static_cast<const uint32_t*>(a.pid)[p];
  }
}

__device__ __forceinline__ void store_id(const MoveArgs& a, uint64_t dst, uint64_t id) {
  if (a.pid_bytes == 8) static_cast<uint64_t*>(a.pid_n)[dst] = id;
  else static_cast<uint32_t*>(a.pid_n)[dst] = (uint32_t)id;
}

// the kick/drift factors of this launch
__device__ __forceinline__ void resolve_factors(MoveArgs& a) {
  if (a.kd) {
    const int j = *a.kstep;
    a.kf = a.kd[2 * j];
    a.df = a.kd[2 * j + 1];
  }
}

// rint(x s) as int64 for a power of two s and |x s| < 2^51: adding 1.5 * 2^52 rounds x s to the
// nearest integer (ties to even, as rint does) in the low mantissa bits; the difference of the bit
// patterns is that integer. x s is exact, so the fused multiply-add rounds once, as the sum would.
__device__ __forceinline__ long long rint_ll(double x, double s) {
  const double magic = 6755399441055744.0;
  return __double_as_longlong(__builtin_fma(x, s, magic)) - __double_as_longlong(magic);
}

// fixed-point velocity moments of one particle: rint(v_d 2^32) and sum_d rint(v_d^2 2^24). The
// second needs |v| < 2^13.5 for rint_ll; larger speeds (up to the 2^15 overflow limit) take the
// general conversion, decided per wavefront.
__device__ __forceinline__ void velocity_moments(const float* v, long long* q) {
  const bool big = fabsf(v[0]) >= 8192.0f || fabsf(v[1]) >= 8192.0f || fabsf(v[2]) >= 8192.0f;
  q[3] = 0;
  if (__ballot(big) == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double vd = (double)v[d];
      q[d] = rint_ll(vd, 4294967296.0);
      q[3] += rint_ll(vd * vd, 16777216.0);
    }
  } else {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double vd = (double)v[d];
      q[d] = rint_ll(vd, 4294967296.0);
      q[3] += __double2ll_rn(vd * vd * 16777216.0);
    }
  }
}

struct Moved {
  float v[3];
  int k[3];
  int chi[3];
  bool ok;
  float vv, tq;  // |v|^2 after the kick and |t|^2 of the interpolated gradient (step passes)
};

constexpr int DG = F + 2;  // precomputed-gradient tile side: fine cells -1 .. F of the tile

// Gradient source: either the potential tile (4-point difference per corner) or the tile of
// precomputed unnormalised gradients D = 8 (phi[i+1] - phi[i-1]) - (phi[i+2] - phi[i-2]).
template <bool PRE>
__device__ __forceinline__ float grad_at(const float* ph, const float* gd, int d, int x, int y, int z) {
  // (x, y, z): fine cell relative to the tile origin, in -1 .. F
  if constexpr (PRE) {
    return gd[d * DG * DG * DG + ((z + 1) * DG + (y + 1)) * DG + (x + 1)];
  } else {
    const int e = d == 0 ? 1 : (d == 1 ? PH : PH * PH);
    const int b = ((z + 3) * PH + (y + 3)) * PH + (x + 3);
    const float aa = ph[b + e] - ph[b - e];
    const float bb = ph[b + 2 * e] - ph[b - 2 * e];
    return __builtin_fmaf(8.0f, aa, -bb);  // 8 aa is exact: the same value as 8 aa - bb
  }
}

// New coarse cell along one dimension: k in {-1, 0, 1}, the code of the position inside it, and
// whether the value is usable; a non-finite value, a move beyond one coarse cell or a speed beyond
// the range of the moment accumulators raises its error flag. In range (the usual case) only the
// first branch runs; NaN fails its comparisons.
template <int SH>
__device__ __forceinline__ bool new_cell(float ln, float vd, uint32_t* flags, int& k, int& cq) {
  bool ok = true;
  float lw;
  if (ln >= -4.0f && ln < 8.0f && fabsf(vd) < 32768.0f) {
    k = ln < 0.0f ? -1 : (ln >= 4.0f ? 1 : 0);
    lw = __builtin_fmaf(-4.0f, (float)k, ln);  // ln, ln + 4 or ln - 4, each one rounding
  } else {
    k = 0;
    lw = ln;
    if (!(ln == ln) || fabsf(ln) == INFINITY || !(vd == vd) || fabsf(vd) == INFINITY) {
      set_flag(flags, FLAG_NONFINITE);
      ok = false;
      lw = 0.0f;
    } else if (ln < -4.0f || ln >= 8.0f) {
      set_flag(flags, FLAG_CFL);
      ok = false;
      lw = 0.0f;
    } else if (ln < 0.0f) {
      k = -1;
      lw = ln + 4.0f;
    } else if (ln >= 4.0f) {
      k = 1;
      lw = ln - 4.0f;
    }
    if (fabsf(vd) >= 32768.0f) {
      set_flag(flags, FLAG_OVERFLOW);
      ok = false;
    }
  }
  int q = (int)floorf(lw * (float)(1 << (SH - 1)));
  cq = q < 0 ? 0 : (q > (1 << (SH + 1)) - 1 ? (1 << (SH + 1)) - 1 : q);
  return ok;
}

template <int NCHI, int NNU, int MODE, bool PRE, bool MEAS = false>
__device__ __forceinline__ Moved move_particle(const MoveArgs& a, const float* ph, const float* gd, int s, int64_t p,
                                               uint32_t li, const TileGeom& g) {
  using CT = chi_t<NCHI>;
  using NT = nu_t<NNU>;
  constexpr int SH = 8 * NCHI - 1;
  const int o[3] = {s % T, (s / T) % T, s / (T * T)};
  const int64_t c = (g.cx0 + o[0]) + (int64_t)a.nc * ((g.cy0 + o[1]) + (int64_t)a.nc * (g.cz0 + o[2]));
  float l[3], v[3];
  Moved m;
  m.vv = 0.0f;
  m.tq = 0.0f;
  if constexpr (MODE == 2) {
    const int lat[3] = {(int)(li % a.q), (int)((li / a.q) % a.q), (int)(li / (a.q * a.q))};
    const int64_t gx = (int64_t)(g.cx0 + o[0]) * a.q + lat[0];
    const int64_t gy = (int64_t)(g.cy0 + o[1]) * a.q + lat[1];
    const int64_t gz = (int64_t)(g.cz0 + o[2]) * a.q + lat[2];
    const int64_t pi = (gz * a.np + gy) * a.lat_pitch_f + gx;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float ps = (d == 0 ? a.psi0 : (d == 1 ? a.psi1 : a.psi2))[pi];
      const float l0 = (float)(2 * lat[d] + 1) * a.lunit;
      v[d] = a.vfac * ps;
      l[d] = l0 + ps;
    }
  } else {
    const CT* chi = static_cast<const CT*>(a.chi);
    const NT* nu = static_cast<const NT*>(a.nu);
    const float unit = (float)(1.0 / (double)(1 << SH));
    int ch[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      ch[d] = (int)chi[d * a.cap + p];
      l[d] = (float)(2 * ch[d] + 1) * unit;
      int nuv = (int)nu[d * a.cap + p];
      nuv = nuv < -a.vhalf ? -a.vhalf : (nuv > a.vhalf ? a.vhalf : nuv);
      v[d] = __builtin_fmaf(a.vs[c], a.tdec[nuv + a.vhalf], a.vc[d * a.nc3 + c]);
    }
    if constexpr (MODE == 0) {
      // CIC corners (fine cells relative to the tile origin) and exact dyadic weights
      int i0[3];
      float w0[3], w1[3];
      const float wunit = (float)(1.0 / (double)(1 << SH));
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int pl = o[d] * (1 << (SH + 2)) + 2 * ch[d] + 1 - (1 << (SH - 1));
        i0[d] = pl >> SH;
        const int f = pl & ((1 << SH) - 1);
        w1[d] = (float)f * wunit;
        w0[d] = 1.0f - w1[d];  // exact: both are multiples of 2^-SH in [0, 1]
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        float sacc[2];
#pragma unroll
        for (int cz = 0; cz < 2; ++cz) {
          float racc[2];
#pragma unroll
          for (int cy = 0; cy < 2; ++cy) {
            const float d0 = grad_at<PRE>(ph, gd, d, i0[0], i0[1] + cy, i0[2] + cz);
            const float d1 = grad_at<PRE>(ph, gd, d, i0[0] + 1, i0[1] + cy, i0[2] + cz);
            racc[cy] = __builtin_fmaf(w1[0], d1, w0[0] * d0);
          }
          sacc[cz] = __builtin_fmaf(w1[1], racc[1], w0[1] * racc[0]);
        }
        const float t = __builtin_fmaf(w1[2], sacc[1], w0[2] * sacc[0]);
        v[d] = __builtin_fmaf(t, a.kf, v[d]);
        if constexpr (MEAS) m.tq = d == 0 ? t * t : m.tq + t * t;
      }
      if constexpr (MEAS) m.vv = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) l[d] = __builtin_fmaf(v[d], a.df, l[d]);
  }
  m.ok = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int k, cq;
    if (!new_cell<SH>(l[d], v[d], a.flags, k, cq)) m.ok = false;
    m.k[d] = k;
    m.chi[d] = cq;
    m.v[d] = m.ok ? v[d] : 0.0f;
  }
  return m;
}

// Potential tile (fine cells -3 .. F+2 of the tile, wrapped) and, with PRE, the unnormalised
// 4-point gradient of every corner cell -1 .. F. The gradient uses the same IEEE operations as the
// per-corner evaluation, so both paths give identical bits.
template <int MODE, bool PRE, int NTH>
__device__ __forceinline__ void load_potential(const MoveArgs& a, float* ph, float* gd, const TileGeom& g) {
  if constexpr (MODE == 0) {
    const int fx0 = g.cx0 * 4 - 3, fy0 = g.cy0 * 4 - 3, fz0 = g.cz0 * 4 - 3;
    const int64_t plane = (int64_t)a.nm * a.pitch_f;
    // all loads of the tile in flight at once, then into LDS
    if (fx0 >= 0 && fy0 >= 0 && fz0 >= 0 && fx0 + PH <= a.nm && fy0 + PH <= a.nm && fz0 + PH <= a.nm &&
        plane < (1 << 26)) {
      // the halo does not cross the box boundary: element e of the tile lies at a 32-bit offset
      // from the tile's first element (below 22 planes of fewer than 2^26 floats); its row index
      // z nm + y and the row pitch are below 2^24, so 24-bit multiplies form the offset
      const float* src = a.mesh + (int64_t)fz0 * plane + (int64_t)fy0 * a.pitch_f + fx0;
      const uint32_t nmu = (uint32_t)a.nm, rs = (uint32_t)a.pitch_f;
      constexpr int NE = PH * PH * PH;
      constexpr int NL = (NE + NTH - 1) / NTH;
      float stage[NL];
#pragma unroll
      for (int k = 0; k < NL; ++k) {
        const uint32_t e = threadIdx.x + k * NTH;
        if (NE % NTH == 0 || e < (uint32_t)NE) {
          const uint32_t q = e / PH, x = e - q * PH;
          const uint32_t z = q / PH, y = q - z * PH;
          stage[k] = src[__umul24(__umul24(z, nmu) + y, rs) + x];
        }
      }
#pragma unroll
      for (int k = 0; k < NL; ++k) {
        const uint32_t e = threadIdx.x + k * NTH;
        if (NE % NTH == 0 || e < (uint32_t)NE) ph[e] = stage[k];
      }
    } else {
      // half-waves take rows (z, y), wrapped periodically; lanes take x
      const int hw = threadIdx.x >> 5, x = threadIdx.x & 31;
      const int gx = wrapi(fx0 + x, a.nm);
      constexpr int NR = (PH * PH + NTH / 32 - 1) / (NTH / 32);
      float stage[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const int r = hw + k * (NTH / 32);
        if (x < PH && r < PH * PH) {
          const int z = r / PH, y = r - z * PH;
          const int gy = wrapi(fy0 + y, a.nm), gz = wrapi(fz0 + z, a.nm);
          stage[k] = a.mesh[((int64_t)gz * a.nm + gy) * a.pitch_f + gx];
        }
      }
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const int r = hw + k * (NTH / 32);
        if (x < PH && r < PH * PH) ph[r * PH + x] = stage[k];
      }
    }
    if constexpr (PRE) {
      __syncthreads();
      const int hw = threadIdx.x >> 5, x = threadIdx.x & 31;
      for (int r = hw; r < DG * DG; r += NTH / 32) {
        if (x < DG) {
          const int z = r / DG, y = r - z * DG;
          const int i = r * DG + x;
#pragma unroll
          for (int d = 0; d < 3; ++d) gd[d * DG * DG * DG + i] = grad_at<false>(ph, gd, d, x - 1, y - 1, z - 1);
        }
      }
    }
  }
}

// own cells of the tile: counts, starts and the exclusive prefix
template <int MODE>
__device__ __forceinline__ uint32_t own_cells(const MoveArgs& a, const TileGeom& g, uint32_t* pre, uint64_t* start,
                                              uint32_t* wsum) {
  uint32_t cntv = 0;
  if (threadIdx.x < TC) {
    const int s = threadIdx.x;
    const int64_t c = (g.cx0 + s % T) + (int64_t)a.nc * ((g.cy0 + (s / T) % T) + (int64_t)a.nc * (g.cz0 + s / (T * T)));
    if constexpr (MODE == 2) {
      cntv = (uint32_t)(a.q * a.q * a.q);
      start[s] = (uint64_t)c * cntv;
    } else {
      cntv = a.cnt[c];
      start[s] = a.off[c];
    }
  }
  return block_exclusive_scan(cntv, pre, TC, wsum);
}

// Each wave owns a contiguous run of whole cells holding about total/W particles, so that a cell
// is never shared between waves (ranks need no ordering across waves).
__device__ __forceinline__ void wave_cells(const uint32_t* pre, uint32_t total, int wave, int nwaves, int& c0, int& c1) {
  auto lower = [&](uint64_t t) {
    int lo = 0, hi = TC;  // smallest s with pre[s] >= t
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((uint64_t)pre[mid] < t) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  };
  c0 = wave == 0 ? 0 : lower((uint64_t)total * wave / nwaves);
  c1 = wave == nwaves - 1 ? TC : lower((uint64_t)total * (wave + 1) / nwaves);
}

__device__ __forceinline__ int find_cell_in(const uint32_t* pre, int lo, int hi, uint32_t i) {
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The tile's per (own cell, displacement) counts (LDS, [cell][27]) to mig[d][cell]: a wavefront
// writes one displacement of all 64 own cells, a lane per cell, so the array offset is uniform.
template <int NTH>
__device__ __forceinline__ void flush_counts(const MoveArgs& a, const TileGeom& g, const uint32_t* cnt) {
  static_assert(TC == 64 && NTH % 64 == 0, "one lane per own cell");
  const int s = threadIdx.x & 63;
  uint32_t* const col = a.mig + (g.cx0 + (int64_t)a.nc * (g.cy0 + (int64_t)a.nc * g.cz0)) + s % T +
                        (int64_t)a.nc * ((s / T) % T) + (int64_t)a.nc * a.nc * (s / (T * T));
  for (int d = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); d < 27; d += NTH / 64) col[d * a.nc3] = cnt[s * 27 + d];
}

template <int MODE, bool PRE>
struct MoveLds {
  static constexpr int kPh = MODE == 0 ? PH * PH * PH : 1;
  static constexpr int kGd = (MODE == 0 && PRE) ? 3 * DG * DG * DG : 1;
  // moments: in LDS over the tile and its ring, flushed at the end; with the potential tile in LDS
  // (MODE 0) they go to the global accumulators directly, so that three workgroups fit a CU
  static constexpr bool kGlobalMom = MODE == 0;
  static constexpr int kMom = kGlobalMom ? TC * 4 : RC * 4;  // own cells only, or tile and ring
};

// count pass over one tile (logical block lb of the box)
template <int NCHI, int NNU, int MODE, bool PRE, int NTH, bool MEAS>
__device__ __forceinline__ void move_count_tile(MoveArgs a, const unsigned lb) {
  resolve_factors(a);
  using L = MoveLds<MODE, PRE>;
  __shared__ float ph[L::kPh];
  __shared__ float gd[L::kGd];
  __shared__ uint32_t mcnt[TC * 27];
  __shared__ unsigned long long mom[L::kMom];
  __shared__ uint32_t pre[TC + 1];
  __shared__ uint64_t start[TC];
  __shared__ uint32_t wsum[NTH / 64];
  const TileGeom g = tile_of(lb, a.nt);
  load_potential<MODE, PRE, NTH>(a, ph, gd, g);
  for (int i = threadIdx.x; i < TC * 27; i += NTH) mcnt[i] = 0u;
  for (int i = threadIdx.x; i < L::kMom; i += NTH) mom[i] = 0ull;
  const uint32_t total = own_cells<MODE>(a, g, pre, start, wsum);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int c0, c1;
  wave_cells(pre, total, wave, NTH / 64, c0, c1);
  const uint32_t p0 = pre[c0], p1 = pre[c1];
  for (uint32_t base = p0; base < p1; base += 64) {
    const uint32_t i = base + lane;
    const bool active = i < p1;  // active lanes form a prefix of the wave
    int key = -1, r = 0;
    long long q[4];
    float vm[3] = {0.f, 0.f, 0.f};
    float vv = 0.f, tq = 0.f;
    if (active) {
      const int s = find_cell_in(pre, c0, c1, i);
      const uint32_t li = i - pre[s];
      const int64_t p = (int64_t)start[s] + li;
      const Moved m = move_particle<NCHI, NNU, MODE, PRE, MEAS>(a, ph, gd, s, p, li, g);
      const int dcode = (m.k[2] + 1) * 9 + (m.k[1] + 1) * 3 + (m.k[0] + 1);
      key = s * 27 + dcode;
      r = (s % T + 1 + m.k[0]) + RG * ((s / T) % T + 1 + m.k[1]) + RG * RG * (s / (T * T) + 1 + m.k[2]);
      vm[0] = m.v[0];
      vm[1] = m.v[1];
      vm[2] = m.v[2];
      vv = m.vv;
      tq = m.tq;
    }
    if constexpr (MEAS) raise_maxima(a.amax, vv, tq);
    velocity_moments(vm, q);
    // sum over runs of consecutive lanes with the same (cell, displacement): most particles stay
    // in their cell, so one atomic per run replaces up to 64 conflicting ones
    const int kprev = __shfl_up(key, 1, 64);
    const bool head = lane == 0 || kprev != key;
    // st: the first lane of this lane's run, the highest run head at or below it (lane 0 is one)
    const unsigned long long heads = __ballot(head);
    const int st = 63 - __clzll(heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull)));
    // run sums from one prefix scan: the scan at the lane minus the scan before the run
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const unsigned long long ps = wave_scan_u64((unsigned long long)q[d]);
      const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)ps, st - 1, 64);
      const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(ps >> 32), st - 1, 64);
      const unsigned long long before = st > 0 ? (((unsigned long long)hi << 32) | lo) : 0ull;
      q[d] = (long long)(ps - before);
    }
    const int knext = __shfl_down(key, 1, 64);
    const bool tail = lane == 63 || knext != key;
    if (active && tail) {
      atomicAdd(&mcnt[key], (uint32_t)(lane - st + 1));
      if constexpr (L::kGlobalMom) {
        // new cell inside the tile: the tile's LDS accumulators; in the ring: the global ones
        const int rx = r % RG, ry = (r / RG) % RG, rz = r / (RG * RG);
        if (rx >= 1 && rx <= T && ry >= 1 && ry <= T && rz >= 1 && rz <= T) {
          const int so = (rx - 1) + T * ((ry - 1) + T * (rz - 1));
#pragma unroll
          for (int d = 0; d < 4; ++d) atomicAdd(&mom[so * 4 + d], (unsigned long long)q[d]);
        } else {
          const int gx = wrapi(g.cx0 - 1 + rx, a.nc), gy = wrapi(g.cy0 - 1 + ry, a.nc);
          const int gz = wrapi(g.cz0 - 1 + rz, a.nc);
          const int64_t cn = gx + (int64_t)a.nc * (gy + (int64_t)a.nc * gz);
#pragma unroll
          for (int d = 0; d < 4; ++d)
            atomicAdd(reinterpret_cast<unsigned long long*>(&a.mom[d * a.nc3 + cn]), (unsigned long long)q[d]);
        }
      } else {
#pragma unroll
        for (int d = 0; d < 4; ++d) atomicAdd(&mom[r * 4 + d], (unsigned long long)q[d]);
      }
    }
  }
  __syncthreads();
  flush_counts<NTH>(a, g, mcnt);
  if constexpr (L::kGlobalMom) {
    for (int i = threadIdx.x; i < TC * 4; i += NTH) {
      const unsigned long long v = mom[i];
      if (v == 0ull) continue;
      const int so = i / 4, q = i % 4;
      const int64_t c = (g.cx0 + so % T) + (int64_t)a.nc * ((g.cy0 + (so / T) % T) + (int64_t)a.nc * (g.cz0 + so / (T * T)));
      atomicAdd(reinterpret_cast<unsigned long long*>(&a.mom[q * a.nc3 + c]), v);
    }
  } else {
    for (int i = threadIdx.x; i < RC * 4; i += NTH) {
      const unsigned long long v = mom[i];
      if (v == 0ull) continue;
      const int r = i / 4, q = i % 4;
      const int gx = wrapi(g.cx0 - 1 + r % RG, a.nc), gy = wrapi(g.cy0 - 1 + (r / RG) % RG, a.nc);
      const int gz = wrapi(g.cz0 - 1 + r / (RG * RG), a.nc);
      const int64_t c = gx + (int64_t)a.nc * (gy + (int64_t)a.nc * gz);
      atomicAdd(reinterpret_cast<unsigned long long*>(&a.mom[q * a.nc3 + c]), v);
    }
  }
}

// at least six wavefronts per SIMD (three 512-thread workgroups per CU): at most 80 VGPRs
template <int NCHI, int NNU, int MODE, bool PRE, int NTH, bool MEAS = false>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(6))) void k_move_count(MoveArgs a) {
  move_count_tile<NCHI, NNU, MODE, PRE, NTH, MEAS>(a, xcd_block(blockIdx.x, gridDim.x));
}

// every box of an ensemble in one launch (a box's workgroups: its tiles)
template <int NCHI, int NNU, int MODE, bool PRE, int NTH>
__global__ __launch_bounds__(NTH) __attribute__((amdgpu_waves_per_eu(6))) void k_move_count_boxes(BoxTable<MoveArgs> t) {
  const unsigned l = xcd_block(blockIdx.x, gridDim.x);
  const int b = box_of(t.first, t.nbox, l);
  move_count_tile<NCHI, NNU, MODE, PRE, NTH, false>(t.args[b], l - t.first[b]);
}

// Eq. (nu) by the edge table: the code nu with ext[nu + h] <= u < ext[nu + h + 1] (h = (M-1)/2;
// ext is the edge table with -inf and +inf at its ends), i.e. -h + #{edges <= u}. A bucket table
// over t = u / (1 + |u|) gives the code at the lower end of the bucket. Every bucket holds at most
// one edge (checked when the tables are built) and t, from an approximate reciprocal, is off by
// far less than a bucket width, so the bucket found is the right one or a neighbour and the start
// is within two codes of the answer; each exact step moves one code towards it, so two steps
// reach it. With CHECKED, loops behind them (then never entered) keep the result exact whatever
// the start. The sentinels keep every read inside the table, NaN included.
template <bool CHECKED, typename BT>
__device__ __forceinline__ int encode_nu(float u, const float* ext, const BT* bucket, int nbucket, int vhalf) {
  const float t = u * __builtin_amdgcn_rcpf(1.0f + fabsf(u));
  int b = (int)((t + 1.0f) * (0.5f * (float)nbucket));
  b = b < 0 ? 0 : (b > nbucket - 1 ? nbucket - 1 : b);
  int nu = bucket[b];
#pragma unroll
  for (int r = 0; r < 2; ++r) nu += (int)(u >= ext[nu + vhalf + 1]) - (int)(u < ext[nu + vhalf]);
  if constexpr (CHECKED) {
    while (u >= ext[nu + vhalf + 1]) ++nu;
    while (u < ext[nu + vhalf]) --nu;
  }
  return nu;
}

template <int NCHI, int NNU, int MODE, bool PRE, int NTH>
__device__ __forceinline__ void move_scatter_tile(MoveArgs a, const unsigned lb) {
  resolve_factors(a);
  using CT = chi_t<NCHI>;
  using NT = nu_t<NNU>;
  __shared__ float ph[MoveLds<MODE, PRE>::kPh];
  __shared__ float gd[MoveLds<MODE, PRE>::kGd];
  __shared__ uint32_t grp[TC * 27];
  __shared__ uint32_t pre[TC + 1];
  __shared__ uint64_t start[TC];
  __shared__ uint32_t wsum[NTH / 64];
  __shared__ float edges_lds[NNU == 1 ? 256 : 1];
  __shared__ int16_t bucket_lds[NNU == 1 ? 1024 : 1];
  // the flag word is requested first and tested after the set-up (the last barrier): a wave that
  // returns then cannot hold up the others
  const uint32_t failed = __atomic_load_n(a.flags, __ATOMIC_RELAXED);
  const TileGeom g = tile_of(lb, a.nt);
  load_potential<MODE, PRE, NTH>(a, ph, gd, g);
  for (int i = threadIdx.x; i < TC * 27; i += NTH) grp[i] = 0u;
  const int nedge = 2 * a.vhalf + 2;
  if constexpr (NNU == 1) {
    for (int i = threadIdx.x; i < nedge; i += NTH) edges_lds[i] = a.tedge[i];
    for (int i = threadIdx.x; i < a.nbucket; i += NTH) bucket_lds[i] = a.tbucket[i];
  }
  const float* edges = (NNU == 1) ? edges_lds : a.tedge;
  const int16_t* bucket = (NNU == 1) ? bucket_lds : a.tbucket;
  const uint32_t total = own_cells<MODE>(a, g, pre, start, wsum);
  if (__builtin_amdgcn_readfirstlane(failed)) return;  // a failed step is not applied
  CT* chi_n = static_cast<CT*>(a.chi_n);
  NT* nu_n = static_cast<NT*>(a.nu_n);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long lt = (1ull << lane) - 1ull;
  int c0, c1;
  wave_cells(pre, total, wave, NTH / 64, c0, c1);
  const uint32_t p0 = pre[c0], p1 = pre[c1];
  // particles of this wave's cells in storage order; the running count per (source cell,
  // displacement) gives every particle its rank inside the new cell
  for (uint32_t base = p0; base < p1; base += 64) {
    const uint32_t i = base + lane;
    const bool active = i < p1;
    Moved m{};
    int s = c0, key = 0, dcode = 0;
    if (active) {
      s = find_cell_in(pre, c0, c1, i);
      const uint32_t li = i - pre[s];
      const int64_t p = (int64_t)start[s] + li;
      m = move_particle<NCHI, NNU, MODE, PRE>(a, ph, gd, s, p, li, g);
      dcode = (m.k[2] + 1) * 9 + (m.k[1] + 1) * 3 + (m.k[0] + 1);
      key = s * 27 + dcode;
    }
    unsigned long long peers = __ballot(active);
#pragma unroll
    for (int b = 0; b < 11; ++b) {
      const bool bit = (key >> b) & 1;
      const unsigned long long bb = __ballot(active && bit);
      peers &= bit ? bb : ~bb;
    }
    const int rin = __popcll(peers & lt);
    const int leader = active ? __ffsll((long long)peers) - 1 : lane;
    uint32_t gbase = 0;
    if (active && rin == 0) {
      gbase = grp[key];
      grp[key] = gbase + (uint32_t)__popcll(peers);
    }
    gbase = (uint32_t)__shfl((int)gbase, leader, 64);
    if (active) {
      int ox, oy, oz;
      tile_xyz(s, ox, oy, oz);
      const int nx = wrapi(g.cx0 + ox + m.k[0], a.nc), ny = wrapi(g.cy0 + oy + m.k[1], a.nc);
      const int nz = wrapi(g.cz0 + oz + m.k[2], a.nc);
      const int64_t cn = nx + (int64_t)a.nc * (ny + (int64_t)a.nc * nz);
      const uint64_t dst = a.off_n[cn] + a.slot[(int64_t)(26 - dcode) * a.nc3 + cn] + gbase + (uint32_t)rin;
      if (dst < (uint64_t)a.cap) {
        const float inv = a.vinv[cn];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const float u = (m.v[d] - a.vc_n[d * a.nc3 + cn]) * inv;
          nu_n[d * a.cap + dst] = (NT)encode_nu<false>(u, edges, bucket, a.nbucket, a.vhalf);
          chi_n[d * a.cap + dst] = (CT)m.chi[d];
        }
        if (a.pid_bytes) store_id(a, dst, particle_id<MODE>(a, g, s, (int64_t)start[s] + (i - pre[s]), i - pre[s]));
      } else {
        set_flag(a.flags, FLAG_COUNT);
      }
    }
  }
}

template <int NCHI, int NNU, int MODE, bool PRE, int NTH>
__global__ __launch_bounds__(NTH) void k_move_scatter(MoveArgs a) {
  move_scatter_tile<NCHI, NNU, MODE, PRE, NTH>(a, xcd_block(blockIdx.x, gridDim.x));
}

template <int NCHI, int NNU, int MODE, bool PRE, int NTH>
__global__ __launch_bounds__(NTH) void k_move_scatter_boxes(BoxTable<MoveArgs> t) {
  const unsigned l = xcd_block(blockIdx.x, gridDim.x);
  const int b = box_of(t.first, t.nbox, l);
  move_scatter_tile<NCHI, NNU, MODE, PRE, NTH>(t.args[b], l - t.first[b]);
}

// ---------------------------------------------------------------------------------------------
// Dense move passes (at least half as many particles as fine cells): one coarse cell per wave at
// a time, so the cell's offset, mean velocity and scale are wave-uniform; the stayers of a cell
// (the large majority) are summed with one cross-lane reduction; particles of a cell are visited
// in storage order by a single wave, which makes the running rank per displacement exact.
// ---------------------------------------------------------------------------------------------

template <int NCHI, int NNU, bool SCATTER, bool MEAS>
__device__ __forceinline__ void move_dense_tile(MoveArgs a, const unsigned lb) {
  resolve_factors(a);
  using CT = chi_t<NCHI>;
  using NT = nu_t<NNU>;
  constexpr int NTH = 1024;
  constexpr int SH = 8 * NCHI - 1;
  // one region holds the potential tile, then the gradient tile computed from it: with the
  // moments added to the global accumulators directly, two workgroups fit a CU
  constexpr int NG = 3 * DG * DG * DG;
  static_assert(PH * PH * PH <= NG, "the potential tile must fit the gradient region");
  __shared__ float tile[NG];
  float* const ph = tile;
  float* const gd = tile;
  __shared__ uint32_t grp[TC * 27];              // count pass: per (cell, displacement) counts; scatter: ranks
  __shared__ uint32_t pre[TC + 1];
  __shared__ uint64_t start[TC];
  __shared__ uint32_t wsum[NTH / 64];
  __shared__ float tdec_lds[NNU == 1 ? 255 : 1];
  __shared__ float edges_lds[(SCATTER && NNU == 1) ? 256 : 1];
  __shared__ int8_t bucket_lds[(SCATTER && NNU == 1) ? 1024 : 1];  // 1-byte codes fit int8
  const TileGeom g = tile_of(lb, a.nt);
  // scatter: the flag word is requested first and tested after the set-up (the last barrier)
  const uint32_t failed = SCATTER ? __atomic_load_n(a.flags, __ATOMIC_RELAXED) : 0u;
  // mean velocity and decode scale of the tile's cells
  __shared__ float4 cellv[TC];
  uint32_t cnt_r = 0;  // particle count of own cell threadIdx.x
  {
    // every global read of the set-up in flight at once: the code tables, the own cells' counts,
    // starts, mean velocities and decode scales, then the potential tile
    static_assert(NTH >= 1024 && NTH >= TC, "one table entry and at most one own cell per thread");
    float tdec_r = 0.0f, edge_r = 0.0f;
    int bucket_r = 0;
    if constexpr (NNU == 1) {
      if (threadIdx.x < 255) tdec_r = a.tdec[threadIdx.x];
      if constexpr (SCATTER) {
        if (threadIdx.x < 256) edge_r = a.tedge[threadIdx.x];
        if ((int)threadIdx.x < a.nbucket) bucket_r = a.tbucket[threadIdx.x];
      }
    }
    float4 cv_r = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    uint64_t start_r = 0;
    if (threadIdx.x < TC) {
      const int sx = threadIdx.x;
      const int64_t c = (g.cx0 + sx % T) + (int64_t)a.nc * ((g.cy0 + (sx / T) % T) + (int64_t)a.nc * (g.cz0 + sx / (T * T)));
      cnt_r = a.cnt[c];
      start_r = a.off[c];
      cv_r = make_float4(a.vc[c], a.vc[a.nc3 + c], a.vc[2 * a.nc3 + c], a.vs[c]);
    }
    load_potential<0, false, NTH>(a, ph, nullptr, g);
    if constexpr (NNU == 1) {
      if (threadIdx.x < 255) tdec_lds[threadIdx.x] = tdec_r;
      if constexpr (SCATTER) {
        if (threadIdx.x < 256) edges_lds[threadIdx.x] = edge_r;
        if ((int)threadIdx.x < a.nbucket) bucket_lds[threadIdx.x] = (int8_t)bucket_r;
      }
    }
    if (threadIdx.x < TC) {
      cellv[threadIdx.x] = cv_r;
      start[threadIdx.x] = start_r;
    }
  }
  __syncthreads();
  {
    // gradient of every corner cell -1 .. F of the tile, over the potential: the z component lies
    // beyond the potential tile and is stored at once; x and y go through registers
    constexpr int G3 = DG * DG * DG;
    static_assert(2 * G3 >= PH * PH * PH, "the z gradient must not overlap the potential tile");
    constexpr int K = (G3 + NTH - 1) / NTH;
    auto grad_of = [&](int d, int i) {
      const int z = i / (DG * DG), y = (i / DG) % DG, x = i % DG;
      return grad_at<false>(ph, nullptr, d, x - 1, y - 1, z - 1);
    };
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = threadIdx.x + k * NTH;
      if (G3 % NTH == 0 || i < G3) gd[2 * G3 + i] = grad_of(2, i);
    }
    float gx[K], gy[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = threadIdx.x + k * NTH;
      if (G3 % NTH == 0 || i < G3) {
        gx[k] = grad_of(0, i);
        gy[k] = grad_of(1, i);
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = threadIdx.x + k * NTH;
      if (G3 % NTH == 0 || i < G3) {
        gd[i] = gx[k];
        gd[G3 + i] = gy[k];
      }
    }
  }
  for (int i = threadIdx.x; i < TC * 27; i += NTH) grp[i] = 0u;
  // scatter: [0] the number of the tile's chunks ranked so far, [1] set if a wait gave up
  __shared__ uint32_t turn[2];
  if (threadIdx.x == 0) turn[0] = turn[1] = 0u;
  const float* tdec = NNU == 1 ? tdec_lds : a.tdec;
  const float* edges = NNU == 1 ? edges_lds : a.tedge;
  using BT = std::conditional_t<NNU == 1, int8_t, int16_t>;
  const BT* bucket;
  if constexpr (NNU == 1) bucket = bucket_lds;
  else bucket = a.tbucket;
  // count pass: moments of the new cells inside the tile, flushed to the global accumulators at the end
  __shared__ unsigned long long omom[SCATTER ? 1 : TC * 4];
  if constexpr (!SCATTER)
    for (int i = threadIdx.x; i < TC * 4; i += NTH) omom[i] = 0ull;
  block_exclusive_scan(cnt_r, pre, TC, wsum);  // ends with a barrier
  if (SCATTER && __builtin_amdgcn_readfirstlane(failed)) return;  // a failed step is not applied
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const unsigned long long lt = (1ull << lane) - 1ull;
  const float unit = (float)(1.0 / (double)(1 << SH));
  CT* chi_n = static_cast<CT*>(a.chi_n);
  NT* nu_n = static_cast<NT*>(a.nu_n);
  // kick, drift, new cell and code of one particle (cell s at tile offsets (ci, o1, o2), codes chc,
  // nuc); inactive lanes keep v = l = 0
  auto physics = [&](bool active, int s, int ci, int o1, int o2, const int* chc, const int* nuc, float* v, int* k,
                     int* cq) {
    float l[3] = {0.f, 0.f, 0.f};
    v[0] = v[1] = v[2] = 0.f;
    float vv = 0.f, tq = 0.f;
    int ch[3] = {0, 0, 0};
    if (active) {
      const float4 cv = cellv[s];
      const float vcv[3] = {cv.x, cv.y, cv.z};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        ch[d] = chc[d];
        int nuv = nuc[d];
        nuv = nuv < -a.vhalf ? -a.vhalf : (nuv > a.vhalf ? a.vhalf : nuv);
        l[d] = (float)(2 * ch[d] + 1) * unit;
        v[d] = __builtin_fmaf(cv.w, tdec[nuv + a.vhalf], vcv[d]);
      }
      // CIC corners relative to the tile, exact dyadic weights, interpolated gradient
      const int o[3] = {ci, o1, o2};
      int i0[3];
      float w0[3], w1[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int pl = o[d] * (1 << (SH + 2)) + 2 * ch[d] + 1 - (1 << (SH - 1));
        i0[d] = pl >> SH;
        const int f = pl & ((1 << SH) - 1);
        w1[d] = (float)f * unit;
        w0[d] = 1.0f - w1[d];  // exact: both are multiples of 2^-SH in [0, 1]
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        float sacc[2];
#pragma unroll
        for (int cz = 0; cz < 2; ++cz) {
          float racc[2];
#pragma unroll
          for (int cy = 0; cy < 2; ++cy) {
            const float d0 = grad_at<true>(ph, gd, d, i0[0], i0[1] + cy, i0[2] + cz);
            const float d1 = grad_at<true>(ph, gd, d, i0[0] + 1, i0[1] + cy, i0[2] + cz);
            racc[cy] = __builtin_fmaf(w1[0], d1, w0[0] * d0);
          }
          sacc[cz] = __builtin_fmaf(w1[1], racc[1], w0[1] * racc[0]);
        }
        const float t = __builtin_fmaf(w1[2], sacc[1], w0[2] * sacc[0]);
        v[d] = __builtin_fmaf(t, a.kf, v[d]);
        if constexpr (MEAS) tq = d == 0 ? t * t : tq + t * t;
      }
      if constexpr (MEAS) vv = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
#pragma unroll
      for (int d = 0; d < 3; ++d) l[d] = __builtin_fmaf(v[d], a.df, l[d]);
    }
    if constexpr (MEAS) raise_maxima(a.amax, vv, tq);
    // new cell, codes, flags (same rules as the generic path)
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (!new_cell<SH>(l[d], v[d], a.flags, k[d], cq[d])) ok = false;
    if (!ok) {
#pragma unroll
      for (int d = 0; d < 3; ++d) v[d] = 0.0f;
    }
  };
  // Both passes: the wavefronts take every NW-th chunk of 64 of the tile's particles (its 64 cells
  // in storage order, one after the other), so that a crowded cell is shared by all of them; the
  // lanes of a chunk find their cells from the prefix counts by a forward walk shared by the
  // wavefront.
  {
    constexpr int NW = NTH / 64;
    const uint32_t tot = pre[TC];
    const CT* chx = static_cast<const CT*>(a.chi);
    const NT* nux = static_cast<const NT*>(a.nu);
    int ec = 0;  // the cell of the chunk's first particle (wave-uniform, non-decreasing)
    auto locate = [&](uint32_t c0, int& sc, int64_t& p) {
      while ((uint32_t)__builtin_amdgcn_readfirstlane(pre[ec + 1]) <= c0) ++ec;
      const uint32_t i = c0 + (uint32_t)lane;
      sc = ec;
      for (int q = ec + 1; q < TC; ++q) {
        const uint32_t pq = (uint32_t)__builtin_amdgcn_readfirstlane(pre[q]);
        if (pq >= c0 + 64u) break;
        if (pq <= i) sc = q;
      }
      // lanes past the end read the chunk's first particle
      p = i < tot ? (int64_t)start[sc] + (i - pre[sc]) : (int64_t)start[ec] + (c0 - pre[ec]);
    };
    int chn[3] = {0, 0, 0}, nun[3] = {0, 0, 0};
    auto load_at = [&](int64_t p) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        chn[d] = (int)chx[d * a.cap + p];
        nun[d] = (int)nux[d * a.cap + p];
      }
    };
    uint32_t c0 = 64u * (uint32_t)wave;
    int sn = 0;
    int64_t pn = 0;
    if (c0 < tot) {
      locate(c0, sn, pn);
      load_at(pn);
    }
    for (; c0 < tot; c0 += 64u * NW) {
      const uint32_t i = c0 + (uint32_t)lane;
      const bool active = i < tot;
      const int s = sn;
      const int64_t pc = pn;
      const int chc[3] = {chn[0], chn[1], chn[2]}, nuc[3] = {nun[0], nun[1], nun[2]};
      // the codes of the next chunk are requested before this chunk's atomics and stores are issued
      // (past the end the request repeats a particle of this chunk)
      if (c0 + 64u * NW < tot) locate(c0 + 64u * NW, sn, pn);
      load_at(pn);
      int ci, o1, o2;
      tile_xyz(s, ci, o1, o2);
      float v[3];
      int k[3], cq[3];
      physics(active, s, ci, o1, o2, chc, nuc, v, k, cq);
      const int dcode = (k[2] + 1) * 9 + (k[1] + 1) * 3 + (k[0] + 1);
      if constexpr (!SCATTER) {
        const uint32_t cbeg = pre[s], cend = pre[s + 1];
        long long q[4];
        velocity_moments(v, q);  // inactive lanes hold v = 0
        const bool stay = active && dcode == 13;
        const unsigned long long smask = __ballot(stay);
        // stayers: one prefix sum over the chunk, then the difference over each cell's lanes
        unsigned long long ps[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) ps[d] = wave_scan_u64(stay ? (unsigned long long)q[d] : 0ull);
        // The last lane of each of the chunk's cells adds the cell's stayers: their number
        // and moment sums are the differences of the inclusive scans at that lane and at the lane
        // before the cell's first one in the chunk (fetched with one lane shuffle per word).
        const int la = cbeg > c0 ? (int)(cbeg - c0) : 0;  // the cell's first lane in the chunk
        const int from = (la > 0 ? la - 1 : 0) * 4;
        const bool tail = active && (i + 1u == cend || lane == 63);
        const unsigned long long seg = (lane == 63 ? ~0ull : ((2ull << lane) - 1ull)) & ~((1ull << la) - 1ull);
        const uint32_t nst = (uint32_t)__popcll(smask & seg);
        unsigned long long sum4[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(from, (int)(uint32_t)ps[d]);
          const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(from, (int)(uint32_t)(ps[d] >> 32));
          sum4[d] = ps[d] - (la > 0 ? (((unsigned long long)hi << 32) | lo) : 0ull);
        }
        if (tail && nst > 0u) {
          atomicAdd(&grp[s * 27 + 13], nst);
#pragma unroll
          for (int d = 0; d < 4; ++d) atomicAdd(&omom[s * 4 + d], sum4[d]);
        }
        if (active && !stay) {
          atomicAdd(&grp[s * 27 + dcode], 1u);
          // new cell inside the tile: the tile's LDS accumulators; in the ring: the global ones
          const int tx = ci + k[0], ty = o1 + k[1], tz = o2 + k[2];
          if (tx >= 0 && tx < T && ty >= 0 && ty < T && tz >= 0 && tz < T) {
            const int so = tx + T * (ty + T * tz);
#pragma unroll
            for (int d = 0; d < 4; ++d) atomicAdd(&omom[so * 4 + d], (unsigned long long)q[d]);
          } else {
            // the cell index and byte offsets fit 32 bits (nc^3 < 2^28); the plane bases are uniform
            const uint32_t nx = (uint32_t)wrapi(g.cx0 + tx, a.nc), ny = (uint32_t)wrapi(g.cy0 + ty, a.nc);
            const uint32_t nz = (uint32_t)wrapi(g.cz0 + tz, a.nc), ncu = (uint32_t)a.nc;
            const uint32_t boff = (nx + ncu * (ny + ncu * nz)) * 8u;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
              char* plane = reinterpret_cast<char*>(a.mom + (int64_t)d * a.nc3);
              atomicAdd(reinterpret_cast<unsigned long long*>(plane + boff), (unsigned long long)q[d]);
            }
          }
        }
      } else {
        // Scatter: the rank inside the (new cell, source offset) slot is the number of the
        // particles before this one in storage order with the same (source cell, displacement).
        // Within the chunk it comes from the lanes with the same key: the cell's lanes are one
        // contiguous range, the displacement is matched with one ballot per bit of its code.
        // Across chunks it comes from the running count per key in LDS, which the chunks update
        // strictly in storage order: chunk c waits until c chunks have been ranked (wavefronts of
        // one workgroup are all resident, and chunk c - 1's wavefront never waits for chunk c, so
        // the wait ends; it is also bounded, and one that gives up raises an error flag).
        const int key = s * 27 + dcode;
        const uint32_t cbeg = pre[s], cend = pre[s + 1];
        const int la = cbeg > c0 ? (int)(cbeg - c0) : 0;  // the cell's lanes: [la, cend - c0)
        const uint32_t le = cend - c0;
        unsigned long long peers =
            __ballot(active) & (le >= 64u ? ~0ull : ((1ull << le) - 1ull)) & ~((1ull << la) - 1ull);
#pragma unroll
        for (int bt = 0; bt < 5; ++bt) {
          const bool bit = (dcode >> bt) & 1;
          const unsigned long long bb = __ballot(active && bit);
          peers &= bit ? bb : ~bb;
        }
        const uint32_t rin = lanes_below(peers), npeer = (uint32_t)__popcll(peers);
        // the lowest lane of the key: it alone advances the key's running count
        const int leader = peers ? __ffsll((long long)peers) - 1 : lane;
        // the ranks are formed before the turn is awaited (the compiler would otherwise move them
        // into the ordered section, which the chunks pass through one at a time)
        asm volatile("" ::"v"(rin), "v"(npeer), "v"(leader));
        // destination cell data, requested before the turn is awaited
        const int nx = wrapi(g.cx0 + ci + k[0], a.nc), ny = wrapi(g.cy0 + o1 + k[1], a.nc);
        const int nz = wrapi(g.cz0 + o2 + k[2], a.nc);
        const int64_t cn = nx + (int64_t)a.nc * (ny + (int64_t)a.nc * nz);
        uint64_t dbase = 0;
        float inv = 0.0f, vcn[3] = {0.0f, 0.0f, 0.0f};
        if (active) {
          dbase = a.off_n[cn] + a.slot[(int64_t)(26 - dcode) * a.nc3 + cn];
          inv = a.vinv[cn];
#pragma unroll
          for (int d = 0; d < 3; ++d) vcn[d] = a.vc_n[d * a.nc3 + cn];
        }
        const uint32_t chunk = c0 / 64u;
        {
          uint32_t spins = 0;
          while (__hip_atomic_load(&turn[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) != chunk &&
                 __hip_atomic_load(&turn[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0u) {
            __builtin_amdgcn_s_sleep(0);
            if (++spins >= a.turn_limit) {
              if (lane == 0) {
                __hip_atomic_store(&turn[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                set_flag(a.flags, FLAG_COUNT);
              }
              break;
            }
          }
        }
        // the ordered section: one LDS read-modify-write per key (by its lowest lane), then the turn
        // passes on; the key's other lanes take the count from that lane afterwards
        uint32_t b0 = 0u;
        if (active && rin == 0u) b0 = atomicAdd(&grp[key], npeer);
        if (lane == 0) __hip_atomic_store(&turn[0], chunk + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        b0 = (uint32_t)__shfl((int)b0, leader);
        if (active) {
          const uint64_t dst = dbase + b0 + rin;
          if (dst < (uint64_t)a.cap) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              const float u = (v[d] - vcn[d]) * inv;
              nu_n[d * a.cap + dst] = (NT)encode_nu<false>(u, edges, bucket, a.nbucket, a.vhalf);
              chi_n[d * a.cap + dst] = (CT)cq[d];
            }
            if (a.pid_bytes) store_id(a, dst, particle_id<0>(a, g, s, pc, 0u));
          } else {
            set_flag(a.flags, FLAG_COUNT);
          }
        }
      }
    }
  }
  if constexpr (!SCATTER) {
    __syncthreads();
    flush_counts<NTH>(a, g, grp);
    if (threadIdx.x < TC * 4) {
      const int so = threadIdx.x / 4, d = threadIdx.x % 4;
      const unsigned long long m = omom[threadIdx.x];
      const int64_t c = (g.cx0 + so % T) + (int64_t)a.nc * ((g.cy0 + (so / T) % T) + (int64_t)a.nc * (g.cz0 + so / (T * T)));
      if (m) atomicAdd(reinterpret_cast<unsigned long long*>(&a.mom[d * a.nc3 + c]), m);
    }
  }
}

// two 1024-thread workgroups per CU: at most 64 VGPRs
template <int NCHI, int NNU, bool SCATTER, bool MEAS = false>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_move_dense(MoveArgs a) {
  move_dense_tile<NCHI, NNU, SCATTER, MEAS>(a, xcd_block(blockIdx.x, gridDim.x));
}

template <int NCHI, int NNU, bool SCATTER>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_move_dense_boxes(BoxTable<MoveArgs> t) {
  const unsigned l = xcd_block(blockIdx.x, gridDim.x);
  const int b = box_of(t.first, t.nbox, l);
  move_dense_tile<NCHI, NNU, SCATTER, false>(t.args[b], l - t.first[b]);
}

// ---------------------------------------------------------------------------------------------
// Link: per new cell, counts from the 27 source cells in offset order (z, y, x each -1, 0, +1),
// the slot prefix per source offset, the mean velocity and the 3-D velocity variance.
// ---------------------------------------------------------------------------------------------
struct LinkArgs {
  const uint32_t* mig;
  uint32_t* slot;
  uint32_t* cnt_n;
  int64_t* mom;
  float* vc_n;
  double* dev;
  uint64_t* blk_n;
  int64_t* blk_q;
  int nc;
  int64_t nc3;
  const uint32_t* cnt_direct;  // load path: counts given directly (no migration counts)
  uint32_t* flags;
};

// the per-cell dispersion term n dev 2^20 stays below 2^54, so that the int64 sums of the 256 cells
// of a link block cannot overflow; the sum over the blocks is exact in 128 bits (k_scan_blocks)
constexpr double kDevTermLimit = 18014398509481984.0;  // 2^54

__device__ __forceinline__ void link_block(const LinkArgs& a, const unsigned blk) {
  __shared__ unsigned long long sn[LINK_BLK];
  __shared__ long long sq[LINK_BLK];
  if (workgroup_step_failed(a.flags)) return;
  const int64_t c = (int64_t)blk * LINK_BLK + threadIdx.x;
  uint32_t n = 0;
  long long q = 0;
  if (c < a.nc3) {
    if (a.cnt_direct) {
      n = a.cnt_direct[c];
    } else {
      const int x = (int)(c % a.nc), y = (int)((c / a.nc) % a.nc), z = (int)(c / ((int64_t)a.nc * a.nc));
      uint32_t run = 0;
      for (int j = 0; j < 27; ++j) {
        const int ox = j % 3 - 1, oy = (j / 3) % 3 - 1, oz = j / 9 - 1;
        const int64_t src = wrapi(x + ox, a.nc) + (int64_t)a.nc * (wrapi(y + oy, a.nc) + (int64_t)a.nc * wrapi(z + oz, a.nc));
        const uint32_t mcount = a.mig[(int64_t)(26 - j) * a.nc3 + src];
        a.slot[(int64_t)j * a.nc3 + c] = run;
        run += mcount;
      }
      n = run;
    }
    a.cnt_n[c] = n;
    const long long s1x = a.mom[c], s1y = a.mom[a.nc3 + c], s1z = a.mom[2 * a.nc3 + c], s2 = a.mom[3 * a.nc3 + c];
    a.mom[c] = 0;
    a.mom[a.nc3 + c] = 0;
    a.mom[2 * a.nc3 + c] = 0;
    a.mom[3 * a.nc3 + c] = 0;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0, dev = 0.0;
    const double nd = (double)n;
    if (n > 0) {
      const double d1 = nd * 4294967296.0;
      m0 = (double)s1x / d1;
      m1 = (double)s1y / d1;
      m2 = (double)s1z / d1;
      const double d2 = nd * 16777216.0;
      const double e2 = (double)s2 / d2;
      double mm = m0 * m0;
      mm = mm + m1 * m1;
      mm = mm + m2 * m2;
      dev = e2 - mm;
      if (!(dev > 0.0)) dev = 0.0;
    }
    a.vc_n[c] = (float)m0;
    a.vc_n[a.nc3 + c] = (float)m1;
    a.vc_n[2 * a.nc3 + c] = (float)m2;
    a.dev[c] = dev;
    const double term = (dev * nd) * 1048576.0;
    if (term < kDevTermLimit) {
      q = __double2ll_rn(term);
    } else {
      atomicOr(a.flags, FLAG_OVERFLOW);
      q = 0;
    }
  }
  sn[threadIdx.x] = n;
  sq[threadIdx.x] = q;
  __syncthreads();
  for (int s = LINK_BLK / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sn[threadIdx.x] += sn[threadIdx.x + s];
      sq[threadIdx.x] += sq[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.blk_n[blk] = sn[0];
    a.blk_q[blk] = sq[0];
  }
}

__global__ __launch_bounds__(LINK_BLK) void k_link(LinkArgs a) { link_block(a, blockIdx.x); }

__global__ __launch_bounds__(LINK_BLK) void k_link_boxes(BoxTable<LinkArgs> t) {
  const int b = box_of(t.first, t.nbox, blockIdx.x);
  link_block(t.args[b], blockIdx.x - t.first[b]);
}

// Nearest FP64 value (ties to even) of the unsigned 128-bit integer hi 2^64 + lo. Above 2^64 the
// value is shifted right into 64 bits with the shifted-out bits kept as a sticky lowest bit, which
// keeps the rounding to 53 bits exact; a 64-bit unsigned conversion is one rounding of the exact sum
// of its two halves.
__device__ __forceinline__ double u128_to_double(unsigned long long hi, unsigned long long lo) {
  if (hi == 0ull) return (double)lo;
  const int s = 64 - __clzll((long long)hi);  // 1 .. 64
  const unsigned long long keep = s == 64 ? hi : ((hi << (64 - s)) | (lo >> s));
  const unsigned long long lost = s == 64 ? lo : (lo & ((1ull << s) - 1ull));
  return ldexp((double)(keep | (lost != 0ull ? 1ull : 0ull)), s);
}

// single workgroup: exclusive scan of the per-block counts; the global dispersion, the exact sum of
// the per-block int64 terms (each in [0, 2^62)) in 128 bits
struct ScanArgs {
  const uint64_t* blk_n;
  const int64_t* blk_q;
  uint64_t* blk_off;
  int64_t nblk;
  uint64_t* off_end;
  int64_t n_expect;
  double* scal;
  uint32_t* flags;
};

__device__ __forceinline__ void scan_blocks(const ScanArgs& a) {
  __shared__ unsigned long long qh[1024], ql[1024];
  __shared__ unsigned long long wtot[16];
  if (workgroup_step_failed(a.flags)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // each wavefront takes one contiguous range of the blocks, its lanes consecutive entries (the
  // loads of a wavefront coalesce); first its total count and the lanes' 128-bit dispersion sums
  const int64_t per = (a.nblk + 15) / 16;
  const int64_t b0 = min((int64_t)wave * per, a.nblk), b1 = min(b0 + per, a.nblk);
  unsigned long long s = 0, hi = 0, lo = 0;
#pragma unroll 4
  for (int64_t b = b0 + lane; b < b1; b += 64) {
    s += a.blk_n[b];
    const unsigned long long q = (unsigned long long)a.blk_q[b];
    lo += q;
    hi += lo < q ? 1ull : 0ull;
  }
  const unsigned long long ws = wave_sum_u64(s);
  if (lane == 0) wtot[wave] = ws;
  qh[tid] = hi;
  ql[tid] = lo;
  __syncthreads();
  // then the exclusive prefix of its range, 64 entries at a time, from the totals of the
  // wavefronts before it
  unsigned long long base = 0;
  for (int w = 0; w < wave; ++w) base += wtot[w];
  for (int64_t c = b0; c < b1; c += 64) {
    const int64_t b = c + lane;
    const unsigned long long n = b < b1 ? a.blk_n[b] : 0ull;
    const unsigned long long inc = wave_scan_u64(n);
    if (b < b1) a.blk_off[b] = base + inc - n;
    base += read_lane_u64(inc, 63);
  }
  for (int o = 512; o > 0; o >>= 1) {
    if (tid < o) {
      const unsigned long long l2 = ql[tid] + ql[tid + o];
      qh[tid] += qh[tid + o] + (l2 < ql[tid] ? 1ull : 0ull);
      ql[tid] = l2;
    }
    __syncthreads();
  }
  if (tid == 0) {
    unsigned long long total = 0;
    for (int w = 0; w < 16; ++w) total += wtot[w];
    *a.off_end = total;
    if ((int64_t)total != a.n_expect) atomicOr(a.flags, FLAG_COUNT);
    double sg2 = u128_to_double(qh[0], ql[0]) / ((3.0 * (double)a.n_expect) * 1048576.0);
    if (!(sg2 > 0.0)) sg2 = 8.673617379884035e-19;  // 2^-60
    a.scal[0] = sg2;
  }
}

__global__ __launch_bounds__(1024) void k_scan_blocks(ScanArgs a) { scan_blocks(a); }

// one workgroup per box
__global__ __launch_bounds__(1024) void k_scan_blocks_boxes(const ScanArgs* __restrict__ tab) {
  scan_blocks(tab[blockIdx.x]);
}

struct FinArgs {
  const uint32_t* cnt_n;
  const uint64_t* blk_off;
  uint64_t* off_n;
  const double* dev;
  const double* scal;
  float* vs_n;
  float* vinv;
  int64_t nc3;
  int sigma_mode;
  double sq2pi;
  const uint32_t* flags;
};

__device__ __forceinline__ void finalize_block(const FinArgs& a, const unsigned blk) {
  __shared__ uint32_t pre[LINK_BLK + 1];
  __shared__ uint32_t wsum[LINK_BLK / 64];
  if (workgroup_step_failed(a.flags)) return;
  const int64_t c = (int64_t)blk * LINK_BLK + threadIdx.x;
  const uint32_t n = (c < a.nc3) ? a.cnt_n[c] : 0u;
  block_exclusive_scan(n, pre, LINK_BLK, wsum);
  if (c >= a.nc3) return;
  a.off_n[c] = a.blk_off[blk] + pre[threadIdx.x];
  const double sg2 = a.scal[0];
  double s2c = sg2;
  if (a.sigma_mode == CUBE_SIGMA_PER_CELL) {
    s2c = a.dev[c] / 3.0;
    if (n < 2 || s2c < sg2 * 9.5367431640625e-07) s2c = sg2;
  }
  const double sc = sqrt(s2c) * a.sq2pi;
  a.vs_n[c] = (float)sc;
  a.vinv[c] = (float)(1.0 / sc);
}

__global__ __launch_bounds__(LINK_BLK) void k_finalize(FinArgs a) { finalize_block(a, blockIdx.x); }

__global__ __launch_bounds__(LINK_BLK) void k_finalize_boxes(BoxTable<FinArgs> t) {
  const int b = box_of(t.first, t.nbox, blockIdx.x);
  finalize_block(t.args[b], blockIdx.x - t.first[b]);
}

// ---------------------------------------------------------------------------------------------
// Load path: host particles -> codes, stable sort by cell, moments, encode
// ---------------------------------------------------------------------------------------------
struct LoadArgs {
  const double* x;   // (n,3)
  const double* v;   // (n,3)
  int64_t n;
  int nc, nchi;
  uint32_t* key;
  uint32_t* idx;
  uint16_t* chi_tmp;  // 3 x n
  float* v_tmp;       // 3 x n
  uint32_t* cnt;
  int64_t* mom;
  int64_t nc3;
  uint32_t* flags;
};

__global__ void k_load_codes(LoadArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int nb = 1 << (8 * a.nchi);
  int cell[3];
  for (int d = 0; d < 3; ++d) {
    double xc = a.x[3 * i + d] * 0.25;
    if (!(fabs(xc) < 1e15)) {
      atomicOr(a.flags, FLAG_NONFINITE);
      xc = 0.0;
    }
    if (xc < 0.0 || xc >= (double)a.nc) xc = xc - (double)a.nc * floor(xc / (double)a.nc);
    int c = (int)floor(xc);
    if (c >= a.nc) c -= a.nc;
    if (c < 0) c = 0;
    long long b = (long long)floor((xc - (double)c) * (double)nb);
    b = b < 0 ? 0 : (b > nb - 1 ? nb - 1 : b);
    cell[d] = c;
    a.chi_tmp[d * a.n + i] = (uint16_t)b;
  }
  const uint32_t cid = (uint32_t)(cell[0] + a.nc * (cell[1] + a.nc * cell[2]));
  a.key[i] = cid;
  a.idx[i] = (uint32_t)i;
  long long s2 = 0;
  for (int d = 0; d < 3; ++d) {
    const float vf = (float)a.v[3 * i + d];
    a.v_tmp[d * a.n + i] = vf;
    if (!(vf == vf) || fabsf(vf) >= 32768.0f) atomicOr(a.flags, FLAG_OVERFLOW);
    const double vd = (double)vf;
    atomicAdd(reinterpret_cast<unsigned long long*>(&a.mom[d * a.nc3 + cid]),
              (unsigned long long)__double2ll_rn(vd * 4294967296.0));
    s2 += __double2ll_rn(vd * vd * 16777216.0);
  }
  atomicAdd(reinterpret_cast<unsigned long long*>(&a.mom[3 * a.nc3 + cid]), (unsigned long long)s2);
  atomicAdd(&a.cnt[cid], 1u);
}

template <int NCHI, int NNU>
__global__ void k_load_encode(const uint32_t* key_sorted, const uint32_t* idx_sorted, const uint16_t* chi_tmp,
                              const float* v_tmp, int64_t n, void* chi_out, void* nu_out, int64_t cap,
                              const float* vc, const float* vinv, int64_t nc3, const float* edges,
                              const int16_t* bucket, int nbucket, int vhalf, void* pid_out, int pid_bytes) {
  using CT = chi_t<NCHI>;
  using NT = nu_t<NNU>;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t src = idx_sorted[j];
  const int64_t c = key_sorted[j];
  CT* co = static_cast<CT*>(chi_out);
  NT* no = static_cast<NT*>(nu_out);
  const float inv = vinv[c];
  for (int d = 0; d < 3; ++d) {
    co[d * cap + j] = (CT)chi_tmp[d * n + src];
    const float u = (v_tmp[d * n + src] - vc[d * nc3 + c]) * inv;
    no[d * cap + j] = (NT)encode_nu<true>(u, edges, bucket, nbucket, vhalf);
  }
  // the ID of a loaded particle is its index in the input
  if (pid_bytes == 8) static_cast<uint64_t*>(pid_out)[j] = (uint64_t)src;
  else if (pid_bytes == 4) static_cast<uint32_t*>(pid_out)[j] = (uint32_t)src;
}

// IDs 0 .. n-1 in storage order
__global__ void k_pid_iota(void* pid, int pid_bytes, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  if (pid_bytes == 8) static_cast<uint64_t*>(pid)[j] = (uint64_t)j;
  else static_cast<uint32_t*>(pid)[j] = (uint32_t)j;
}

// ---------------------------------------------------------------------------------------------
// White noise: Philox4x32-10 (Salmon et al. 2011) keyed by (seed, lattice index), Box-Muller.
// ---------------------------------------------------------------------------------------------
__device__ __forceinline__ void philox_round(uint32_t* c, uint32_t k0, uint32_t k1) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

// grid: x covers one z plane of n^2 points, y = z (keeps each grid dimension below 2^32 items)
__global__ void k_noise(float* out, int n, int64_t pitch_f, uint64_t seed) {
  const int64_t ixy = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ixy >= (int64_t)n * n) return;
  const int64_t i = (int64_t)blockIdx.y * n * n + ixy;
  uint32_t c[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u, 0u};
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    philox_round(c, k0, k1);
  }
  const double u0 = ((double)c[0] + 0.5) * 2.3283064365386962890625e-10;
  const double u1 = ((double)c[1] + 0.5) * 2.3283064365386962890625e-10;
  const double w = sqrt(-2.0 * log(u0)) * cos(6.283185307179586 * u1);
  const int64_t x = i % n, y = (i / n) % n, z = i / ((int64_t)n * n);
  out[(z * n + y) * pitch_f + x] = (float)w;
}

}  // namespace

// =============================================================================================
// host launchers
// =============================================================================================
#define CUBE_XV_DISPATCH(nchi, nnu, CALL)                                     \
  do {                                                                        \
    if ((nchi) == 1 && (nnu) == 1) CALL(1, 1);                                \
    else if ((nchi) == 1 && (nnu) == 2) CALL(1, 2);                           \
    else if ((nchi) == 2 && (nnu) == 1) CALL(2, 1);                           \
    else CALL(2, 2);                                                          \
  } while (0)

// the deposit's arguments for the state of parity cur, and its grid (columns x z chunks)
static DepArgs deposit_args(const Sim& s, int cur, dim3* grid) {
  DepArgs a;
  a.chi = s.chi[cur];
  a.cnt = s.cnt[cur];
  a.off = s.off[cur];
  a.cap = s.capacity;
  a.mesh = s.mesh;
  a.pitch_f = (int64_t)s.mesh_plan.row_floats();
  a.nm = s.nm;
  a.nc = s.nc;
  a.nt = s.nc / DTX > 0 ? s.nc / DTX : 1;
  // z chunks: enough workgroups to fill the chip, each chunk at least 4 coarse layers thick
  const int cols = a.nt * a.nt;
  int nchunk = 16384 / cols;
  nchunk = nchunk < 1 ? 1 : (nchunk > s.nc / 4 ? s.nc / 4 : nchunk);
  a.zc = (s.nc + nchunk - 1) / nchunk;
  nchunk = (s.nc + a.zc - 1) / a.zc;
  a.inv_mean = (double)s.nm * (double)s.nm * (double)s.nm / ((double)s.n * ldexp(1.0, 3 * (8 * s.nchi - 1)));
  a.interleave = s.deposit_variant & 1;
  *grid = dim3((unsigned)cols, (unsigned)nchunk);
  return a;
}

void launch_deposit(Sim& s, hipStream_t st) {
  dim3 grid;
  const DepArgs a = deposit_args(s, s.cur, &grid);
  if (s.deposit_variant & 2) {
    if (s.nchi == 1) k_deposit<1, 512><<<grid, 512, 0, st>>>(a);
    else k_deposit<2, 512><<<grid, 512, 0, st>>>(a);
  } else {
    if (s.nchi == 1) k_deposit<1, 256><<<grid, 256, 0, st>>>(a);
    else k_deposit<2, 256><<<grid, 256, 0, st>>>(a);
  }
  CUBE_HIP(hipGetLastError());
}

// arguments of the link, block-scan and finalize kernels that build state nxt
static LinkArgs link_args(const Sim& s, int nxt, const uint32_t* cnt_direct) {
  LinkArgs l;
  l.mig = s.mig;
  l.slot = s.slot;
  l.cnt_n = s.cnt[nxt];
  l.mom = s.mom;
  l.vc_n = s.vc[nxt];
  l.dev = s.dev;
  l.blk_n = s.blk_n;
  l.blk_q = s.blk_q;
  l.nc = s.nc;
  l.nc3 = s.nc3;
  l.cnt_direct = cnt_direct;
  l.flags = s.flags;
  return l;
}

static ScanArgs scan_args(const Sim& s, int nxt) {
  return ScanArgs{s.blk_n, s.blk_q, s.blk_off, s.nblk, s.off[nxt] + s.nc3, s.n, s.scal, s.flags};
}

static FinArgs fin_args(const Sim& s, int nxt) {
  FinArgs f;
  f.cnt_n = s.cnt[nxt];
  f.blk_off = s.blk_off;
  f.off_n = s.off[nxt];
  f.dev = s.dev;
  f.scal = s.scal;
  f.vs_n = s.vs[nxt];
  f.vinv = s.vinv;
  f.nc3 = s.nc3;
  f.sigma_mode = s.p.sigma_mode;
  f.sq2pi = std::sqrt(2.0 / M_PI);
  f.flags = s.flags;
  return f;
}

static void link_scan_finalize(Sim& s, int nxt, const uint32_t* cnt_direct, hipStream_t st) {
  k_link<<<(unsigned)s.nblk, LINK_BLK, 0, st>>>(link_args(s, nxt, cnt_direct));
  CUBE_HIP(hipGetLastError());
  k_scan_blocks<<<1, 1024, 0, st>>>(scan_args(s, nxt));
  CUBE_HIP(hipGetLastError());
  k_finalize<<<(unsigned)s.nblk, LINK_BLK, 0, st>>>(fin_args(s, nxt));
  CUBE_HIP(hipGetLastError());
}

__global__ void k_step_end(uint32_t* flags, int* step, uint32_t code) {
  if (threadIdx.x != 0) return;
  if (step) {
    code = (uint32_t)step[0] + 2u;
    step[0] += 1;
  }
  if (flags[0] != 0u && flags[1] == 0u) flags[1] = code;
}

void launch_step_end(Sim& s, hipStream_t st, uint32_t code, bool dev_sched) {
  k_step_end<<<1, 64, 0, st>>>(s.flags, dev_sched ? s.step_dev : nullptr, code);
  CUBE_HIP(hipGetLastError());
}

// flags[0] |= f, when step is null or the device step counter equals `at`
__global__ void k_raise_flag(uint32_t* flags, const int* step, int at, uint32_t f) {
  if (threadIdx.x == 0 && (!step || step[0] == at)) flags[0] |= f;
}

void launch_raise_flag(Sim& s, hipStream_t st, uint32_t f, bool dev_sched, int at) {
  k_raise_flag<<<1, 64, 0, st>>>(s.flags, dev_sched ? s.step_dev : nullptr, at, f);
  CUBE_HIP(hipGetLastError());
}

// the move passes' arguments from the state of parity cur to the other (no step maxima, no
// initial-condition fields)
static MoveArgs move_args(const Sim& s, int cur, float kfac, float dfac, bool dev_sched) {
  const int nxt = cur ^ 1;
  MoveArgs a{};
  a.chi = s.chi[cur];
  a.nu = s.nu[cur];
  a.cnt = s.cnt[cur];
  a.off = s.off[cur];
  a.vc = s.vc[cur];
  a.vs = s.vs[cur];
  a.chi_n = s.chi[nxt];
  a.nu_n = s.nu[nxt];
  a.off_n = s.off[nxt];
  a.vc_n = s.vc[nxt];
  a.vinv = s.vinv;
  a.cap = s.capacity;
  a.mesh = s.mesh;
  a.pitch_f = (int64_t)s.mesh_plan.row_floats();
  a.nm = s.nm;
  a.nc = s.nc;
  a.nt = s.nc / T;
  a.nc3 = s.nc3;
  a.kf = kfac;
  a.df = dfac;
  a.tdec = s.tdec;
  a.tedge = s.tedge;
  a.tbucket = s.tbucket;
  a.nbucket = s.nbucket;
  a.vhalf = (s.vm - 1) / 2;
  a.mig = s.mig;
  a.slot = s.slot;
  a.mom = s.mom;
  a.flags = s.flags;
  a.kd = dev_sched ? s.sched_dev : nullptr;
  a.kstep = dev_sched ? s.step_dev : nullptr;
  a.pid = s.pid[cur];
  a.pid_n = s.pid[nxt];
  a.pid_bytes = s.pid_bytes;
  a.amax = nullptr;
  a.turn_limit = s.turn_limit;
  return a;
}

// which kernel each move pass of a step (mode 0) uses: the gradient tile or the per-corner gradient
static void move_kernels(const Sim& s, int mode, bool* tile_count, bool* tile_scatter) {
  // gradient tile per pass: variant 1 both, 2 scatter only, 3 count only, -1 when particles are at
  // least half as many as fine cells
  const bool dense = 2 * s.n >= (int64_t)s.nm * s.nm * s.nm;
  const int mv = s.move_variant;
  *tile_count = mode == 0 && (mv < 0 ? dense : (mv == 1 || mv == 3));
  *tile_scatter = mode == 0 && (mv < 0 ? dense : (mv == 1 || mv == 2));
}

void launch_move(Sim& s, int mode, float kfac, float dfac, float* const* psi, float vfac, hipStream_t st,
                 hipEvent_t* evs, bool dev_sched) {
  const int nxt = s.cur ^ 1;
  MoveArgs a = move_args(s, s.cur, kfac, dfac, dev_sched);
  // step maxima for adaptive time steps (a small fill kernel clears them: no memset node in
  // captured graphs, although adaptive simulations are never captured)
  a.amax = (mode == 0 && s.amax) ? s.amax : nullptr;
  if (a.amax) {
    k_clear_u32<<<1, 64, 0, st>>>(s.amax, 2);
    CUBE_HIP(hipGetLastError());
  }
  if (mode == 2) {
    a.psi0 = psi[0];
    a.psi1 = psi[1];
    a.psi2 = psi[2];
    a.lat_pitch_f = (int64_t)s.lat_plan.row_floats();
    a.np = s.np;
    a.q = s.np / s.nc;
    a.vfac = vfac;
    a.lunit = (float)(2.0 / (double)a.q);
  }
  const unsigned grid = (unsigned)((int64_t)a.nt * a.nt * a.nt);
  bool tile_count, tile_scatter;
  move_kernels(s, mode, &tile_count, &tile_scatter);
#define CUBE_COUNT(X, V)                                                                        \
  do {                                                                                          \
    if (tile_count && a.amax) k_move_dense<X, V, false, true><<<grid, 1024, 0, st>>>(a);         \
    else if (tile_count) k_move_dense<X, V, false><<<grid, 1024, 0, st>>>(a);                    \
    else if (mode == 0 && a.amax) k_move_count<X, V, 0, false, 512, true><<<grid, 512, 0, st>>>(a); \
    else if (mode == 0) k_move_count<X, V, 0, false, 512><<<grid, 512, 0, st>>>(a);              \
    else if (mode == 1) k_move_count<X, V, 1, false, 256><<<grid, 256, 0, st>>>(a);              \
    else k_move_count<X, V, 2, false, 256><<<grid, 256, 0, st>>>(a);                             \
  } while (0)
#define CUBE_SCATTER(X, V)                                                                      \
  do {                                                                                          \
    if (tile_scatter) k_move_dense<X, V, true><<<grid, 1024, 0, st>>>(a);                        \
    else if (mode == 0) k_move_scatter<X, V, 0, false, 512><<<grid, 512, 0, st>>>(a);            \
    else if (mode == 1) k_move_scatter<X, V, 1, false, 256><<<grid, 256, 0, st>>>(a);            \
    else k_move_scatter<X, V, 2, false, 256><<<grid, 256, 0, st>>>(a);                           \
  } while (0)
  if (evs) CUBE_HIP(hipEventRecord(evs[0], st));
  CUBE_XV_DISPATCH(s.nchi, s.nnu, CUBE_COUNT);
  CUBE_HIP(hipGetLastError());
  if (evs) CUBE_HIP(hipEventRecord(evs[1], st));
  link_scan_finalize(s, nxt, nullptr, st);
  if (evs) CUBE_HIP(hipEventRecord(evs[2], st));
  CUBE_XV_DISPATCH(s.nchi, s.nnu, CUBE_SCATTER);
  CUBE_HIP(hipGetLastError());
  if (evs) CUBE_HIP(hipEventRecord(evs[3], st));
#undef CUBE_COUNT
#undef CUBE_SCATTER
  s.cur = nxt;
}

// ---- ensemble steps: one launch per stage over every box ---------------------------------------
size_t EnsembleStep::put(const void* p, size_t bytes) {
  const size_t off = (staged.size() + 255) & ~(size_t)255;
  staged.resize(off + bytes);
  if (bytes) std::memcpy(staged.data() + off, p, bytes);
  return off;
}

void EnsembleStep::upload() {
  if (dbase || staged.empty()) return;
  CUBE_HIP(hipMalloc(&dbase, staged.size()));
  CUBE_HIP(hipMemcpy(dbase, staged.data(), staged.size(), hipMemcpyHostToDevice));
}

EnsembleStep::~EnsembleStep() {
  if (dbase) (void)hipFree(dbase);
}

namespace {

// a staged per-box argument table with the first workgroup of each box
struct StagedBoxes {
  size_t args, first;
  int nbox;
  unsigned blocks;  // workgroups of the launch
};

template <class A>
StagedBoxes stage_boxes(EnsembleStep& es, const std::vector<A>& args, const std::vector<uint32_t>& per_box,
                        int threads) {
  std::vector<uint32_t> first(1, 0u);
  uint64_t t = 0;
  for (uint32_t b : per_box) {
    t += b;
    first.push_back((uint32_t)t);
  }
  // a dispatch holds fewer than 2^32 work-items
  if (t * (uint64_t)threads >= (1ull << 32)) throw Error{CUBE_E_INVALID, "ensemble too large for one launch per stage"};
  return StagedBoxes{es.put(args), es.put(first), (int)args.size(), (unsigned)t};
}

template <class A>
BoxTable<A> table_of(const EnsembleStep* e, const StagedBoxes& g) {
  return BoxTable<A>{e->at<A>(g.args), e->at<uint32_t>(g.first), g.nbox};
}

struct EndArgs {
  uint32_t* flags;
  int* step;
};

// k_step_end of every box (device step counters), one thread per box
__global__ void k_step_end_boxes(const EndArgs* __restrict__ tab, int nbox) {
  const int b = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (b >= nbox) return;
  uint32_t* flags = tab[b].flags;
  int* step = tab[b].step;
  const uint32_t code = (uint32_t)step[0] + 2u;
  step[0] += 1;
  if (flags[0] != 0u && flags[1] == 0u) flags[1] = code;
}

}  // namespace

void ensemble_deposit(EnsembleStep& es, const std::vector<Sim*>& boxes) {
  const EnsembleStep* e = &es;
  for (int nchi = 1; nchi <= 2; ++nchi)
    for (int blk : {256, 512}) {
      std::vector<DepArgs> args;
      std::vector<uint32_t> per;
      for (Sim* s : boxes) {
        if (s->nchi != nchi || ((s->deposit_variant & 2) ? 512 : 256) != blk) continue;
        dim3 g;
        args.push_back(deposit_args(*s, s->cur, &g));
        per.push_back(g.x * g.y);
      }
      if (args.empty()) continue;
      const StagedBoxes g = stage_boxes(es, args, per, blk);
      es.launches.push_back([e, g, nchi, blk](hipStream_t st) {
        const BoxTable<DepArgs> t = table_of<DepArgs>(e, g);
        if (nchi == 1 && blk == 512) k_deposit_boxes<1, 512><<<g.blocks, 512, 0, st>>>(t);
        else if (nchi == 1) k_deposit_boxes<1, 256><<<g.blocks, 256, 0, st>>>(t);
        else if (blk == 512) k_deposit_boxes<2, 512><<<g.blocks, 512, 0, st>>>(t);
        else k_deposit_boxes<2, 256><<<g.blocks, 256, 0, st>>>(t);
        CUBE_HIP(hipGetLastError());
      });
    }
}

void ensemble_move(EnsembleStep& es, const std::vector<Sim*>& boxes) {
  const EnsembleStep* e = &es;
  // one pass over the boxes grouped by codec and kernel (gradient tile or per-corner gradient)
  auto pass = [&](bool scatter) {
    for (int xv = 0; xv < 4; ++xv)
      for (int tile = 0; tile <= 1; ++tile) {
        const int nchi = 1 + (xv >> 1), nnu = 1 + (xv & 1);
        std::vector<MoveArgs> args;
        std::vector<uint32_t> per;
        for (Sim* s : boxes) {
          bool tc, ts;
          move_kernels(*s, 0, &tc, &ts);
          if (s->nchi != nchi || s->nnu != nnu || (scatter ? ts : tc) != (tile != 0)) continue;
          args.push_back(move_args(*s, s->cur, 0.0f, 0.0f, true));
          const int64_t nt = s->nc / T;
          per.push_back((uint32_t)(nt * nt * nt));
        }
        if (args.empty()) continue;
        const StagedBoxes g = stage_boxes(es, args, per, tile ? 1024 : 512);
        es.launches.push_back([e, g, nchi, nnu, tile, scatter](hipStream_t st) {
          const BoxTable<MoveArgs> t = table_of<MoveArgs>(e, g);
#define CUBE_PASS(X, V)                                                                                 \
  do {                                                                                                  \
    if (tile && scatter) k_move_dense_boxes<X, V, true><<<g.blocks, 1024, 0, st>>>(t);                   \
    else if (tile) k_move_dense_boxes<X, V, false><<<g.blocks, 1024, 0, st>>>(t);                        \
    else if (scatter) k_move_scatter_boxes<X, V, 0, false, 512><<<g.blocks, 512, 0, st>>>(t);            \
    else k_move_count_boxes<X, V, 0, false, 512><<<g.blocks, 512, 0, st>>>(t);                           \
  } while (0)
          CUBE_XV_DISPATCH(nchi, nnu, CUBE_PASS);
#undef CUBE_PASS
          CUBE_HIP(hipGetLastError());
        });
      }
  };
  pass(false);
  // link, block scan and finalize of every box
  std::vector<LinkArgs> la;
  std::vector<ScanArgs> sa;
  std::vector<FinArgs> fa;
  std::vector<uint32_t> per;
  for (Sim* s : boxes) {
    const int nxt = s->cur ^ 1;
    la.push_back(link_args(*s, nxt, nullptr));
    sa.push_back(scan_args(*s, nxt));
    fa.push_back(fin_args(*s, nxt));
    per.push_back((uint32_t)s->nblk);
  }
  const StagedBoxes gl = stage_boxes(es, la, per, LINK_BLK);
  const StagedBoxes gf = stage_boxes(es, fa, per, LINK_BLK);
  const size_t os = es.put(sa);
  const unsigned nbox = (unsigned)boxes.size();
  es.launches.push_back([e, gl, gf, os, nbox](hipStream_t st) {
    k_link_boxes<<<gl.blocks, LINK_BLK, 0, st>>>(table_of<LinkArgs>(e, gl));
    CUBE_HIP(hipGetLastError());
    k_scan_blocks_boxes<<<nbox, 1024, 0, st>>>(e->at<ScanArgs>(os));
    CUBE_HIP(hipGetLastError());
    k_finalize_boxes<<<gf.blocks, LINK_BLK, 0, st>>>(table_of<FinArgs>(e, gf));
    CUBE_HIP(hipGetLastError());
  });
  pass(true);
}

void ensemble_step_end(EnsembleStep& es, const std::vector<Sim*>& boxes) {
  std::vector<EndArgs> t;
  for (Sim* s : boxes) t.push_back(EndArgs{s->flags, s->step_dev});
  const size_t ot = es.put(t);
  const int nbox = (int)boxes.size();
  const EnsembleStep* e = &es;
  es.launches.push_back([e, ot, nbox](hipStream_t st) {
    k_step_end_boxes<<<(unsigned)((nbox + 63) / 64), 64, 0, st>>>(e->at<EndArgs>(ot), nbox);
    CUBE_HIP(hipGetLastError());
  });
}

void launch_load(Sim& s, const double* dx, const float* /*unused*/, int64_t n, hipStream_t st) {
  // scratch for the load path
  const int nxt = s.cur ^ 1;
  uint32_t* key = static_cast<uint32_t*>(s.dmalloc(sizeof(uint32_t) * n * 4));
  uint32_t* idx = key + n;
  uint32_t* key2 = key + 2 * n;
  uint32_t* idx2 = key + 3 * n;
  uint16_t* chi_tmp = static_cast<uint16_t*>(s.dmalloc(sizeof(uint16_t) * 3 * n));
  float* v_tmp = static_cast<float*>(s.dmalloc(sizeof(float) * 3 * n));
  CUBE_HIP(hipMemsetAsync(s.cnt[nxt], 0, sizeof(uint32_t) * s.nc3, st));
  LoadArgs a;
  a.x = dx;
  a.v = dx + 3 * n;
  a.n = n;
  a.nc = s.nc;
  a.nchi = s.nchi;
  a.key = key;
  a.idx = idx;
  a.chi_tmp = chi_tmp;
  a.v_tmp = v_tmp;
  a.cnt = s.cnt[nxt];
  a.mom = s.mom;
  a.nc3 = s.nc3;
  a.flags = s.flags;
  if (n > 0) {
    k_load_codes<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(a);
    CUBE_HIP(hipGetLastError());
  }
  // stable sort of (cell id, input index) by cell id
  uint32_t *ks = key, *is = idx;
  sort_pairs_by_key(s, key, idx, key2, idx2, n, (uint32_t)(s.nc3 - 1), st, &ks, &is);
  link_scan_finalize(s, nxt, s.cnt[nxt], st);
#define CUBE_ENC(X, V)                                                                                       \
  k_load_encode<X, V><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(ks, is, chi_tmp, v_tmp, n, s.chi[nxt],    \
                                                                   s.nu[nxt], s.capacity, s.vc[nxt], s.vinv, \
                                                                   s.nc3, s.tedge, s.tbucket, s.nbucket, (s.vm - 1) / 2, \
                                                                   s.pid[nxt], s.pid_bytes)
  if (n > 0) {
    CUBE_XV_DISPATCH(s.nchi, s.nnu, CUBE_ENC);
    CUBE_HIP(hipGetLastError());
  }
#undef CUBE_ENC
  CUBE_HIP(hipStreamSynchronize(st));
  s.dfree(v_tmp);
  s.dfree(chi_tmp);
  s.dfree(key);
  s.cur = nxt;
}

void launch_pid_iota(Sim& s, hipStream_t st) {
  if (!s.pid_bytes || s.n == 0) return;
  k_pid_iota<<<(unsigned)((s.n + 255) / 256), 256, 0, st>>>(s.pid[s.cur], s.pid_bytes, s.n);
  CUBE_HIP(hipGetLastError());
}

// largest |v|^2 of the decoded state (the velocity bound of the first adaptive steps): one thread
// per particle, its cell found by bisection in the cell offsets
template <int NNU>
__global__ void k_state_speed(const void* nu, const uint64_t* off, const float* vc, const float* vs,
                              const float* tdec, int64_t n, int64_t cap, int64_t nc3, int vhalf, uint32_t* out) {
  using NT = nu_t<NNU>;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float vv = 0.0f;
  if (i < n) {
    int64_t lo = 0, hi = nc3;  // the cell c with off[c] <= i < off[c + 1]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (off[mid] <= (uint64_t)i) lo = mid;
      else hi = mid;
    }
    const NT* nv = static_cast<const NT*>(nu);
    float v[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int c = (int)nv[d * cap + i];
      c = c < -vhalf ? -vhalf : (c > vhalf ? vhalf : c);
      v[d] = __builtin_fmaf(vs[lo], tdec[c + vhalf], vc[d * nc3 + lo]);
    }
    vv = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
  }
  vv = wave_max(vv);
  if ((threadIdx.x & 63) == 0 && vv > 0.0f) atomicMax(out, __float_as_uint(vv));
}

float launch_state_speed2(Sim& s, hipStream_t st) {
  k_clear_u32<<<1, 64, 0, st>>>(s.amax, 2);
  CUBE_HIP(hipGetLastError());
  if (s.n > 0) {
    const unsigned grid = (unsigned)((s.n + 255) / 256);
    const int vh = (s.vm - 1) / 2;
    if (s.nnu == 1)
      k_state_speed<1><<<grid, 256, 0, st>>>(s.nu[s.cur], s.off[s.cur], s.vc[s.cur], s.vs[s.cur], s.tdec, s.n,
                                             s.capacity, s.nc3, vh, s.amax);
    else
      k_state_speed<2><<<grid, 256, 0, st>>>(s.nu[s.cur], s.off[s.cur], s.vc[s.cur], s.vs[s.cur], s.tdec, s.n,
                                             s.capacity, s.nc3, vh, s.amax);
    CUBE_HIP(hipGetLastError());
  }
  uint32_t bits = 0;
  CUBE_HIP(hipMemcpyAsync(&bits, s.amax, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  CUBE_HIP(hipStreamSynchronize(st));
  float f;
  std::memcpy(&f, &bits, sizeof(f));
  return f;
}

// 1-byte coarse density (Sec. 2.1): min(count, 255) per cell
__global__ void k_counts_u8(const uint32_t* cnt, int64_t nc3, uint8_t* rho1) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc3) return;
  const uint32_t v = cnt[c];
  rho1[c] = (uint8_t)(v < 255u ? v : 255u);
}

int64_t launch_counts_u8(Sim& s, uint8_t* rho1, uint32_t* over, hipStream_t st) {
  const uint32_t* cnt = s.cnt[s.cur];
  k_counts_u8<<<(unsigned)((s.nc3 + 255) / 256), 256, 0, st>>>(cnt, s.nc3, rho1);
  CUBE_HIP(hipGetLastError());
  // the true counts of the cells marked 255, in cell order (a stable selection)
  return select_at_least_255(s, cnt, s.nc3, over, st);
}

void launch_noise(const FFTPlan& pl, float* out, uint64_t seed, hipStream_t st) {
  const int64_t plane = (int64_t)pl.n * pl.n;
  const dim3 grid((unsigned)((plane + 255) / 256), (unsigned)pl.n);
  k_noise<<<grid, 256, 0, st>>>(out, pl.n, (int64_t)pl.row_floats(), seed);
  CUBE_HIP(hipGetLastError());
}

}  // namespace cube

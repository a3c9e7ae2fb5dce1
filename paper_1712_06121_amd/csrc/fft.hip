// Three-dimensional real FFT for the Poisson solve, the power spectrum and the initial
// conditions, written for gfx950 (64-wide wavefronts, 160 KB LDS per CU).
//
// The paper solves the mesh force "in Fourier space" with FFTW (Sec. 1, Sec. 2.3.3); here the
// transform is a hand-written Stockham autosort FFT held in LDS:
//   x pass : rows along x are contiguous; each workgroup loads a few rows, does a complex FFT
//            of length N/2 on the even/odd-packed row and untangles the real spectrum
//            (frequencies 0..N/2, the Nyquist value at index N/2 of the padded row).
//   y pass : a workgroup loads a block of BX adjacent x-frequency columns for all N rows
//            (BX*8-byte coalesced segments) and transforms them along y.
//   z pass : the same column kernel along z. For the Poisson solve the forward z transform,
//            the Green's function -3/2 Omega_m / |k|^2 (and the 1/N^3 normalisation) and the
//            inverse z transform are fused into one pass, so the solve costs five passes over
//            the mesh: x, y, z+G+z^-1, y^-1, x^-1.
// All passes work in place on one buffer of N x N rows of pitch_c complex values.
#include <map>
#include <tuple>

#include "cube_internal.h"

namespace cube {
namespace {

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }
// radix of the next stage for a remaining length `rem` (3 * 2^m or 2^m): the factor 3 first, then
// one radix-2 or radix-4 stage so that the rest is a power of 8
constexpr int next_radix(int rem) {
  return rem % 3 == 0 ? 3 : ((ilog2c(rem) % 3 == 1) ? 2 : ((ilog2c(rem) % 3 == 2) ? 4 : 8));
}

__device__ __forceinline__ float2 operator+(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 operator-(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// The file is compiled without floating-point contraction, and the fused multiply-adds are
// written out: every instantiation (transform size, column width, layout) then rounds the same
// operations the same way, so the variants of a pass give bit-identical results.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 conjf2(float2 a) { return make_float2(a.x, -a.y); }

// multiply by exp(DIR i pi / 2): DIR = -1 gives -i a, DIR = +1 gives i a
template <int DIR>
__device__ __forceinline__ float2 mul_pi2(float2 a) {
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// twiddle exp(DIR 2 pi i idx / n) from a table of exp(-2 pi i t / n): the whole table (QN = 0) or,
// for QN = n, its first quarter t = 0 .. n/4 - 1, the rest following by exact quarter turns
// (exp(-2 pi i (q n/4 + u) / n) = (-i)^q exp(-2 pi i u / n))
template <int DIR, int QN = 0>
__device__ __forceinline__ float2 twid(const float2* __restrict__ tw, int idx) {
  float2 w;
  if constexpr (QN == 0) {
    w = tw[idx];
  } else {
    constexpr int Q = QN / 4;
    const int q = idx / Q, u = idx - q * Q;
    const float2 b = tw[u];
    // odd q swaps the components; the signs flip as (q & 2) for x and ((q + 1) & 2) for y
    const float sx = (q & 1) ? b.y : b.x, sy = (q & 1) ? b.x : b.y;
    w = make_float2(__uint_as_float(__float_as_uint(sx) ^ ((uint32_t)(q & 2) << 30)),
                    __uint_as_float(__float_as_uint(sy) ^ ((uint32_t)((q + 1) & 2) << 30)));
  }
  if (DIR > 0) w.y = -w.y;
  return w;
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v);

template <>
__device__ __forceinline__ void dft<2, -1>(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}
template <>
__device__ __forceinline__ void dft<2, 1>(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

// length-3 DFT: y_k = sum_j v_j exp(DIR 2 pi i j k / 3)
template <int DIR>
__device__ __forceinline__ void dft3(float2* v) {
  const float h = 0.86602540378443864676f * (float)DIR;  // DIR * sqrt(3) / 2
  const float2 t1 = v[1] + v[2];
  const float2 d = v[1] - v[2];
  const float2 t2 = make_float2(__builtin_fmaf(-0.5f, t1.x, v[0].x), __builtin_fmaf(-0.5f, t1.y, v[0].y));
  v[0] = v[0] + t1;
  v[1] = make_float2(__builtin_fmaf(-h, d.y, t2.x), __builtin_fmaf(h, d.x, t2.y));
  v[2] = make_float2(__builtin_fmaf(h, d.y, t2.x), __builtin_fmaf(-h, d.x, t2.y));
}
template <>
__device__ __forceinline__ void dft<3, -1>(float2* v) { dft3<-1>(v); }
template <>
__device__ __forceinline__ void dft<3, 1>(float2* v) { dft3<1>(v); }

template <int DIR>
__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
  float2 t0 = v0 + v2, t1 = v0 - v2, t2 = v1 + v3, t3 = mul_pi2<DIR>(v1 - v3);
  v0 = t0 + t2;
  v2 = t0 - t2;
  v1 = t1 + t3;
  v3 = t1 - t3;
}
template <>
__device__ __forceinline__ void dft<4, -1>(float2* v) { dft4<-1>(v[0], v[1], v[2], v[3]); }
template <>
__device__ __forceinline__ void dft<4, 1>(float2* v) { dft4<1>(v[0], v[1], v[2], v[3]); }

template <int DIR>
__device__ __forceinline__ void dft8(float2* v) {
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  // o1 exp(DIR i pi / 4) = c u1 and o3 exp(DIR 3 i pi / 4) = c u3 (d = +-1: u1, u3 are exact), the
  // products by c fused into the butterfly's additions
  const float c = 0.70710678118654752440f;
  const float d = (float)DIR;
  const float2 u1 = make_float2(o1.x - d * o1.y, o1.y + d * o1.x);
  const float2 u3 = make_float2(-(o3.x + d * o3.y), d * o3.x - o3.y);
  const float2 w2 = mul_pi2<DIR>(o2);
  v[0] = e0 + o0;
  v[4] = e0 - o0;
  v[1] = make_float2(__builtin_fmaf(c, u1.x, e1.x), __builtin_fmaf(c, u1.y, e1.y));
  v[5] = make_float2(__builtin_fmaf(-c, u1.x, e1.x), __builtin_fmaf(-c, u1.y, e1.y));
  v[2] = e2 + w2;
  v[6] = e2 - w2;
  v[3] = make_float2(__builtin_fmaf(c, u3.x, e3.x), __builtin_fmaf(c, u3.y, e3.y));
  v[7] = make_float2(__builtin_fmaf(-c, u3.x, e3.x), __builtin_fmaf(-c, u3.y, e3.y));
}
template <>
__device__ __forceinline__ void dft<8, -1>(float2* v) { dft8<-1>(v); }
template <>
__device__ __forceinline__ void dft<8, 1>(float2* v) { dft8<1>(v); }

// One radix-R Stockham stage over NL lines of length L held in LDS. Element t of line l sits at
// lds[l * LS + t * TS]. Twiddles come from a table of exp(-2 pi i t / (L * TWS)), or with QT from
// the first quarter of it.
template <int L, int R, int NS, int NL, int LS, int TS, int BLOCK, int DIR, int TWS, bool QT = false>
__device__ __forceinline__ void stockham_stage(float2* lds, const float2* __restrict__ tw) {
  constexpr int NBF = L / R;
  constexpr int NB = NL * NBF;
  constexpr int PER = (NB + BLOCK - 1) / BLOCK;
  float2 v[PER][R];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int i = threadIdx.x + p * BLOCK;
    if (NB % BLOCK == 0 || i < NB) {
      const int l = (TS == 1) ? i / NBF : i % NL;
      const int j = (TS == 1) ? i % NBF : i / NL;
      const float2* base = lds + l * LS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[p][r] = base[(j + r * NBF) * TS];
      if (NS > 1) {
        const int k = j % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) v[p][r] = cmul(v[p][r], twid<DIR, QT ? L * TWS : 0>(tw, r * k * (L / (NS * R)) * TWS));
      }
      dft<R, DIR>(v[p]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int i = threadIdx.x + p * BLOCK;
    if (NB % BLOCK == 0 || i < NB) {
      const int l = (TS == 1) ? i / NBF : i % NL;
      const int j = (TS == 1) ? i % NBF : i / NL;
      const int k = j % NS;
      const int dst = (j / NS) * NS * R + k;
      float2* base = lds + l * LS;
#pragma unroll
      for (int r = 0; r < R; ++r) base[(dst + r * NS) * TS] = v[p][r];
    }
  }
  __syncthreads();
}

template <int L, int NS, int NL, int LS, int TS, int BLOCK, int DIR, int TWS, bool QT = false>
__device__ __forceinline__ void fft_lds(float2* lds, const float2* __restrict__ tw) {
  if constexpr (NS < L) {
    constexpr int R = next_radix(L / NS);
    stockham_stage<L, R, NS, NL, LS, TS, BLOCK, DIR, TWS, QT>(lds, tw);
    fft_lds<L, NS * R, NL, LS, TS, BLOCK, DIR, TWS, QT>(lds, tw);
  }
}

// ---- x pass: real rows <-> half spectrum ---------------------------------------------------
// rows per workgroup: the largest power of two with at most 2048 complex values in LDS that
// divides the row count
constexpr int rows_per_block(int n) {
  int nl = 1;
  while (2 * nl * (n / 2) <= 2048 && (n * n) % (2 * nl) == 0) nl *= 2;
  return nl;
}

template <int N>
struct RowCfg {
  static constexpr int H = N / 2;
  static constexpr int NL = rows_per_block(N);
  static constexpr int BLOCK = 256;
};

template <int N>
__device__ __forceinline__ void fft_x_r2c_rows(float* __restrict__ data, int64_t pitch_f, const float2* __restrict__ tw,
                                               const unsigned lb) {
  constexpr int H = RowCfg<N>::H, NL = RowCfg<N>::NL, BLOCK = RowCfg<N>::BLOCK;
  __shared__ float2 lds[NL * H];
  // the first quarter of the twiddle table in LDS: the stages then make no global read, whose
  // latency every stage would otherwise wait for
  __shared__ float2 twq[N / 4];
  for (int i = threadIdx.x; i < N / 4; i += BLOCK) twq[i] = tw[i];
  const int64_t row0 = (int64_t)lb * NL;
  constexpr int F4 = N / 4;
  constexpr int LPT = (NL * F4 + BLOCK - 1) / BLOCK;
  float4 stage[LPT];
#pragma unroll
  for (int k = 0; k < LPT; ++k) {
    const int i = threadIdx.x + k * BLOCK;
    const int l = i / F4, c = i % F4;
    if ((NL * F4) % BLOCK == 0 || i < NL * F4)
      stage[k] = *reinterpret_cast<const float4*>(data + (row0 + l) * pitch_f + 4 * c);
  }
#pragma unroll
  for (int k = 0; k < LPT; ++k) {
    const int i = threadIdx.x + k * BLOCK;
    const int l = i / F4, c = i % F4;
    if ((NL * F4) % BLOCK == 0 || i < NL * F4) {
      lds[l * H + 2 * c] = make_float2(stage[k].x, stage[k].y);
      lds[l * H + 2 * c + 1] = make_float2(stage[k].z, stage[k].w);
    }
  }
  __syncthreads();
  fft_lds<H, 1, NL, H, 1, BLOCK, -1, 2, true>(lds, twq);
  constexpr int NP = H / 2 + 1;
  for (int i = threadIdx.x; i < NL * NP; i += BLOCK) {
    const int l = i / NP, k = i % NP;
    const float2 zk = lds[l * H + k];
    const float2 zm = conjf2(lds[l * H + (k == 0 ? 0 : H - k)]);
    const float2 e = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y + zm.y));
    const float2 dd = zk - zm;
    const float2 o = make_float2(0.5f * dd.y, -0.5f * dd.x);
    const float2 wo = cmul(tw[k], o);
    float2* out = reinterpret_cast<float2*>(data + (row0 + l) * pitch_f);
    out[k] = e + wo;
    if (k != H - k) out[H - k] = conjf2(e - wo);
  }
}

template <int N>
__device__ __forceinline__ void fft_x_c2r_rows(float* __restrict__ data, int64_t pitch_f, const float2* __restrict__ tw,
                                               const unsigned lb) {
  constexpr int H = N / 2, NL = RowCfg<N>::NL, BLOCK = RowCfg<N>::BLOCK;
  constexpr int LS = H + 1;
  __shared__ float2 lds[NL * LS];
  __shared__ float2 twq[N / 4];  // the first quarter of the twiddle table
  for (int i = threadIdx.x; i < N / 4; i += BLOCK) twq[i] = tw[i];
  const int64_t row0 = (int64_t)lb * NL;
  constexpr int LPT = (NL * LS + BLOCK - 1) / BLOCK;
  float2 stage[LPT];
#pragma unroll
  for (int k = 0; k < LPT; ++k) {
    const int i = threadIdx.x + k * BLOCK;
    if (i < NL * LS) {
      const int l = i / LS, c = i % LS;
      stage[k] = reinterpret_cast<const float2*>(data + (row0 + l) * pitch_f)[c];
    }
  }
#pragma unroll
  for (int k = 0; k < LPT; ++k) {
    const int i = threadIdx.x + k * BLOCK;
    if (i < NL * LS) lds[i] = stage[k];
  }
  __syncthreads();
  constexpr int NP = H / 2 + 1;
  for (int i = threadIdx.x; i < NL * NP; i += BLOCK) {
    const int l = i / NP, k = i % NP;
    const float2 xk = lds[l * LS + k];
    const float2 xm = conjf2(lds[l * LS + H - k]);
    const float2 a = xk + xm;
    const float2 b = cmul(conjf2(tw[k]), xk - xm);
    lds[l * LS + k] = make_float2(a.x - b.y, a.y + b.x);
    if (k != 0 && k != H - k) lds[l * LS + H - k] = make_float2(a.x + b.y, -a.y + b.x);
  }
  __syncthreads();
  fft_lds<H, 1, NL, LS, 1, BLOCK, 1, 2, true>(lds, twq);
  constexpr int F4 = N / 4;
  for (int i = threadIdx.x; i < NL * F4; i += BLOCK) {
    const int l = i / F4, c = i % F4;
    const float2 a = lds[l * LS + 2 * c], b = lds[l * LS + 2 * c + 1];
    *reinterpret_cast<float4*>(data + (row0 + l) * pitch_f + 4 * c) = make_float4(a.x, a.y, b.x, b.y);
  }
}

template <int N>
__global__ __launch_bounds__(256) void k_fft_x_r2c(float* __restrict__ data, int64_t pitch_f,
                                                  const float2* __restrict__ tw) {
  fft_x_r2c_rows<N>(data, pitch_f, tw, xcd_block(blockIdx.x, gridDim.x));
}

template <int N>
__global__ __launch_bounds__(256) void k_fft_x_c2r(float* __restrict__ data, int64_t pitch_f,
                                                  const float2* __restrict__ tw) {
  fft_x_c2r_rows<N>(data, pitch_f, tw, xcd_block(blockIdx.x, gridDim.x));
}

// the x passes of several meshes of one size in one launch: per workgroups of each mesh, in order
template <int N>
__global__ __launch_bounds__(256) void k_fft_x_r2c_boxes(float* const* __restrict__ data, int64_t pitch_f,
                                                        const float2* __restrict__ tw, unsigned per) {
  const unsigned l = xcd_block(blockIdx.x, gridDim.x);
  fft_x_r2c_rows<N>(data[l / per], pitch_f, tw, l % per);
}

template <int N>
__global__ __launch_bounds__(256) void k_fft_x_c2r_boxes(float* const* __restrict__ data, int64_t pitch_f,
                                                        const float2* __restrict__ tw, unsigned per) {
  const unsigned l = xcd_block(blockIdx.x, gridDim.x);
  fft_x_c2r_rows<N>(data[l / per], pitch_f, tw, l % per);
}

// ---- y / z passes: blocks of BX columns ------------------------------------------------------
// BX: complex columns per workgroup (4 or 8 for N >= 1024, 8 or 16 below: 16 needs N <= 512 to
// fit LDS). The padding of the rows leaves room for the widest.
template <int N, int BX>
struct ColCfg {
  static constexpr int NQ = N * BX / 2;
  static constexpr int BLOCK = (N >= 2048) ? (BX >= 8 ? 1024 : 512) : (NQ % 256 == 0 ? 256 : (NQ % 128 == 0 ? 128 : 64));
};
constexpr int col_bx_default(int n) { return n >= 1024 ? 8 : 16; }
constexpr int col_bx_pitch(int n) { return n >= 1024 ? 8 : 16; }

enum ColMode { COL_FWD = 0, COL_INV = 1, COL_GREEN = 2, COL_POWER = 3, COL_PSI = 4 };

struct ColArgs {
  const float* k2;   // squared angular wavenumber per index
  float gconst;      // Green's constant (includes 1/N^3)
  double* acc;       // power accumulators (3 x (N/2 + 1))
  const float* tab;  // initial-condition factor per |n|^2
  int dim;           // initial-condition component
  int half;          // N / 2
  int order;         // workgroup order: 0 dispatch order, 1 XCD-contiguous ranges
  CoarseTerm ct;     // two-level force: the coarse-mesh term of the Poisson solve (ct.spec null: none)
};

__device__ __forceinline__ int signed_freq(int t, int n) { return t <= n / 2 ? t : t - n; }

// Where complex value c of column block cb, transform index t and other index o lives: at
// cb * cb_s + o * o_s + t * t_s + c (complex units). The mesh layout has cb_s = BX; the z-contiguous
// scratch layout [cb][y][z][BX] lets the z transforms read and write contiguous blocks.
struct ColGeom {
  int64_t cb_s, t_s, o_s;
  int cb_r;  // column blocks per layout block: block cb starts at (cb / cb_r) cb_s + (cb % cb_r) BX
};

// one column block; lb: the block's logical index in the pass over one mesh, gx x gy blocks
// (column blocks x other indices)
template <int N, int MODE, int BX>
__device__ __forceinline__ void fft_col_block(const float2* __restrict__ src, float2* __restrict__ dst,
                                              const ColGeom& gs, const ColGeom& gt, const float2* __restrict__ tw,
                                              const ColArgs& a, const unsigned lb, const unsigned gx,
                                              const unsigned gy) {
  constexpr int BLOCK = ColCfg<N, BX>::BLOCK;
  __shared__ float2 lds[N * BX];
  // the first quarter of the twiddle table and (z pass) the squared wavenumbers, in LDS: the
  // transforms then make no global read, whose latency every stage would otherwise wait for
  __shared__ float2 twq[N / 4];
  __shared__ float k2s[MODE == COL_GREEN ? N : 1];
  for (int i = threadIdx.x; i < N / 4; i += BLOCK) twq[i] = tw[i];
  if constexpr (MODE == COL_GREEN)
    for (int i = threadIdx.x; i < N; i += BLOCK) k2s[i] = a.k2[i];
  int cb, o;
  const unsigned paired = (gx - 1) * gy;
  if (a.order == 2 && lb < paired) {
    // groups of 2 x 2 (column block, other index): four consecutive blocks of one XCD cover whole
    // 128-byte lines both in the mesh (neighbouring column blocks) and in the scratch layout
    // (neighbouring other indices); the last column block (Nyquist column) comes after
    const unsigned g = lb >> 2, r = lb & 3, hc = (gx - 1) / 2;
    cb = 2 * (g % hc) + (r & 1);
    o = 2 * (g / hc) + (r >> 1);
  } else if (a.order == 2) {
    cb = gx - 1;
    o = lb - paired;
  } else {
    cb = lb % gx;
    o = lb / gx;
  }
  const int64_t base = (int64_t)o * gs.o_s + (int64_t)(cb / gs.cb_r) * gs.cb_s + (int64_t)(cb % gs.cb_r) * BX;
  const int64_t tstride = gs.t_s;
  constexpr int Q = BX / 2;
  // every load of the block in flight at once (registers), then into LDS
  constexpr int LPT = N * Q / BLOCK;
  static_assert(N * Q % BLOCK == 0, "block must divide the column block");
  float4 stage[LPT];
#pragma unroll
  for (int k = 0; k < LPT; ++k) {
    const int i = threadIdx.x + k * BLOCK;
    const int t = i / Q, c = i % Q;
    stage[k] = *reinterpret_cast<const float4*>(src + base + (int64_t)t * tstride + 2 * c);
  }
#pragma unroll
  for (int k = 0; k < LPT; ++k) {
    const int i = threadIdx.x + k * BLOCK;
    const int t = i / Q, c = i % Q;
    lds[t * BX + 2 * c] = make_float2(stage[k].x, stage[k].y);
    lds[t * BX + 2 * c + 1] = make_float2(stage[k].z, stage[k].w);
  }
  __syncthreads();
  if constexpr (MODE == COL_FWD || MODE == COL_GREEN || MODE == COL_POWER)
    fft_lds<N, 1, BX, 1, BX, BLOCK, -1, 1, true>(lds, twq);
  if constexpr (MODE == COL_GREEN) {
    // z pass: t = z frequency index, column x_c = cb*BX + b, o = y index
    const float ky2 = k2s[o];
    if (!a.ct.spec) {
      for (int i = threadIdx.x; i < N * BX; i += BLOCK) {
        const int t = i / BX, b = i % BX;
        const int xc = cb * BX + b;
        const float kk = k2s[xc] + ky2 + k2s[t];
        const float g = (xc == 0 && o == 0 && t == 0) ? 0.0f : a.gconst / kk;
        const float2 v = lds[i];
        lds[i] = make_float2(v.x * g, v.y * g);
      }
    } else {
      // two-level force: G [(1 - S) D_f + S R^3 D_c / B] on the modes with every |n_i| < N_c / 2,
      // G (1 - S) D_f elsewhere; S = exp(-k^2 r_s^2), D_c the coarse density's spectrum and 1/B the
      // restriction's inverse transfer per axis (a table over the signed coarse frequencies)
      const CoarseTerm& c = a.ct;
      const int fy = signed_freq(o, N);
      const bool ylow = fy > -c.half && fy < c.half;
      const int yc = fy < 0 ? fy + 2 * c.half : fy;
      for (int i = threadIdx.x; i < N * BX; i += BLOCK) {
        const int t = i / BX, b = i % BX;
        const int xc = cb * BX + b;
        const float kk = k2s[xc] + ky2 + k2s[t];
        const float g = (xc == 0 && o == 0 && t == 0) ? 0.0f : a.gconst / kk;
        const float s = expf(-kk * c.rs2);
        const float2 v = lds[i];
        float2 r = make_float2(v.x * (1.0f - s), v.y * (1.0f - s));
        const int fz = signed_freq(t, N);
        if (ylow && fz > -c.half && fz < c.half && xc < c.half) {
          const int zc = fz < 0 ? fz + 2 * c.half : fz;
          const float2 dc = c.spec[((int64_t)zc * (2 * c.half) + yc) * c.pitch_c + xc];
          const float2 bt = cmul(cmul(c.inv_b[fz + c.half], c.inv_b[fy + c.half]), c.inv_b[xc + c.half]);
          const float2 u = cmul(dc, bt);
          const float sc = s * c.scale;
          r = make_float2(__builtin_fmaf(sc, u.x, r.x), __builtin_fmaf(sc, u.y, r.y));
        }
        lds[i] = make_float2(r.x * g, r.y * g);
      }
    }
    __syncthreads();
  }
  if constexpr (MODE == COL_PSI) {
    const int fy = signed_freq(o, N);
    for (int i = threadIdx.x; i < N * BX; i += BLOCK) {
      const int t = i / BX, b = i % BX;
      const int xc = cb * BX + b;
      const int fz = signed_freq(t, N);
      const int n2 = xc * xc + fy * fy + fz * fz;
      const bool nyq = (xc >= a.half) || (fy == a.half) || (fz == a.half) || (fy == -a.half) || (fz == -a.half);
      const int nd = a.dim == 0 ? xc : (a.dim == 1 ? fy : fz);
      const float f = (nyq || n2 == 0) ? 0.0f : a.tab[n2] * (float)nd;
      const float2 v = lds[i];
      lds[i] = make_float2(-v.y * f, v.x * f);
    }
    __syncthreads();
  }
  if constexpr (MODE == COL_POWER) {
    // shell sums of |delta_k|^2; only real frequencies 0..N/2 along x
    constexpr int NB = N / 2 + 1;
    __shared__ double acc[3 * NB];
    for (int i = threadIdx.x; i < 3 * NB; i += BLOCK) acc[i] = 0.0;
    __syncthreads();
    const int fy = signed_freq(o, N);
    for (int i = threadIdx.x; i < N * BX; i += BLOCK) {
      const int t = i / BX, b = i % BX;
      const int xc = cb * BX + b;
      if (xc > a.half) continue;
      const int fz = signed_freq(t, N);
      const int n2 = xc * xc + fy * fy + fz * fz;
      if (n2 == 0) continue;
      int m = (int)sqrtf((float)n2);
      while ((2 * m + 1) * (2 * m + 1) <= 4 * n2) ++m;
      while (m > 0 && (2 * m - 1) * (2 * m - 1) > 4 * n2) --m;
      if (m < 1 || m > a.half) continue;
      const double w = (xc == 0 || xc == a.half) ? 1.0 : 2.0;
      const float2 v = lds[i];
      const double p = __builtin_fma((double)v.x, (double)v.x, (double)v.y * (double)v.y);
      atomicAdd(&acc[m], w * p);
      atomicAdd(&acc[NB + m], w * sqrt((double)n2));
      atomicAdd(&acc[2 * NB + m], w);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * NB; i += BLOCK) {
      const double v = acc[i];
      if (v != 0.0) atomicAdd(&a.acc[i], v);
    }
    return;
  }
  if constexpr (MODE == COL_INV || MODE == COL_GREEN || MODE == COL_PSI)
    fft_lds<N, 1, BX, 1, BX, BLOCK, 1, 1, true>(lds, twq);
  const int64_t obase = (int64_t)o * gt.o_s + (int64_t)(cb / gt.cb_r) * gt.cb_s + (int64_t)(cb % gt.cb_r) * BX;
  for (int i = threadIdx.x; i < N * Q; i += BLOCK) {
    const int t = i / Q, c = i % Q;
    const float2 u = lds[t * BX + 2 * c], w = lds[t * BX + 2 * c + 1];
    *reinterpret_cast<float4*>(dst + obase + (int64_t)t * gt.t_s + 2 * c) = make_float4(u.x, u.y, w.x, w.y);
  }
}

template <int N, int MODE, int BX>
__global__ __launch_bounds__((ColCfg<N, BX>::BLOCK)) void k_fft_col(const float2* __restrict__ src, float2* __restrict__ dst,
                                                                 ColGeom gs, ColGeom gt,
                                                                 const float2* __restrict__ tw, ColArgs a) {
  const unsigned bid = blockIdx.x + gridDim.x * blockIdx.y;
  const unsigned lb = a.order ? xcd_block(bid, gridDim.x * gridDim.y) : bid;
  fft_col_block<N, MODE, BX>(src, dst, gs, gt, tw, a, lb, gridDim.x, gridDim.y);
}

// a y or z pass over several meshes of one size in one launch: gx x gy workgroups per mesh, in
// order; each mesh has its own source, destination and Green's constant
struct ColBox {
  const float2* src;
  float2* dst;
  float gconst;
};

template <int N, int MODE, int BX>
__global__ __launch_bounds__((ColCfg<N, BX>::BLOCK)) void k_fft_col_boxes(const ColBox* __restrict__ boxes, ColGeom gs,
                                                                       ColGeom gt, const float2* __restrict__ tw,
                                                                       ColArgs a, unsigned gx, unsigned gy) {
  const unsigned per = gx * gy;
  const unsigned l = a.order ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const ColBox& m = boxes[l / per];
  ColArgs ab = a;
  ab.gconst = m.gconst;
  fft_col_block<N, MODE, BX>(m.src, m.dst, gs, gt, tw, ab, l % per, gx, gy);
}

// ---- host dispatch ---------------------------------------------------------------------------
template <int N>
void run_x(const FFTPlan& pl, float* data, bool forward, hipStream_t st) {
  const int64_t rows = (int64_t)N * N;
  const dim3 grid((unsigned)(rows / RowCfg<N>::NL));
  if (forward)
    k_fft_x_r2c<N><<<grid, RowCfg<N>::BLOCK, 0, st>>>(data, (int64_t)pl.row_floats(), pl.tw);
  else
    k_fft_x_c2r<N><<<grid, RowCfg<N>::BLOCK, 0, st>>>(data, (int64_t)pl.row_floats(), pl.tw);
  CUBE_HIP(hipGetLastError());
}

enum Layout { MESH = 0, ZSCRATCH = 1 };

// strides of the y (axis 1) or z (axis 2) transform in a layout, for column blocks of BX; the
// scratch layout [b][y][z][LB] groups LB = pl.colbx columns (LB a multiple of BX)
template <int N, int BX>
ColGeom col_geom(const FFTPlan& pl, int layout, int axis) {
  const int64_t pc = pl.pitch_c;
  if (layout == MESH) {
    if (axis == 1) return ColGeom{BX, pc, (int64_t)N * pc, 1};  // t = y, o = z
    return ColGeom{BX, (int64_t)N * pc, pc, 1};                 // t = z, o = y
  }
  const int64_t lb = pl.colbx, blk = (int64_t)N * N * lb;
  const int r = (int)(lb / BX);
  if (axis == 1) return ColGeom{blk, (int64_t)N * lb, lb, r};   // t = y, o = z
  return ColGeom{blk, lb, (int64_t)N * lb, r};                  // t = z, o = y
}

template <int N, int MODE, int BX>
void run_col_bx(const FFTPlan& pl, const float* src, int ls, float* dst, int ld, int axis, const ColArgs& a,
                hipStream_t st) {
  const int ncb = (N / 2) / BX + 1;  // the last block holds the Nyquist column and padding
  const dim3 grid(ncb, N);
  k_fft_col<N, MODE, BX><<<grid, ColCfg<N, BX>::BLOCK, 0, st>>>(
      reinterpret_cast<const float2*>(src), reinterpret_cast<float2*>(dst), col_geom<N, BX>(pl, ls, axis),
      col_geom<N, BX>(pl, ld, axis), pl.tw, a);
  CUBE_HIP(hipGetLastError());
}

// a y or z pass from layout ls to layout ld (MESH or ZSCRATCH) with column blocks of width bx
// workgroup order of a y or z pass: passes on the mesh along y and passes on the scratch layout:
// XCD-contiguous ranges (neighbouring column blocks share 128-byte lines in one L2); y passes
// between the layouts: 2 x 2 groups when the paired column blocks are even in number; z passes on
// the mesh: tunable
inline int col_order(const FFTPlan& pl, int n, int ls, int ld, int axis, int bx) {
  const int ncb = (n / 2) / bx + 1;
  if (ls != ld) return ((ncb - 1) % 2 == 0) ? 2 : 1;
  return (axis == 1 || ls == ZSCRATCH) ? 1 : pl.zorder;
}

template <int N, int MODE>
void run_col(const FFTPlan& pl, const float* src, int ls, float* dst, int ld, int axis, const ColArgs& a0,
             hipStream_t st, int bx) {
  ColArgs a = a0;
  a.order = col_order(pl, N, ls, ld, axis, bx);
  if constexpr (N < 1024) {
    if (bx == 16) {
      run_col_bx<N, MODE, 16>(pl, src, ls, dst, ld, axis, a, st);
      return;
    }
  } else {
    if (bx == 4) {
      run_col_bx<N, MODE, 4>(pl, src, ls, dst, ld, axis, a, st);
      return;
    }
  }
  run_col_bx<N, MODE, 8>(pl, src, ls, dst, ld, axis, a, st);
}

template <int N, int MODE>
void run_col(const FFTPlan& pl, const float* src, float* dst, int axis, const ColArgs& a, hipStream_t st) {
  run_col<N, MODE>(pl, src, MESH, dst, MESH, axis, a, st, pl.colbx);
}

template <int N>
void solve_n(const FFTPlan& pl, float* d, float gconst, hipStream_t st, hipEvent_t* ev, const CoarseTerm* ct) {
  ColArgs a{pl.k2, gconst, nullptr, nullptr, 0, N / 2, 0, ct ? *ct : CoarseTerm{}};
  if (ev) CUBE_HIP(hipEventRecord(ev[0], st));
  run_x<N>(pl, d, true, st);
  if (ev) CUBE_HIP(hipEventRecord(ev[1], st));
  if (pl.zlayout && pl.zscratch) {
    // y pass into the z-contiguous scratch, z pass + Green's function there, y pass back
    float* zs = reinterpret_cast<float*>(pl.zscratch);
    run_col<N, COL_FWD>(pl, d, MESH, zs, ZSCRATCH, 1, a, st, pl.colbx);
    if (ev) CUBE_HIP(hipEventRecord(ev[2], st));
    run_col<N, COL_GREEN>(pl, zs, ZSCRATCH, zs, ZSCRATCH, 2, a, st, pl.zbx);
    if (ev) CUBE_HIP(hipEventRecord(ev[3], st));
    run_col<N, COL_INV>(pl, zs, ZSCRATCH, d, MESH, 1, a, st, pl.colbx);
  } else {
    run_col<N, COL_FWD>(pl, d, d, 1, a, st);
    if (ev) CUBE_HIP(hipEventRecord(ev[2], st));
    run_col<N, COL_GREEN>(pl, d, d, 2, a, st);
    if (ev) CUBE_HIP(hipEventRecord(ev[3], st));
    run_col<N, COL_INV>(pl, d, d, 1, a, st);
  }
  if (ev) CUBE_HIP(hipEventRecord(ev[4], st));
  run_x<N>(pl, d, false, st);
  if (ev) CUBE_HIP(hipEventRecord(ev[5], st));
}

template <int N>
void forward_n(const FFTPlan& pl, float* d, hipStream_t st) {
  ColArgs a{pl.k2, 0.f, nullptr, nullptr, 0, N / 2, 0};
  run_x<N>(pl, d, true, st);
  run_col<N, COL_FWD>(pl, d, d, 1, a, st);
  run_col<N, COL_FWD>(pl, d, d, 2, a, st);
}

template <int N>
void power_n(const FFTPlan& pl, float* d, double* acc, hipStream_t st) {
  ColArgs a{pl.k2, 0.f, acc, nullptr, 0, N / 2, 0};
  run_x<N>(pl, d, true, st);
  run_col<N, COL_FWD>(pl, d, d, 1, a, st);
  run_col<N, COL_POWER>(pl, d, d, 2, a, st);
}

template <int N>
void ic_n(const FFTPlan& pl, const float* wk, float* out, const float* tab, int dim, hipStream_t st) {
  ColArgs a{pl.k2, 0.f, nullptr, tab, dim, N / 2, 0};
  run_col<N, COL_PSI>(pl, wk, out, 2, a, st);
  run_col<N, COL_INV>(pl, out, out, 1, a, st);
  run_x<N>(pl, out, false, st);
}

// ---- ensemble solves: each pass one launch over several meshes of one size --------------------
template <int N>
void run_x_boxes(const FFTPlan& pl, float* const* data, unsigned nbox, bool forward, hipStream_t st) {
  const unsigned per = (unsigned)((int64_t)N * N / RowCfg<N>::NL);
  if (forward)
    k_fft_x_r2c_boxes<N><<<nbox * per, RowCfg<N>::BLOCK, 0, st>>>(data, (int64_t)pl.row_floats(), pl.tw, per);
  else
    k_fft_x_c2r_boxes<N><<<nbox * per, RowCfg<N>::BLOCK, 0, st>>>(data, (int64_t)pl.row_floats(), pl.tw, per);
  CUBE_HIP(hipGetLastError());
}

template <int N, int MODE, int BX>
void run_col_boxes_bx(const FFTPlan& pl, const ColBox* boxes, unsigned nbox, int ls, int ld, int axis,
                      const ColArgs& a, hipStream_t st) {
  const unsigned ncb = (N / 2) / BX + 1;
  k_fft_col_boxes<N, MODE, BX><<<nbox * ncb * N, ColCfg<N, BX>::BLOCK, 0, st>>>(
      boxes, col_geom<N, BX>(pl, ls, axis), col_geom<N, BX>(pl, ld, axis), pl.tw, a, ncb, (unsigned)N);
  CUBE_HIP(hipGetLastError());
}

template <int N, int MODE>
void run_col_boxes(const FFTPlan& pl, const ColBox* boxes, unsigned nbox, int ls, int ld, int axis,
                   const ColArgs& a0, hipStream_t st, int bx) {
  ColArgs a = a0;
  a.order = col_order(pl, N, ls, ld, axis, bx);
  if constexpr (N < 1024) {
    if (bx == 16) {
      run_col_boxes_bx<N, MODE, 16>(pl, boxes, nbox, ls, ld, axis, a, st);
      return;
    }
  } else {
    if (bx == 4) {
      run_col_boxes_bx<N, MODE, 4>(pl, boxes, nbox, ls, ld, axis, a, st);
      return;
    }
  }
  run_col_boxes_bx<N, MODE, 8>(pl, boxes, nbox, ls, ld, axis, a, st);
}

// the Poisson solves of boxes whose meshes have size N and the same FFT variants: the five passes
// of solve_n, each over all of them; per box its mesh, scratch copy and Green's constant
template <int N>
void solve_boxes_n(EnsembleStep& es, const std::vector<Sim*>& g) {
  const FFTPlan pl = g[0]->mesh_plan;  // row pitch, variants and the (size-only) twiddle and k^2 tables
  const bool zs = pl.zlayout && pl.zscratch;
  std::vector<float*> data;
  std::vector<ColBox> yf, zp, yi;
  for (Sim* s : g) {
    float2* m = reinterpret_cast<float2*>(s->mesh);
    float2* z = zs ? s->mesh_plan.zscratch : m;
    const float gc = gconst(*s);
    data.push_back(s->mesh);
    yf.push_back(ColBox{m, z, gc});
    zp.push_back(ColBox{z, z, gc});
    yi.push_back(ColBox{z, m, gc});
  }
  const size_t od = es.put(data), oyf = es.put(yf), ozp = es.put(zp), oyi = es.put(yi);
  const unsigned nb = (unsigned)g.size();
  const EnsembleStep* e = &es;
  es.launches.push_back([=](hipStream_t st) {
    const ColArgs a{pl.k2, 0.f, nullptr, nullptr, 0, N / 2, 0, CoarseTerm{}};
    float* const* d = e->at<float*>(od);
    const int lz = zs ? ZSCRATCH : MESH;
    run_x_boxes<N>(pl, d, nb, true, st);
    run_col_boxes<N, COL_FWD>(pl, e->at<ColBox>(oyf), nb, MESH, lz, 1, a, st, pl.colbx);
    run_col_boxes<N, COL_GREEN>(pl, e->at<ColBox>(ozp), nb, lz, lz, 2, a, st, zs ? pl.zbx : pl.colbx);
    run_col_boxes<N, COL_INV>(pl, e->at<ColBox>(oyi), nb, lz, MESH, 1, a, st, pl.colbx);
    run_x_boxes<N>(pl, d, nb, false, st);
  });
}

#define CUBE_FFT_DISPATCH(n, CALL)                        \
  switch (n) {                                            \
    case 16: CALL(16); break;                             \
    case 32: CALL(32); break;                             \
    case 48: CALL(48); break;                             \
    case 64: CALL(64); break;                             \
    case 96: CALL(96); break;                             \
    case 128: CALL(128); break;                           \
    case 192: CALL(192); break;                           \
    case 256: CALL(256); break;                           \
    case 384: CALL(384); break;                           \
    case 512: CALL(512); break;                           \
    case 1024: CALL(1024); break;                         \
    case 2048: CALL(2048); break;                         \
    default: throw Error{CUBE_E_INVALID, "unsupported FFT size"}; \
  }


}  // namespace

// Cross power of two density meshes over one box (Sec. 3, Eqs. (cps) and (ccc)): per shell m of the
// smaller mesh (size n), the sums over its modes of w Re(conj(a_k) b_k), w |a_k|^2, w |b_k|^2, w |k|
// and w (w = 1 on the x = 0 and x = n/2 planes, 2 elsewhere: the conjugate half). Each mode is read
// from both half spectra at its own indices. Meshes of one size contribute every mode; of two
// sizes, the modes with every |f_i| < n/2 (the smaller mesh's Nyquist planes are aliased there).
struct CrossArgs {
  const float2* a;
  const float2* b;
  int64_t pa, pb;  // complex values per row
  int na, nb, n;   // mesh sizes, the smaller one
  int all;         // 1: one size, every mode
  double* acc;     // 5 x (n/2 + 1): P_ab, P_aa, P_bb, |n|, weight
};

// one workgroup per z index of the smaller mesh
__global__ __launch_bounds__(1024) void k_cross_shells(CrossArgs c) {
  extern __shared__ double sacc[];
  const int half = c.n / 2, nsh = half + 1;
  for (int i = threadIdx.x; i < 5 * nsh; i += blockDim.x) sacc[i] = 0.0;
  __syncthreads();
  const int iz = blockIdx.x;
  const int fz = signed_freq(iz, c.n);
  const bool zok = c.all || (fz != half);
  const int nx = c.all ? half + 1 : half;
  const int64_t rows = zok ? (int64_t)c.n * nx : 0;
  const int za = fz < 0 ? fz + c.na : fz, zb = fz < 0 ? fz + c.nb : fz;
  for (int64_t i = threadIdx.x; i < rows; i += blockDim.x) {
    const int iy = (int)(i / nx), fx = (int)(i % nx);
    const int fy = signed_freq(iy, c.n);
    if (!c.all && fy == half) continue;
    const int n2 = fx * fx + fy * fy + fz * fz;
    if (n2 == 0) continue;
    int m = (int)sqrtf((float)n2);
    while ((2 * m + 1) * (2 * m + 1) <= 4 * n2) ++m;
    while (m > 0 && (2 * m - 1) * (2 * m - 1) > 4 * n2) --m;
    if (m < 1 || m > half) continue;
    const int ya = fy < 0 ? fy + c.na : fy, yb = fy < 0 ? fy + c.nb : fy;
    const float2 u = c.a[((int64_t)za * c.na + ya) * c.pa + fx];
    const float2 v = c.b[((int64_t)zb * c.nb + yb) * c.pb + fx];
    const double w = (fx == 0 || fx == half) ? 1.0 : 2.0;
    atomicAdd(&sacc[m], w * __builtin_fma((double)u.x, (double)v.x, (double)u.y * v.y));
    atomicAdd(&sacc[nsh + m], w * __builtin_fma((double)u.x, (double)u.x, (double)u.y * u.y));
    atomicAdd(&sacc[2 * nsh + m], w * __builtin_fma((double)v.x, (double)v.x, (double)v.y * v.y));
    atomicAdd(&sacc[3 * nsh + m], w * sqrt((double)n2));
    atomicAdd(&sacc[4 * nsh + m], w);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 5 * nsh; i += blockDim.x) {
    const double x = sacc[i];
    if (x != 0.0) atomicAdd(&c.acc[i], x);
  }
}

void cross_shells(const FFTPlan& pa, const float* a, const FFTPlan& pb, const float* b, double* acc,
                  hipStream_t st) {
  CrossArgs c;
  c.a = reinterpret_cast<const float2*>(a);
  c.b = reinterpret_cast<const float2*>(b);
  c.pa = pa.pitch_c;
  c.pb = pb.pitch_c;
  c.na = pa.n;
  c.nb = pb.n;
  c.n = std::min(pa.n, pb.n);
  c.all = pa.n == pb.n;
  c.acc = acc;
  const size_t lds = sizeof(double) * 5 * (c.n / 2 + 1);
  k_cross_shells<<<c.n, 1024, lds, st>>>(c);
  CUBE_HIP(hipGetLastError());
}

// Refined initial conditions: the modes a coarser lattice holds without aliasing (every
// |n_i| < np/2 of the source, size np) overwrite the same modes of the finer lattice's transformed
// noise, times (N/np)^{3/2} so that both hold one Gaussian field. One thread per source mode.
__global__ void k_splice_modes(const float2* __restrict__ src, int64_t ps, int ns, float2* __restrict__ dst,
                               int64_t pd, int nd, float scale) {
  const int half = ns / 2;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)ns * ns * half;
  if (i >= total) return;
  const int fx = (int)(i % half);
  const int iy = (int)((i / half) % ns), iz = (int)(i / ((int64_t)half * ns));
  const int fy = signed_freq(iy, ns), fz = signed_freq(iz, ns);
  if (fy == half || fz == half) return;  // the source's Nyquist planes are aliased
  const int yd = fy < 0 ? fy + nd : fy, zd = fz < 0 ? fz + nd : fz;
  const float2 v = src[((int64_t)iz * ns + iy) * ps + fx];
  dst[((int64_t)zd * nd + yd) * pd + fx] = make_float2(v.x * scale, v.y * scale);
}

void splice_modes(const FFTPlan& ps, const float* src, const FFTPlan& pd, float* dst, float scale, hipStream_t st) {
  const int64_t total = (int64_t)ps.n * ps.n * (ps.n / 2);
  k_splice_modes<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(reinterpret_cast<const float2*>(src), ps.pitch_c,
                                                                   ps.n, reinterpret_cast<float2*>(dst), pd.pitch_c,
                                                                   pd.n, scale);
  CUBE_HIP(hipGetLastError());
}

bool fft_coarse_size_supported(int n) { return n == 16 || fft_size_supported(n); }

// ---- restriction to the coarse mesh (two-level force) ------------------------------------------
// Tent weights (1, 3, 5, 7, 7, 5, 3, 1) / 32 over the fine offsets -2 .. 5 from a coarse cell's first
// fine cell along each axis (the fine cells whose centres lie within 4 fine cells of the coarse
// cell's centre, weight 1 - d / 4), summed in that order along x, then y, then z. A workgroup owns
// 8 x 8 coarse columns and a chunk of coarse layers and walks the fine planes along z: each plane
// is restricted along x and y into 64 values kept in a ring of 8 planes, and every fourth plane
// completes a coarse layer. The next plane's values are requested before the current one is used.
namespace {
constexpr int RT = 8;           // coarse cells per column side
constexpr int RF = 4 * RT + 4;  // fine cells per side of a loaded plane (offsets -2 .. 4 RT + 1)
constexpr int RBLK = 256;
constexpr int RLD = (RF * RF + RBLK - 1) / RBLK;

__device__ __forceinline__ int wrapn(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__global__ __launch_bounds__(RBLK) void k_restrict(const float* __restrict__ mesh, int64_t pitch_f, int nm, int nc,
                                                   int zc, float* __restrict__ out, int64_t opitch_f) {
  __shared__ float plane[RF * RF];
  __shared__ float xr[RF * RT];
  __shared__ float ring[8 * RT * RT];
  constexpr float w[8] = {0.03125f, 0.09375f, 0.15625f, 0.21875f, 0.21875f, 0.15625f, 0.09375f, 0.03125f};
  const int ncol = nc / RT;
  const unsigned lb = xcd_block(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int bxy = (int)(lb % gridDim.x), bz = (int)(lb / gridDim.x);
  const int cx0 = (bxy % ncol) * RT, cy0 = (bxy / ncol) * RT;
  const int cz0 = bz * zc, cz1 = min(cz0 + zc, nc);
  const int fx0 = 4 * cx0 - 2, fy0 = 4 * cy0 - 2;
  int col[RLD];
  int64_t row[RLD];
#pragma unroll
  for (int k = 0; k < RLD; ++k) {
    const int i = threadIdx.x + k * RBLK;
    const int y = i / RF, x = i - (i / RF) * RF;
    col[k] = wrapn(fx0 + x, nm);
    row[k] = (int64_t)wrapn(fy0 + (i < RF * RF ? y : 0), nm) * pitch_f;
  }
  auto fetch = [&](int fz, float* v) {
    const float* pl = mesh + (int64_t)wrapn(fz, nm) * nm * pitch_f;
#pragma unroll
    for (int k = 0; k < RLD; ++k)
      if (threadIdx.x + k * RBLK < RF * RF) v[k] = pl[row[k] + col[k]];
  };
  float cur[RLD], nxt[RLD];
  const int fz_end = 4 * cz1 + 1;
  fetch(4 * cz0 - 2, cur);
  for (int fz = 4 * cz0 - 2; fz <= fz_end; ++fz) {
    fetch(fz < fz_end ? fz + 1 : fz, nxt);
#pragma unroll
    for (int k = 0; k < RLD; ++k)
      if (threadIdx.x + k * RBLK < RF * RF) plane[threadIdx.x + k * RBLK] = cur[k];
    __syncthreads();
    for (int i = threadIdx.x; i < RF * RT; i += RBLK) {
      const int y = i / RT, c = i - (i / RT) * RT;
      float acc = 0.0f;
#pragma unroll
      for (int b = 0; b < 8; ++b) acc = __builtin_fmaf(w[b], plane[y * RF + 4 * c + b], acc);
      xr[i] = acc;
    }
    __syncthreads();
    if (threadIdx.x < RT * RT) {
      const int cy = threadIdx.x / RT, cx = threadIdx.x % RT;
      float acc = 0.0f;
#pragma unroll
      for (int b = 0; b < 8; ++b) acc = __builtin_fmaf(w[b], xr[(4 * cy + b) * RT + cx], acc);
      ring[(fz & 7) * RT * RT + threadIdx.x] = acc;
    }
    __syncthreads();
    // coarse layer c is complete once plane 4 c + 5 is in the ring (planes 4 c - 2 .. 4 c + 5)
    if (((fz - 5) & 3) == 0 && fz >= 4 * cz0 + 5 && threadIdx.x < RT * RT) {
      const int c = (fz - 5) / 4;
      float acc = 0.0f;
#pragma unroll
      for (int b = 0; b < 8; ++b) acc = __builtin_fmaf(w[b], ring[((4 * c - 2 + b) & 7) * RT * RT + threadIdx.x], acc);
      out[((int64_t)c * nc + cy0 + threadIdx.x / RT) * opitch_f + cx0 + threadIdx.x % RT] = acc;
    }
#pragma unroll
    for (int k = 0; k < RLD; ++k) cur[k] = nxt[k];
  }
}
}  // namespace

void launch_restrict(const FFTPlan& fp, const float* mesh, const FFTPlan& cp, float* out, hipStream_t st) {
  const int nc = cp.n, nm = fp.n;
  const int cols = (nc / RT) * (nc / RT);
  int nchunk = 16384 / cols;
  nchunk = nchunk < 1 ? 1 : (nchunk > nc ? nc : nchunk);
  const int zc = (nc + nchunk - 1) / nchunk;
  nchunk = (nc + zc - 1) / zc;
  const dim3 grid((unsigned)cols, (unsigned)nchunk);
  k_restrict<<<grid, RBLK, 0, st>>>(mesh, (int64_t)fp.row_floats(), nm, nc, zc, out, (int64_t)cp.row_floats());
  CUBE_HIP(hipGetLastError());
}

bool fft_size_supported(int n) {
  switch (n) {
    case 32: case 48: case 64: case 96: case 128: case 192: case 256: case 384: case 512: case 1024: case 2048:
      return true;
    default:
      return false;
  }
}

void fft_plan_create(Sim& s, FFTPlan& pl, int n) {
  pl.n = n;
  pl.bx = col_bx_pitch(n);
  pl.colbx = col_bx_default(n);
  pl.zbx = pl.colbx;
  pl.zorder = 0;
  pl.pitch_c = n / 2 + pl.bx;
  std::vector<float2> tw(n);
  std::vector<float> k2(n);
  const double two_pi = 6.283185307179586476925286766559;
  // the first quarter from the cosine and sine, the rest by exact quarter turns of it, as the
  // transforms, which keep only the first quarter in LDS, form them
  const int q = n / 4;
  for (int t = 0; t < q; ++t) {
    const double ang = -two_pi * (double)t / (double)n;
    tw[t] = make_float2((float)cos(ang), (float)sin(ang));
  }
  for (int t = q; t < n; ++t) {
    const float2 b = tw[t % q];
    const int r = t / q;
    tw[t] = r == 1 ? make_float2(b.y, -b.x) : (r == 2 ? make_float2(-b.x, -b.y) : make_float2(-b.y, b.x));
  }
  for (int t = 0; t < n; ++t) {
    const int f = t <= n / 2 ? t : t - n;
    const double k = two_pi * (double)f / (double)n;
    k2[t] = (float)(k * k);
  }
  pl.tw = static_cast<float2*>(s.dmalloc(sizeof(float2) * n));
  pl.k2 = static_cast<float*>(s.dmalloc(sizeof(float) * n));
  CUBE_HIP(hipMemcpy(pl.tw, tw.data(), sizeof(float2) * n, hipMemcpyHostToDevice));
  CUBE_HIP(hipMemcpy(pl.k2, k2.data(), sizeof(float) * n, hipMemcpyHostToDevice));
}

std::vector<int> fft_col_widths(int n) {
  if (n >= 1024) return {4, 8};
  return {8, 16};
}

void fft_plan_destroy(Sim& s, FFTPlan& pl) {
  s.dfree(pl.tw);
  s.dfree(pl.k2);
  pl.tw = nullptr;
  pl.k2 = nullptr;
}

void fft_solve_poisson(const FFTPlan& pl, float* data, float gconst, hipStream_t st, hipEvent_t* evs,
                       const CoarseTerm* ct) {
#define CUBE_CALL(N) solve_n<N>(pl, data, gconst, st, evs, ct)
  CUBE_FFT_DISPATCH(pl.n, CUBE_CALL)
#undef CUBE_CALL
}

void ensemble_solve(EnsembleStep& es, const std::vector<Sim*>& boxes) {
  // boxes grouped by mesh size, scratch layout, column widths and z-pass order
  std::map<std::tuple<int, int, int, int, int>, std::vector<Sim*>> groups;
  for (Sim* s : boxes) {
    if (s->two_level_rs > 0.0)
      throw Error{CUBE_E_INVALID, "ensemble launches need single-level solves (two-level force switched on)"};
    const FFTPlan& pl = s->mesh_plan;
    groups[std::make_tuple(pl.n, (pl.zlayout && pl.zscratch) ? 1 : 0, pl.colbx, pl.zbx, pl.zorder)].push_back(s);
  }
  for (const auto& kv : groups) {
#define CUBE_CALL(N) solve_boxes_n<N>(es, kv.second)
    CUBE_FFT_DISPATCH(std::get<0>(kv.first), CUBE_CALL)
#undef CUBE_CALL
  }
}

void fft_forward_3d(const FFTPlan& pl, float* data, hipStream_t st) {
#define CUBE_CALL(N) forward_n<N>(pl, data, st)
  CUBE_FFT_DISPATCH(pl.n, CUBE_CALL)
#undef CUBE_CALL
}

void fft_power(const FFTPlan& pl, float* data, double* acc, hipStream_t st) {
#define CUBE_CALL(N) power_n<N>(pl, data, acc, st)
  CUBE_FFT_DISPATCH(pl.n, CUBE_CALL)
#undef CUBE_CALL
}

void fft_ic_component(const FFTPlan& pl, const float* wk, float* out, const float* tab, int dim, hipStream_t st) {
#define CUBE_CALL(N) ic_n<N>(pl, wk, out, tab, dim, st)
  CUBE_FFT_DISPATCH(pl.n, CUBE_CALL)
#undef CUBE_CALL
}

}  // namespace cube

// Small kernels: fills, the Philox test-matrix generator, the BF16 cast and
// input scan, and the relative reconstruction error.
#include "rnmf_common.h"
#include <type_traits>

namespace rnmf {

// ---------------------------------------------------------------------------
// Fill (used instead of hipMemsetAsync so that captured graphs replay safely)
// ---------------------------------------------------------------------------
__global__ void fill_u32_kernel(unsigned* p, size_t count, unsigned v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = v;
}

hipError_t launch_fill_u32(unsigned* p, size_t count, unsigned v, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC 2011): counter = (index lo, index hi, stream id, tag),
// key = seed.  Uniform [0,1) from 53 bits; normal by Box-Muller (one normal
// per counter, the cosine branch).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(unsigned c[4], unsigned k0, unsigned k1) {
  const unsigned M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const unsigned W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    unsigned hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    unsigned hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    unsigned n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

constexpr unsigned PHILOX_TAG = 0x524E4D46u;

__device__ __forceinline__ double u53(unsigned lo, unsigned hi) {
  u64 v = ((u64)hi << 21) ^ (u64)(lo >> 11);
  return (double)v * (1.0 / 9007199254740992.0);
}

template <typename T>
__global__ void philox_kernel(T* out, int64_t count, unsigned k0, unsigned k1, unsigned sid, int dist) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) {
    unsigned c[4] = {(unsigned)(uint64_t)i, (unsigned)((uint64_t)i >> 32), sid, PHILOX_TAG};
    philox4x32_10(c, k0, k1);
    double v;
    if (dist == 0 || dist == 2) {
      double u1 = u53(c[0], c[1]) + (1.0 / 9007199254740992.0);  // (0, 1]
      double u2 = u53(c[2], c[3]);
      v = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
      if (dist == 2) v = v > 0.0 ? v : 0.0;  // Gaussian with the negative entries set to zero
    } else {
      v = u53(c[0], c[1]);
    }
    out[i] = (T)v;
  }
}

// The bare block function on caller-given counters and keys (4 and 2 words
// each per element), for reproducing the generator's stream off the device.
__global__ void philox_raw_kernel(const unsigned* __restrict__ ctr, const unsigned* __restrict__ key,
                                  unsigned* __restrict__ out, int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) {
    unsigned c[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
    philox4x32_10(c, key[2 * i], key[2 * i + 1]);
#pragma unroll
    for (int e = 0; e < 4; ++e) out[4 * i + e] = c[e];
  }
}

hipError_t launch_philox_raw(const unsigned* ctr, const unsigned* key, unsigned* out, int64_t count,
                             hipStream_t s) {
  if (count == 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(philox_raw_kernel, dim3((unsigned)blocks), dim3(256), 0, s, ctr, key, out, count);
  return hipGetLastError();
}

hipError_t launch_philox(void* out, int dt, int64_t rows, int64_t cols, uint64_t seed,
                         unsigned sid, int dist, hipStream_t s) {
  int64_t count = rows * cols;
  if (count == 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  unsigned k0 = (unsigned)seed, k1 = (unsigned)(seed >> 32);
  if (dt == 0)
    hipLaunchKernelGGL(philox_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (double*)out, count, k0, k1, sid, dist);
  else
    hipLaunchKernelGGL(philox_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (float*)out, count, k0, k1, sid, dist);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP32 -> BF16 cast (round to nearest even), with the NaN/Inf/negative scan.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bf16_t f32_to_bf16_rne(float f) {
  unsigned b = __float_as_uint(f);
  if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return (bf16_t)((b >> 16) | 0x40u);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (bf16_t)(b >> 16);
}

__device__ __forceinline__ unsigned scan_bits(float v) {
  unsigned f = 0;
  if (!(v == v) || fabsf(v) == INFINITY) f |= ST_NONFINITE;
  else if (v < 0.0f) f |= ST_NEGATIVE;
  return f;
}
__device__ __forceinline__ unsigned scan_bits(double v) {
  unsigned f = 0;
  if (!(v == v) || fabs(v) == INFINITY) f |= ST_NONFINITE;
  else if (v < 0.0) f |= ST_NEGATIVE;
  return f;
}

__device__ __forceinline__ void or_status(unsigned* status, unsigned f) {
  // reduce over the wavefront first so that at most one atomic per wave is issued
  unsigned long long any = __ballot(f != 0);
  if (any) {
    unsigned acc = f;
    for (int o = 32; o > 0; o >>= 1) acc |= __shfl_xor(acc, o);
    if ((threadIdx.x & 63) == 0) atomicOr(status, acc);
  }
}

// A workgroup takes whole rows (no index division per element).  Rows whose
// source and destination are 16-byte aligned move 8 elements per thread and
// step (two 16-byte loads, one 16-byte store, two steps in flight); the rest
// of a row, and unaligned rows, element by element.  Pad columns [n, ldb) are
// zeroed.
__global__ __launch_bounds__(256) void cast_bf16_kernel(const float* __restrict__ X, int64_t m, int64_t n,
                                                        int64_t ldx, bf16_t* __restrict__ Xb, int64_t ldb,
                                                        unsigned* status, int check, int vec) {
  typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  unsigned flag = 0;
  const int64_t n8 = vec ? n / 8 : 0;
  const int t = threadIdx.x;
  for (int64_t r = blockIdx.x; r < m; r += gridDim.x) {
    const float* src = X + r * ldx;
    bf16_t* dst = Xb + r * ldb;
    auto conv8 = [&](const f32x4 a, const f32x4 b) -> u32x4 {
      float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
      unsigned h[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if (check) flag |= scan_bits(v[e]);
        h[e] = f32_to_bf16_rne(v[e]);
      }
      return u32x4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
    };
    int64_t g = t;
    for (; g + 256 < n8; g += 512) {
      const f32x4 a0 = ((const f32x4*)src)[2 * g], b0 = ((const f32x4*)src)[2 * g + 1];
      const f32x4 a1 = ((const f32x4*)src)[2 * (g + 256)], b1 = ((const f32x4*)src)[2 * (g + 256) + 1];
      ((u32x4*)dst)[g] = conv8(a0, b0);
      ((u32x4*)dst)[g + 256] = conv8(a1, b1);
    }
    for (; g < n8; g += 256) {
      const f32x4 a0 = ((const f32x4*)src)[2 * g], b0 = ((const f32x4*)src)[2 * g + 1];
      ((u32x4*)dst)[g] = conv8(a0, b0);
    }
    for (int64_t c = 8 * n8 + t; c < ldb; c += 256) {
      const float v = c < n ? src[c] : 0.0f;
      if (check) flag |= scan_bits(v);
      dst[c] = f32_to_bf16_rne(v);
    }
  }
  if (check) or_status(status, flag);
}

hipError_t launch_cast_bf16(const float* X, int64_t m, int64_t n, int64_t ldx, bf16_t* Xb,
                            int64_t ldb, unsigned* status, int check, hipStream_t s) {
  if (m <= 0 || ldb <= 0) return hipSuccess;
  const int vec = (ldx % 4 == 0 && ((uintptr_t)X % 16) == 0 && ldb % 8 == 0 && ((uintptr_t)Xb % 16) == 0) ? 1 : 0;
  const int64_t blocks = m < 8192 ? m : 8192;
  hipLaunchKernelGGL(cast_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, m, n, ldx, Xb,
                     ldb, status, check, vec);
  return hipGetLastError();
}

template <typename T>
__global__ void check_kernel(const T* __restrict__ X, int64_t m, int64_t n, int64_t ldx, unsigned* status) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned flag = 0;
  for (; i < m * n; i += stride) {
    int64_t r = i / n, c = i - r * n;
    flag |= scan_bits(X[r * ldx + c]);
  }
  or_status(status, flag);
}

hipError_t launch_check_input(const void* X, int dt, int64_t m, int64_t n, int64_t ldx,
                              unsigned* status, hipStream_t s) {
  int64_t work = m * n;
  if (work == 0) return hipSuccess;
  int64_t blocks = (work + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (dt == 0)
    hipLaunchKernelGGL(check_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const double*)X, m, n, ldx, status);
  else
    hipLaunchKernelGGL(check_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const float*)X, m, n, ldx, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Relative error: per 64 x 64 tile of X, D = W H by register-blocked FMA
// (each thread a 4 x 4 block), E = X - D, and sums of E^2 and X^2 in FP64.
// One pair of partial sums per workgroup; a single workgroup then adds the
// partials in index order, so the result is deterministic.
// ---------------------------------------------------------------------------
template <typename XT> __device__ __forceinline__ double ld_x(const XT* p) { return (double)*p; }
template <> __device__ __forceinline__ double ld_x<bf16_t>(const bf16_t* p) {
  return (double)__uint_as_float(((unsigned)*p) << 16);
}

template <typename T, typename XT>
__global__ __launch_bounds__(256) void relerr_kernel(const XT* __restrict__ X, int64_t m, int64_t n,
                                                     int64_t ldx, const T* __restrict__ W,
                                                     const T* __restrict__ H, int k,
                                                     double* __restrict__ part) {
  constexpr int KC = 16;
  __shared__ T Ws[KC][64 + 1];
  __shared__ T Hs[KC][64 + 1];
  __shared__ double red[2][256];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = (T)0;
  for (int k0 = 0; k0 < k; k0 += KC) {
    for (int e = threadIdx.x; e < KC * 64; e += 256) {
      int kk = e / 64, rr = e % 64;
      int64_t r = r0 + rr;
      Ws[kk][rr] = (r < m && k0 + kk < k) ? W[r * k + k0 + kk] : (T)0;
      int64_t c = c0 + rr;
      Hs[kk][rr] = (c < n && k0 + kk < k) ? H[(int64_t)(k0 + kk) * n + c] : (T)0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KC; ++kk) {
      T wa[4], hb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) wa[a] = Ws[kk][ty + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) hb[b] = Hs[kk][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(wa[a], hb[b], acc[a][b]);
    }
    __syncthreads();
  }
  double se = 0.0, sx = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int64_t r = r0 + ty + 16 * a;
    if (r >= m) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int64_t c = c0 + tx + 16 * b;
      if (c >= n) continue;
      double x = ld_x<XT>(X + r * ldx + c);
      T xt = (T)x;
      T e = xt - acc[a][b];
      se += (double)e * (double)e;
      sx += x * x;
    }
  }
  red[0][threadIdx.x] = se;
  red[1][threadIdx.x] = sx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    size_t b = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    part[2 * b] = red[0][0];
    part[2 * b + 1] = red[1][0];
  }
}

__global__ __launch_bounds__(1024) void sum_pairs_kernel(const double* __restrict__ part, int np,
                                                         double* __restrict__ out) {
  __shared__ double red[2][1024];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < np; i += 1024) { a += part[2 * i]; b += part[2 * i + 1]; }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] += red[0][threadIdx.x + o];
      red[1][threadIdx.x] += red[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[0] = red[0][0]; out[1] = red[1][0]; }
}

// FP32 X: ||X - W H||_F^2 and ||X||_F^2 with W H on FP32 matrix cores
// (v_mfma_f32_16x16x4_f32: lane (i, g) holds A[i][g], B[g][i], and D[4g + e][i]
// in element e).  The product is formed transposed, D = H^T W^T, so that lane
// (i, g) holds W H at row i and the 4 adjacent columns 4g .. 4g + 3 of a
// 16 x 16 tile: the lane reads its X values with one 16-byte load (VEC: n and
// ldx multiples of 4, X 16-byte aligned; otherwise element by element).  A
// workgroup owns a balanced range of 16-row tiles (wave w: tiles w, w + 8,
// ...) and keeps their W fragments in registers; H passes through LDS 64
// columns at a time (register prefetch, double buffer).  X is read once, one
// tile ahead of the products that consume it.  Squared differences are added
// per tile in FP32 and across tiles in FP64.
typedef float rfloatx4 __attribute__((ext_vector_type(4)));

template <int RWMAX, bool VEC>
__global__ __launch_bounds__(512) void relerr_mfma_kernel(const float* __restrict__ X, int64_t m, int64_t n,
                                                          int64_t ldx, const float* __restrict__ W,
                                                          const float* __restrict__ H, int k, int tiles, int G,
                                                          double* __restrict__ part) {
  constexpr int KSM = 16;                 // 4-wide reduction steps, k <= 64
  constexpr int PF = KSM * 4 * 64 / 512;  // H elements per thread per block
  __shared__ float hs[2][KSM * 4 * 64];
  __shared__ double red[2][8];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int i = lane & 15, gq = lane >> 4;
  const int gidx = blockIdx.x;
  const int t0 = (int)((int64_t)tiles * gidx / G), t1 = (int)((int64_t)tiles * (gidx + 1) / G);
  const int nt = t1 - t0;
  const int ks = (k + 3) >> 2;
  // row tiles of this wave: wave + 8 rt < nt for rt < nrt
  int nrt = nt > wave ? (nt - wave + 7) / 8 : 0;
  if (nrt > RWMAX) nrt = RWMAX;
  float wf[RWMAX][KSM];
#pragma unroll
  for (int rt = 0; rt < RWMAX; ++rt) {
    const int tau = wave + 8 * rt;
    const int64_t r = (int64_t)(t0 + tau) * 16 + i;
#pragma unroll
    for (int s = 0; s < KSM; ++s) {
      const int kk = 4 * s + gq;
      wf[rt][s] = (tau < nt && r < m && kk < k) ? W[r * k + kk] : 0.0f;
    }
  }
  const int64_t nb = (n + 63) / 64;
  float pre[PF];
  auto fetch = [&](int64_t cb) {
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = t + q * 512;
      const int kk = e >> 6, c = e & 63;
      const int64_t col = cb * 64 + c;
      pre[q] = (kk < k && col < n) ? H[(int64_t)kk * n + col] : 0.0f;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int e = t + q * 512;
      const int kk = e >> 6, c = e & 63;
      // fragment layout [s][ct][g][i]: lane (i, g) of column tile ct reads one word
      hs[buf][((((kk >> 2) * 4) + (c >> 4)) * 4 + (kk & 3)) * 16 + (c & 15)] = pre[q];
    }
  };
  // X of column tile ct of block cb: lane (i, g), row tile tau -> row
  // 16 tau + i, columns 64 cb + 16 ct + 4 g + e (zero outside X)
  auto load_x = [&](int64_t cb, int ct, rfloatx4 (&xv)[RWMAX]) {
    const int64_t col = cb * 64 + ct * 16 + 4 * gq;
#pragma unroll
    for (int rt = 0; rt < RWMAX; ++rt) {
      const int tau = wave + 8 * rt;
      const int64_t row = (int64_t)(t0 + tau) * 16 + i;
      const bool live = tau < nt && row < m;
      rfloatx4 v = rfloatx4{0.f, 0.f, 0.f, 0.f};
      if constexpr (VEC) {
        if (live && col < n) v = *(const rfloatx4*)(X + row * ldx + col);  // n % 4 == 0: all 4 inside
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (live && col + e < n) v[e] = X[row * ldx + col + e];
      }
      xv[rt] = v;
    }
  };
  double se = 0.0, sx = 0.0;
  rfloatx4 xa[RWMAX], xb[RWMAX];
  load_x(0, 0, xa);
  fetch(0);
  store(0);
  __syncthreads();
  for (int64_t cb = 0; cb < nb; ++cb) {
    const int buf = (int)(cb & 1);
    if (cb + 1 < nb) fetch(cb + 1);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      // the next tile's X is in flight while this tile's products run
      if (ct < 3) load_x(cb, ct + 1, xb);
      else if (cb + 1 < nb) load_x(cb + 1, 0, xb);
      float hf[KSM];
#pragma unroll
      for (int s = 0; s < KSM; ++s) hf[s] = (s < ks) ? hs[buf][(s * 4 + ct) * 64 + lane] : 0.0f;
      // the wave's live row tiles are rt < nrt; their product chains are
      // interleaved (one compile-time form per count) so that the matrix
      // cores never wait on the previous product of the same chain
      auto products = [&](auto R) __attribute__((always_inline)) {
        constexpr int NR = decltype(R)::value;
        rfloatx4 d[NR];
#pragma unroll
        for (int rt = 0; rt < NR; ++rt) d[rt] = rfloatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < KSM; ++s)
          if (s < ks)
#pragma unroll
            for (int rt = 0; rt < NR; ++rt) d[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(hf[s], wf[rt][s], d[rt], 0, 0, 0);
#pragma unroll
        for (int rt = 0; rt < NR; ++rt) {
          float le = 0.0f, lx = 0.0f;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float df = xa[rt][e] - d[rt][e];  // rows and columns outside X hold x = 0 and d = 0
            le = fmaf(df, df, le);
            lx = fmaf(xa[rt][e], xa[rt][e], lx);
          }
          se += (double)le;
          sx += (double)lx;
        }
      };
      static_assert(RWMAX == 4, "one products form per live tile count");
      switch (nrt) {
        case 4: products(std::integral_constant<int, 4>{}); break;
        case 3: products(std::integral_constant<int, 3>{}); break;
        case 2: products(std::integral_constant<int, 2>{}); break;
        case 1: products(std::integral_constant<int, 1>{}); break;
        default: break;
      }
#pragma unroll
      for (int rt = 0; rt < RWMAX; ++rt) xa[rt] = xb[rt];
    }
    if (cb + 1 < nb) store(buf ^ 1);
    __syncthreads();
  }
  for (int o = 32; o > 0; o >>= 1) {
    se += __shfl_xor(se, o);
    sx += __shfl_xor(sx, o);
  }
  if (lane == 0) { red[0][wave] = se; red[1][wave] = sx; }
  __syncthreads();
  if (t == 0) {
    double a = 0.0, b = 0.0;
    for (int w = 0; w < 8; ++w) { a += red[0][w]; b += red[1][w]; }
    part[2 * gidx] = a;
    part[2 * gidx + 1] = b;
  }
}

int relerr_parts(int64_t m, int64_t n) { return ceil_div(m, 64) * ceil_div(n, 64); }

hipError_t launch_relerr(const void* X, int xt, int dt, int64_t m, int64_t n, int64_t ldx,
                         const void* W, const void* H, int k, double* part, int nparts_max,
                         double* out, hipStream_t s) {
  // one workgroup per CU over balanced 16-row tiles, at most 32 tiles each;
  // a short matrix (the compressed l x n error) would leave a few workgroups
  // streaming whole rows, so it takes the 64 x 64 tiled kernel instead
  const int64_t tiles = ceil_div(m, 16);
  if (dt == 1 && xt != 2 && k <= 64 && tiles >= 128) {
    int64_t g = 256;
    if (g > tiles) g = tiles;
    if (g < ceil_div(tiles, 32)) g = ceil_div(tiles, 32);
    if (g <= nparts_max) {
      const bool vec = n % 4 == 0 && ldx % 4 == 0 && ((uintptr_t)X & 15) == 0;
      if (vec)
        hipLaunchKernelGGL((relerr_mfma_kernel<4, true>), dim3((unsigned)g), dim3(512), 0, s, (const float*)X, m, n,
                           ldx, (const float*)W, (const float*)H, k, (int)tiles, (int)g, part);
      else
        hipLaunchKernelGGL((relerr_mfma_kernel<4, false>), dim3((unsigned)g), dim3(512), 0, s, (const float*)X, m, n,
                           ldx, (const float*)W, (const float*)H, k, (int)tiles, (int)g, part);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(1024), 0, s, part, (int)g, out);
      return hipGetLastError();
    }
  }
  int gx = ceil_div(n, 64), gy = ceil_div(m, 64);
  if ((int64_t)gx * gy > nparts_max || gy > 65535) return hipErrorInvalidValue;
  dim3 grid(gx, gy);
  if (dt == 0) {
    hipLaunchKernelGGL((relerr_kernel<double, double>), grid, dim3(256), 0, s, (const double*)X, m,
                       n, ldx, (const double*)W, (const double*)H, k, part);
  } else if (xt == 2) {
    hipLaunchKernelGGL((relerr_kernel<float, bf16_t>), grid, dim3(256), 0, s, (const bf16_t*)X, m,
                       n, ldx, (const float*)W, (const float*)H, k, part);
  } else {
    hipLaunchKernelGGL((relerr_kernel<float, float>), grid, dim3(256), 0, s, (const float*)X, m, n,
                       ldx, (const float*)W, (const float*)H, k, part);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(1024), 0, s, part, gx * gy, out);
  return hipGetLastError();
}

}  // namespace rnmf

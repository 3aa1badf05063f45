// Deterministic HALS (Sec. 3.1): the block updates applied to X itself, the
// algorithm that randomized HALS compresses.  One sweep streams X twice:
//   H phase: R = X^T W (TN pass), S = W^T W (FP64 Gram), then the rows of H
//            in turn, H(j,:) <- max(0, H(j,:) + (R(:,j) - H^T S(:,j)) / S_jj);
//   W phase: T = X H^T (NN pass), V = H H^T (FP64 Gram), then the columns of
//            W in turn, W(:,j) <- max(0, W(:,j) + (T(:,j) - W V(:,j)) / V_jj).
// The H rows are independent across columns of H and the W columns are
// independent across rows of W, so both Gauss-Seidel sweeps run without any
// device-wide exchange; a block with an exactly zero scale is skipped.
#include "rnmf_common.h"

namespace rnmf {

namespace {

template <typename T>
__device__ __forceinline__ T clip0h(T x) { return x > (T)0 ? x : (T)0; }

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Rows of H, one wave per column c of H: lane i holds H(i, c) and the running
// gradient g_i = R(c, i) - sum_p S(p, i) H(p, c) (FP64); the Gauss-Seidel
// step for row j broadcasts lane j's values and updates every g by rank one.
// Regularized rule (Sec. 3.4): the scale is S_jj + ah and the numerator gains
// - bh - ah H(j, c); since lane j's g is read only at step j, when H(j, c)
// still holds its old value, that constant is folded into g at the start.
template <typename T>
__global__ __launch_bounds__(256) void hrow_kernel(const T* __restrict__ R, const double* __restrict__ S,
                                                   T* __restrict__ H, int64_t n, int k, double ah, double bh) {
  __shared__ double Ss[KMAX * KMAX];
  for (int e = threadIdx.x; e < k * k; e += 256) Ss[e] = S[e];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  const int i = lane < k ? lane : 0;
  double h = lane < k ? (double)H[(int64_t)lane * n + c] : 0.0;
  double g = lane < k ? (double)R[c * k + lane] : 0.0;
  for (int p = 0; p < k; ++p) g = fma(-Ss[p * k + i], readlane_d(h, p), g);
  g -= fma(ah, h, bh);
  if (lane >= k) g = 0.0;
  const double dj = Ss[i * k + i] + ah;
  const double rs = (lane < k && dj > 0.0) ? 1.0 / dj : 0.0;
  for (int j = 0; j < k; ++j) {
    const double rd = readlane_d(rs, j);
    if (rd > 0.0) {
      const double hj = readlane_d(h, j), gj = readlane_d(g, j);
      // the new entry is rounded to the storage type before it is used
      const double hn = (double)clip0h<T>((T)fma(gj, rd, hj));
      const double delta = hn - hj;
      if (lane == j) h = hn;
      g = fma(-Ss[j * k + i], delta, g);
    }
  }
  if (lane < k) H[(int64_t)lane * n + c] = (T)h;
}

// Columns of W, one thread per row r: V (FP64) and the row (in T, which
// holds every value the update produces exactly) live in LDS, sized for k; for
// each column j the update uses the row as already updated (Gauss-Seidel).
// Regularized rule (Sec. 3.4): scale V_jj + aw, numerator - bw - aw W(r, j).
// The row of W is loaded with all its loads in flight, and T(r, :) is read
// eight columns ahead of its use; a thread past the last row reads row m - 1
// (so no load needs a select) and writes nothing.
template <typename T, int NT>
__global__ __launch_bounds__(256) void wrow_kernel(const T* __restrict__ Tm, const double* __restrict__ V,
                                                   T* __restrict__ W, int64_t m, int k, double aw, double bw) {
  extern __shared__ double wr_lds[];
  double* Vs = wr_lds;        // k x k
  T* ws = (T*)(wr_lds + k * k);  // k x NT: entry (p, t) at p * NT + t
  for (int e0 = threadIdx.x; e0 < k * k; e0 += 8 * NT) {  // eight loads in flight
    double v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int e = e0 + i * NT;
      v[i] = V[e < k * k ? e : 0];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (e0 + i * NT < k * k) Vs[e0 + i * NT] = v[i];
  }
  const int t = threadIdx.x;
  const int64_t r = (int64_t)blockIdx.x * NT + t;
  const bool live = r < m;
  const T* wrow = W + (live ? r : m - 1) * k;
  const T* trow = Tm + (live ? r : m - 1) * k;
  {
    T v[KMAX];
#pragma unroll
    for (int p = 0; p < KMAX; ++p) v[p] = wrow[p < k ? p : k - 1];
#pragma unroll
    for (int p = 0; p < KMAX; ++p)
      if (p < k) ws[p * NT + t] = v[p];
  }
  __syncthreads();
  if (!live) return;
  T tc[8], tn[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) tc[i] = trow[i < k ? i : k - 1];
  for (int j0 = 0; j0 < k; j0 += 8) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int jn = j0 + 8 + i;
      tn[i] = trow[jn < k ? jn : k - 1];
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int j = j0 + i;
      if (j >= k) break;
      const double d = Vs[j * k + j] + aw;
      if (!(d > 0.0)) continue;
      double s0 = 0.0, s1 = 0.0;
      int p = 0;
      for (; p + 2 <= k; p += 2) {
        s0 = fma((double)ws[p * NT + t], Vs[p * k + j], s0);
        s1 = fma((double)ws[(p + 1) * NT + t], Vs[(p + 1) * k + j], s1);
      }
      for (; p < k; ++p) s0 = fma((double)ws[p * NT + t], Vs[p * k + j], s0);
      const double wj = (double)ws[j * NT + t];
      const double num = ((double)tc[i] - (s0 + s1)) - fma(aw, wj, bw);
      ws[j * NT + t] = clip0h<T>((T)(wj + num / d));
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) tc[i] = tn[i];
  }
  for (int q = 0; q < k; ++q) W[r * k + q] = ws[q * NT + t];
}

// Hp (lp x ldp, zero padded) = H (k x n): the small operand of X H^T in the
// transposed layout the NN pass reads.
template <typename T>
__global__ __launch_bounds__(256) void pad_kernel(const T* __restrict__ H, int k, int64_t n, int lp, int64_t ldp,
                                                  T* __restrict__ Hp) {
  const int64_t total = (int64_t)lp * ldp;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / ldp, c = e - (e / ldp) * ldp;
    Hp[e] = (i < k && c < n) ? H[i * n + c] : (T)0;
  }
}

// Partial Gram H H^T of a k x n row-major matrix (k <= RMAX) over a chunk of
// 64 columns (FP64), written in the partial layout of the Cholesky QR Gram
// (entry (a, b), a <= b, at a*LMAX+b).  Used for V = H H^T and for B B^T.
template <typename T, int RMAX>
__global__ __launch_bounds__(256) void hgram_kernel(const T* __restrict__ H, int k, int64_t n,
                                                    double* __restrict__ part) {
  __shared__ double Hs[RMAX][65];
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  for (int e = threadIdx.x; e < k * 64; e += 256) {
    const int i = e / 64, cc = e - (e / 64) * 64;
    Hs[i][cc] = (c0 + cc < n) ? (double)H[(int64_t)i * n + c0 + cc] : 0.0;
  }
  __syncthreads();
  double* dst = part + (size_t)blockIdx.x * LMAX * LMAX;
  const int np = k * (k + 1) / 2;
  for (int q = threadIdx.x; q < np; q += 256) {
    // q -> (a, b) with a <= b, row-major over the upper triangle
    int a = 0, rem = q;
    while (rem >= k - a) { rem -= k - a; ++a; }
    const int b = a + rem;
    double s0 = 0.0, s1 = 0.0;
    for (int cc = 0; cc < 64; cc += 2) {
      s0 = fma(Hs[a][cc], Hs[b][cc], s0);
      s1 = fma(Hs[a][cc + 1], Hs[b][cc + 1], s1);
    }
    dst[a * LMAX + b] = s0 + s1;
  }
}

}  // namespace

hipError_t launch_hrow(const void* R, const double* S, void* H, int64_t n, int k, double ah, double bh, int dt,
                       hipStream_t s) {
  dim3 grid((unsigned)ceil_div(n, 4));
  if (dt == 0)
    hipLaunchKernelGGL(hrow_kernel<double>, grid, dim3(256), 0, s, (const double*)R, S, (double*)H, n, k, ah, bh);
  else
    hipLaunchKernelGGL(hrow_kernel<float>, grid, dim3(256), 0, s, (const float*)R, S, (float*)H, n, k, ah, bh);
  return hipGetLastError();
}

// 256 rows per workgroup where V and the rows fit in 128 KB of LDS (at most
// 96 KB with 128 rows, for any k <= KMAX).
template <typename T>
static hipError_t wrow_t(const T* Tm, const double* V, T* W, int64_t m, int k, double aw, double bw,
                         hipStream_t s) {
  const size_t v_bytes = (size_t)k * k * sizeof(double);
  const size_t b256 = v_bytes + (size_t)k * 256 * sizeof(T), b128 = v_bytes + (size_t)k * 128 * sizeof(T);
  hipError_t e;
  if (b256 <= 128 * 1024) {
    if ((e = hipFuncSetAttribute((const void*)wrow_kernel<T, 256>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)b256)) != hipSuccess)
      return e;
    hipLaunchKernelGGL((wrow_kernel<T, 256>), dim3((unsigned)ceil_div(m, 256)), dim3(256), b256, s, Tm, V, W, m, k,
                       aw, bw);
  } else {
    if ((e = hipFuncSetAttribute((const void*)wrow_kernel<T, 128>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)b128)) != hipSuccess)
      return e;
    hipLaunchKernelGGL((wrow_kernel<T, 128>), dim3((unsigned)ceil_div(m, 128)), dim3(128), b128, s, Tm, V, W, m, k,
                       aw, bw);
  }
  return hipGetLastError();
}

hipError_t launch_wrow(const void* Tm, const double* V, void* W, int64_t m, int k, double aw, double bw, int dt,
                       hipStream_t s) {
  if (k < 1 || k > KMAX) return hipErrorInvalidValue;
  if (dt == 0) return wrow_t((const double*)Tm, V, (double*)W, m, k, aw, bw, s);
  return wrow_t((const float*)Tm, V, (float*)W, m, k, aw, bw, s);
}

hipError_t launch_pad(const void* H, int k, int64_t n, int lp, int64_t ldp, void* Hp, int dt, hipStream_t s) {
  int64_t blocks = ceil_div((int64_t)lp * ldp, 256);
  if (blocks > 4096) blocks = 4096;
  if (dt == 0)
    hipLaunchKernelGGL(pad_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, s, (const double*)H, k, n, lp,
                       ldp, (double*)Hp);
  else
    hipLaunchKernelGGL(pad_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s, (const float*)H, k, n, lp, ldp,
                       (float*)Hp);
  return hipGetLastError();
}

int hgram_splits(int64_t n) { return (int)ceil_div(n, 64); }

hipError_t launch_hgram(const void* H, int k, int64_t n, double* part, int dt, hipStream_t s) {
  if (k < 1 || k > GRAM_ROWS_MAX) return hipErrorInvalidValue;
  dim3 grid((unsigned)hgram_splits(n));
  if (k <= KMAX) {
    if (dt == 0)
      hipLaunchKernelGGL((hgram_kernel<double, KMAX>), grid, dim3(256), 0, s, (const double*)H, k, n, part);
    else
      hipLaunchKernelGGL((hgram_kernel<float, KMAX>), grid, dim3(256), 0, s, (const float*)H, k, n, part);
  } else {
    if (dt == 0)
      hipLaunchKernelGGL((hgram_kernel<double, GRAM_ROWS_MAX>), grid, dim3(256), 0, s, (const double*)H, k, n,
                         part);
    else
      hipLaunchKernelGGL((hgram_kernel<float, GRAM_ROWS_MAX>), grid, dim3(256), 0, s, (const float*)H, k, n,
                         part);
  }
  return hipGetLastError();
}

}  // namespace rnmf

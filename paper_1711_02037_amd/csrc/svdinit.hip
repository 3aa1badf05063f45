// SVD-based initialization (the Remark on initialization after Algorithm 1):
// the nonnegative double SVD of Boutsidis and Gallopoulos (2008) applied to
// the k leading singular triplets of the randomized SVD that the QB
// decomposition gives (Sec. 2.3): X ~ Q B, B = U_B S V^T, so X ~ (Q U_B) S V^T.
//   1. C = B B^T: FP64 partial Grams of 64-column chunks, fixed-order sum;
//   2. C = U_B diag(lambda) U_B^T by cyclic parallel Jacobi in one workgroup
//      (FP64; C and the accumulated rotations in LDS); s_j = sqrt(lambda_j),
//      in descending order;
//   3. U = Q U_B(:, 1:k) into W and V^T = diag(1/s) U_B(:, 1:k)^T B into H,
//      with per-block sums of squares of the positive and negative parts of
//      every column of U and every row of V^T (fixed-order wave sums);
//   4. per component, which parts to keep and the scale (one workgroup):
//      component 1 keeps |u|, |v| scaled by sqrt(s_1); component j > 1 keeps
//      the positive parts if ||u+|| ||v+|| > ||u-|| ||v-||, else the negative
//      parts, scaled to sqrt(s_j * that product) over the kept norms; a
//      component whose two products vanish is zero;
//   5. W and H are replaced in place by the kept parts, scaled.
#include "rnmf_common.h"

namespace rnmf {

namespace {

constexpr int JAC_MAXSW = 40;  // sweeps; well-separated spectra need about 10
constexpr int LB = 64;         // rows (columns) per block in steps 3 and 5

// Circle-method round robin on N (even) indices: in round r pair i joins two
// indices, the N / 2 pairs are disjoint, and over N - 1 rounds every pair of
// indices meets exactly once.
__device__ __forceinline__ void rr_pair(int r, int i, int N, int& p, int& q) {
  if (i == 0) {
    p = N - 1;
    q = r;
  } else {
    p = (r + i) % (N - 1);
    q = (r - i + (N - 1)) % (N - 1);
  }
}

// Eigen-decomposition of the symmetric l x l matrix C (l <= LSVD), one
// workgroup.  Each round rotates N / 2 disjoint index pairs at once: the
// rotation zeroing A(p, q) (the symmetric 2 x 2 Schur decomposition) is
// applied to rows p, q, then to columns p, q of A and of V.  A rotation is
// skipped when |A(p, q)| <= max(1e-15 sqrt(|A(p, p) A(q, q)|), 1e-15 tr C);
// the iteration stops after a sweep without rotations.
__global__ __launch_bounds__(256) void jacobi_kernel(const double* __restrict__ C, int l, int k,
                                                     double* __restrict__ Ub, double* __restrict__ sv) {
  extern __shared__ double smem[];
  const int P = l + 1;
  double* A = smem;
  double* V = A + (size_t)l * P;
  double* cs = V + (size_t)l * P;
  double* sn = cs + LSVD / 2;
  int* pp = (int*)(sn + LSVD / 2);
  int* qq = pp + LSVD / 2;
  __shared__ int rotated;
  __shared__ int order[LSVD];
  const int t = threadIdx.x;
  for (int e = t; e < l * l; e += 256) {
    const int i = e / l, j = e - (e / l) * l;
    A[i * P + j] = C[e];
    V[i * P + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  double tr = 0.0;
  for (int i = 0; i < l; ++i) tr += A[i * P + i];  // same order in every thread
  const double floor_abs = 1e-15 * fabs(tr);
  const int N = l + (l & 1), np = N / 2;
  for (int sw = 0; sw < JAC_MAXSW; ++sw) {
    if (t == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < N - 1; ++r) {
      if (t < np) {
        int p, q;
        rr_pair(r, t, N, p, q);
        double c = 1.0, s = 0.0;
        int use = 0;
        if (p < l && q < l) {
          const double apq = A[p * P + q], app = A[p * P + p], aqq = A[q * P + q];
          if (fabs(apq) > fmax(1e-15 * sqrt(fabs(app * aqq)), floor_abs)) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            use = 1;
          }
        }
        pp[t] = use ? p : -1;
        qq[t] = q;
        cs[t] = c;
        sn[t] = s;
        if (use) rotated = 1;
      }
      __syncthreads();
      // rows p, q of A
      for (int e = t; e < np * l; e += 256) {
        const int i = e / l, j = e - (e / l) * l;
        const int p = pp[i];
        if (p < 0) continue;
        const int q = qq[i];
        const double c = cs[i], s = sn[i];
        const double ap = A[p * P + j], aq = A[q * P + j];
        A[p * P + j] = c * ap - s * aq;
        A[q * P + j] = s * ap + c * aq;
      }
      __syncthreads();
      // columns p, q of A and of V
      for (int e = t; e < np * l; e += 256) {
        const int i = e / l, j = e - (e / l) * l;
        const int p = pp[i];
        if (p < 0) continue;
        const int q = qq[i];
        const double c = cs[i], s = sn[i];
        const double ap = A[j * P + p], aq = A[j * P + q];
        A[j * P + p] = c * ap - s * aq;
        A[j * P + q] = s * ap + c * aq;
        const double vp = V[j * P + p], vq = V[j * P + q];
        V[j * P + p] = c * vp - s * vq;
        V[j * P + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
    const int again = rotated;
    __syncthreads();  // every thread has read the flag before it is cleared
    if (!again) break;
  }
  // the k largest eigenvalues, descending (first index wins a tie)
  if (t == 0) {
    for (int i = 0; i < l; ++i) order[i] = i;
    for (int j = 0; j < k; ++j) {
      int best = j;
      for (int i = j + 1; i < l; ++i)
        if (A[order[i] * P + order[i]] > A[order[best] * P + order[best]]) best = i;
      const int x = order[j];
      order[j] = order[best];
      order[best] = x;
    }
  }
  __syncthreads();
  for (int e = t; e < l * k; e += 256) {
    const int a = e / k, j = e - (e / k) * k;
    Ub[e] = V[a * P + order[j]];
  }
  if (t < k) sv[t] = sqrt(fmax(A[order[t] * P + order[t]], 0.0));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// U = Q U_B(:, 1:k) for LB rows per one-wave block, into W (m x k), and the
// block's sums of squares of the positive and negative parts of each column.
template <typename T>
__global__ __launch_bounds__(LB) void svd_lift_kernel(const T* __restrict__ Q, int64_t m, int l,
                                                      const double* __restrict__ Ub, int k, T* __restrict__ W,
                                                      double* __restrict__ part) {
  __shared__ double qs[LB][LSVD + 1];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * LB;
  const int rows = (int)((m - r0) < LB ? (m - r0) : LB);
  for (int e = t; e < LB * l; e += LB) {
    const int i = e / l, a = e - (e / l) * l;
    qs[i][a] = i < rows ? (double)Q[(r0 + i) * l + a] : 0.0;
  }
  __syncthreads();
  const bool live = t < rows;
  for (int j0 = 0; j0 < k; j0 += 16) {
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    for (int a = 0; a < l; ++a) {
      const double qv = qs[t][a];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (j0 + u < k) acc[u] = fma(qv, Ub[a * k + j0 + u], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int j = j0 + u;
      if (j >= k) break;
      const double v = acc[u];
      if (live) W[(r0 + t) * k + j] = (T)v;
      const double ps = wave_sum(v > 0.0 ? v * v : 0.0);
      const double ns = wave_sum(v < 0.0 ? v * v : 0.0);
      if (t == 0) {
        part[((size_t)blockIdx.x * k + j) * 2] = ps;
        part[((size_t)blockIdx.x * k + j) * 2 + 1] = ns;
      }
    }
  }
}

// V^T = diag(1/s) U_B(:, 1:k)^T B for LB columns per one-wave block, into H
// (k x n), and the block's sums of squares of the positive and negative parts
// of each row.
template <typename T>
__global__ __launch_bounds__(LB) void svd_proj_kernel(const T* __restrict__ B, int64_t n, int l,
                                                      const double* __restrict__ Ub, const double* __restrict__ sv,
                                                      int k, T* __restrict__ H, double* __restrict__ part) {
  const int t = threadIdx.x;
  const int64_t c = (int64_t)blockIdx.x * LB + t;
  const bool live = c < n;
  for (int j0 = 0; j0 < k; j0 += 16) {
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    for (int a = 0; a < l; ++a) {
      const double b = live ? (double)B[(int64_t)a * n + c] : 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (j0 + u < k) acc[u] = fma(b, Ub[a * k + j0 + u], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int j = j0 + u;
      if (j >= k) break;
      const double s = sv[j];
      const double v = s > 0.0 ? acc[u] / s : 0.0;
      if (live) H[(int64_t)j * n + c] = (T)v;
      const double ps = wave_sum(v > 0.0 ? v * v : 0.0);
      const double ns = wave_sum(v < 0.0 ? v * v : 0.0);
      if (t == 0) {
        part[((size_t)blockIdx.x * k + j) * 2] = ps;
        part[((size_t)blockIdx.x * k + j) * 2 + 1] = ns;
      }
    }
  }
}

// Per component j (thread j): norms from the block sums (fixed order), then
// coef = (mode, scale for W, scale for H); mode 0 keeps |x|, 1 the positive
// part, -1 the negative part, 2 gives zero.
__global__ __launch_bounds__(64) void svd_decide_kernel(const double* __restrict__ upart, int nbu,
                                                        const double* __restrict__ vpart, int nbv,
                                                        const double* __restrict__ sv, int k,
                                                        double* __restrict__ coef) {
  const int j = threadIdx.x;
  if (j >= k) return;
  double up = 0.0, un = 0.0, vp = 0.0, vn = 0.0;
  for (int b = 0; b < nbu; ++b) {
    up += upart[((size_t)b * k + j) * 2];
    un += upart[((size_t)b * k + j) * 2 + 1];
  }
  for (int b = 0; b < nbv; ++b) {
    vp += vpart[((size_t)b * k + j) * 2];
    vn += vpart[((size_t)b * k + j) * 2 + 1];
  }
  const double s = sv[j];
  double mode = 0.0, cw, ch;
  if (j == 0) {
    cw = ch = sqrt(s);
  } else {
    const double xp = sqrt(up), xn = sqrt(un), yp = sqrt(vp), yn = sqrt(vn);
    const double mp = xp * yp, mn = xn * yn;
    double sig, nu, nv;
    if (mp > mn) {
      mode = 1.0; sig = mp; nu = xp; nv = yp;
    } else {
      mode = -1.0; sig = mn; nu = xn; nv = yn;
    }
    if (sig > 0.0) {
      const double c = sqrt(s * sig);
      cw = c / nu;
      ch = c / nv;
    } else {
      mode = 2.0;
      cw = ch = 0.0;
    }
  }
  coef[3 * j] = mode;
  coef[3 * j + 1] = cw;
  coef[3 * j + 2] = ch;
}

__device__ __forceinline__ double kept(double mode, double x) {
  if (mode == 0.0) return fabs(x);
  if (mode == 1.0) return x > 0.0 ? x : 0.0;
  if (mode == -1.0) return x < 0.0 ? -x : 0.0;
  return 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void svd_apply_kernel(T* __restrict__ W, int64_t m, T* __restrict__ H, int64_t n,
                                                        int k, const double* __restrict__ coef) {
  const int64_t nw = m * k, total = nw + (int64_t)k * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    if (e < nw) {
      const int j = (int)(e % k);
      W[e] = (T)(coef[3 * j + 1] * kept(coef[3 * j], (double)W[e]));
    } else {
      const int64_t f = e - nw;
      const int j = (int)(f / n);
      H[f] = (T)(coef[3 * j + 2] * kept(coef[3 * j], (double)H[f]));
    }
  }
}

template <typename T>
hipError_t svd_init_t(const T* Q, const T* B, int64_t m, int64_t n, int l, int k, T* W, T* H, const SvdBufs& b,
                      hipStream_t s) {
  const int dt = sizeof(T) == 8 ? 0 : 1;
  hipError_t e = launch_hgram(B, l, n, b.gpart, dt, s);
  if (e != hipSuccess) return e;
  if ((e = launch_gram_sum(b.gpart, hgram_splits(n), l, b.C, s)) != hipSuccess) return e;
  const size_t lds = (size_t)2 * l * (l + 1) * sizeof(double) + LSVD * sizeof(double) + LSVD * sizeof(int);
  e = hipFuncSetAttribute((const void*)jacobi_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(256), lds, s, b.C, l, k, b.Ub, b.sv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nbu = svd_row_blocks(m), nbv = svd_col_blocks(n);
  hipLaunchKernelGGL(svd_lift_kernel<T>, dim3(nbu), dim3(LB), 0, s, Q, m, l, b.Ub, k, W, b.upart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(svd_proj_kernel<T>, dim3(nbv), dim3(LB), 0, s, B, n, l, b.Ub, b.sv, k, H, b.vpart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(svd_decide_kernel, dim3(1), dim3(64), 0, s, b.upart, nbu, b.vpart, nbv, b.sv, k, b.coef);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int64_t blocks = ((m + n) * k + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(svd_apply_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, W, m, H, n, k, b.coef);
  return hipGetLastError();
}

}  // namespace

int svd_row_blocks(int64_t m) { return ceil_div(m, LB); }
int svd_col_blocks(int64_t n) { return ceil_div(n, LB); }

hipError_t launch_svd_init(const void* Q, const void* B, int64_t m, int64_t n, int l, int k, void* W, void* H,
                           int dt, const SvdBufs& b, hipStream_t s) {
  if (l < 1 || l > LSVD || k < 1 || k > l || k > KMAX) return hipErrorInvalidValue;
  if (dt == 0)
    return svd_init_t<double>((const double*)Q, (const double*)B, m, n, l, k, (double*)W, (double*)H, b, s);
  return svd_init_t<float>((const float*)Q, (const float*)B, m, n, l, k, (float*)W, (float*)H, b, s);
}

}  // namespace rnmf

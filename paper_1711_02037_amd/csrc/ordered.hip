// Compressed HALS sweeps with an explicit order of block updates (Sec. 3.2:
// the interleaved cyclic order W(:,1) -> H(1,:) -> ... -> W(:,k) -> H(k,:),
// the blocked orders and the shuffled order; plain rules, S = W^T W).  Every
// block update takes the products of the factors as they are at that moment:
//   W(:,j): T(:,j) = B H(j,:)^T and V(:,j) = H H(j,:)^T (sums over n), then
//           u = W~(:,j) + (T(:,j) - W~ V(:,j)) / V_jj, W(:,j) = max(0, Q u),
//           W~(:,j) = Q^T W(:,j) (a sum over m);
//   H(j,:): S(:,j) = W^T W(:,j) (a sum over m), then for every column c
//           H(j,c) <- max(0, H(j,c) + ((B^T W~)(c,j) - H(:,c) . S(:,j)) / S_jj).
// The sums over n and m are block partials in FP64 added in a fixed order, so
// the result is deterministic.  Blocks with a zero scale are skipped.  The
// persistent sweep kernel covers the blocked orders at full speed; this path
// runs any order with a few launches per block update.
#include "rnmf_common.h"

namespace rnmf {

namespace {

constexpr int OC = 128;  // columns of B and H per partial of T(:,j), V(:,j)
constexpr int OR = 256;  // rows of Q and W per partial of Q^T w and W^T w

// max(0, x), with +0 for x <= 0 and for NaN
__device__ __forceinline__ double clip_d(double x) { return x > 0.0 ? x : 0.0; }

// part(b, a) = sum over the block's columns c of M(a, c) H(j, c), with M the
// rows of B (a < l) and of H (a = l + p): the partial of T(:,j) and V(:,j).
template <typename T>
__global__ __launch_bounds__(256) void ord_tv_part(const T* __restrict__ B, const T* __restrict__ H, int64_t n,
                                                   int l, int k, int j, double* __restrict__ part) {
  __shared__ double hj[OC];
  const int t = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * OC;
  const int cnt = (n - c0) < OC ? (int)(n - c0) : OC;
  for (int c = t; c < OC; c += 256) hj[c] = c < cnt ? (double)H[(int64_t)j * n + c0 + c] : 0.0;
  __syncthreads();
  for (int a = t; a < l + k; a += 256) {
    const T* row = (a < l) ? B + (int64_t)a * n + c0 : H + (int64_t)(a - l) * n + c0;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int c = 0;
    for (; c + 4 <= cnt; c += 4) {
      s0 = fma((double)row[c], hj[c], s0);
      s1 = fma((double)row[c + 1], hj[c + 1], s1);
      s2 = fma((double)row[c + 2], hj[c + 2], s2);
      s3 = fma((double)row[c + 3], hj[c + 3], s3);
    }
    for (; c < cnt; ++c) s0 = fma((double)row[c], hj[c], s0);
    part[(int64_t)blockIdx.x * (l + k) + a] = (s0 + s1) + (s2 + s3);
  }
}

// out(a) = sum over b = 0..nb-1 of part(b, a), in order of b.
__global__ __launch_bounds__(256) void ord_sum(const double* __restrict__ part, int nb, int cnt,
                                               double* __restrict__ out) {
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= cnt) return;
  double s = 0.0;
#pragma unroll 8
  for (int b = 0; b < nb; ++b) s += part[(int64_t)b * cnt + a];
  out[a] = s;
}

// W column j from tv = (T(:,j), V(:,j)): the update vector u (every block
// forms it), the lift and clip of the block's rows, and the block partial of
// Q^T W(:,j) (thread a of group g adds rows g, g + groups, ...).
template <typename T>
__global__ __launch_bounds__(256) void ord_wcol(const T* __restrict__ Q, T* __restrict__ W, const T* __restrict__ Wt,
                                                const double* __restrict__ tv, int64_t m, int l, int k, int j,
                                                double* __restrict__ part) {
  const double d = tv[l + j];
  if (!(d > 0.0)) return;  // V_jj = 0: the column is skipped
  __shared__ double u[LMAX];
  __shared__ double z[OR];
  __shared__ double red[256];
  __shared__ double wts[LMAX * KMAX];
  __shared__ double tvs[LMAX + KMAX];
  const int t = threadIdx.x;
  // W~ and tv go to LDS first (all their loads in flight together), then u
#pragma unroll 8
  for (int e = t; e < l * k; e += 256) wts[e] = (double)Wt[e];
  for (int e = t; e < l + k; e += 256) tvs[e] = tv[e];
  __syncthreads();
  for (int a = t; a < l; a += 256) {
    double s = 0.0;
    for (int p = 0; p < k; ++p) s = fma(wts[a * k + p], tvs[l + p], s);
    u[a] = wts[a * k + j] + (tvs[a] - s) / d;
  }
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * OR;
  const int rows = (m - r0) < OR ? (int)(m - r0) : OR;
  double w = 0.0;
  if (t < rows) {
    const T* q = Q + (r0 + t) * l;
    double s = 0.0;
#pragma unroll 8
    for (int a = 0; a < l; ++a) s = fma((double)q[a], u[a], s);
    const T wv = (T)clip_d(s);
    W[(r0 + t) * k + j] = wv;
    w = (double)wv;
  }
  z[t] = w;
  __syncthreads();
  const int groups = 256 / l, grp = t / l, ta = t - (t / l) * l;
  double s = 0.0;
  if (grp < groups)
#pragma unroll 8
    for (int i = grp; i < rows; i += groups) s = fma((double)Q[(r0 + i) * l + ta], z[i], s);
  red[t] = s;
  __syncthreads();
  for (int a = t; a < l; a += 256) {
    double v = 0.0;
    for (int g = 0; g < groups; ++g) v += red[g * l + a];
    part[(int64_t)blockIdx.x * l + a] = v;
  }
}

// W~(:,j) = the fixed-order sum of the partials of Q^T W(:,j) (skipped with
// the column).
template <typename T>
__global__ __launch_bounds__(256) void ord_wfin(const double* __restrict__ part, int nb, int l, int k, int j,
                                                const double* __restrict__ tv, T* __restrict__ Wt) {
  if (!(tv[l + j] > 0.0)) return;
  const int a = threadIdx.x;
  if (a >= l) return;
  double s = 0.0;
#pragma unroll 8
  for (int b = 0; b < nb; ++b) s += part[(int64_t)b * l + a];
  Wt[a * k + j] = (T)s;
}

// part(b, p) = sum over the block's rows r of W(r, p) W(r, j): the partial of
// S(:,j) = W^T W(:,j).
template <typename T>
__global__ __launch_bounds__(256) void ord_scol_part(const T* __restrict__ W, int64_t m, int k, int j,
                                                     double* __restrict__ part) {
  __shared__ double z[OR];
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * OR;
  const int rows = (m - r0) < OR ? (int)(m - r0) : OR;
  z[t] = t < rows ? (double)W[(r0 + t) * k + j] : 0.0;
  __syncthreads();
  const int groups = 256 / k, grp = t / k, tp = t - (t / k) * k;
  double s = 0.0;
  if (grp < groups)
#pragma unroll 8
    for (int i = grp; i < rows; i += groups) s = fma((double)W[(r0 + i) * k + tp], z[i], s);
  red[t] = s;
  __syncthreads();
  for (int p = t; p < k; p += 256) {
    double v = 0.0;
    for (int g = 0; g < groups; ++g) v += red[g * k + p];
    part[(int64_t)blockIdx.x * k + p] = v;
  }
}

// Row j of H, one thread per column c, with S(:,j) in sv.
template <typename T>
__global__ __launch_bounds__(256) void ord_hrow(const T* __restrict__ B, const T* __restrict__ Wt, T* __restrict__ H,
                                                const double* __restrict__ sv, int64_t n, int l, int k, int j) {
  const double d = sv[j];
  if (!(d > 0.0)) return;  // S_jj = 0: the row is skipped
  __shared__ double wj[LMAX];
  __shared__ double s[KMAX];
  const int t = threadIdx.x;
  for (int a = t; a < l; a += 256) wj[a] = (double)Wt[a * k + j];
  for (int p = t; p < k; p += 256) s[p] = sv[p];
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * 256 + t;
  if (c >= n) return;
  double r = 0.0;
#pragma unroll 8
  for (int a = 0; a < l; ++a) r = fma((double)B[(int64_t)a * n + c], wj[a], r);
  double hs = 0.0;
#pragma unroll 8
  for (int p = 0; p < k; ++p) hs = fma((double)H[(int64_t)p * n + c], s[p], hs);
  const double v = (double)H[(int64_t)j * n + c] + (r - hs) / d;
  H[(int64_t)j * n + c] = (T)clip_d(v);
}

}  // namespace

int ord_part_elems(int64_t m, int64_t n, int l, int k) {
  const int64_t nbn = (n + OC - 1) / OC, nbm = (m + OR - 1) / OR;
  int64_t e = nbn * (l + k);
  if (nbm * l > e) e = nbm * l;
  if (nbm * k > e) e = nbm * k;
  return (int)e;
}

template <typename T>
static hipError_t ordered_t(const T* Q, const T* B, T* W, T* Wt, T* H, int64_t m, int64_t n, int l, int k, int e,
                            double* part, double* vec, hipStream_t s) {
  const int nbn = (int)((n + OC - 1) / OC), nbm = (int)((m + OR - 1) / OR);
  if (e < k) {
    const int j = e;
    hipLaunchKernelGGL(ord_tv_part<T>, dim3(nbn), dim3(256), 0, s, B, H, n, l, k, j, part);
    hipLaunchKernelGGL(ord_sum, dim3((l + k + 255) / 256), dim3(256), 0, s, part, nbn, l + k, vec);
    hipLaunchKernelGGL(ord_wcol<T>, dim3(nbm), dim3(256), 0, s, Q, W, Wt, vec, m, l, k, j, part);
    hipLaunchKernelGGL(ord_wfin<T>, dim3(1), dim3(256), 0, s, part, nbm, l, k, j, vec, Wt);
  } else {
    const int j = e - k;
    hipLaunchKernelGGL(ord_scol_part<T>, dim3(nbm), dim3(256), 0, s, W, m, k, j, part);
    hipLaunchKernelGGL(ord_sum, dim3(1), dim3(256), 0, s, part, nbm, k, vec);
    hipLaunchKernelGGL(ord_hrow<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, B, Wt, H, vec, n, l, k, j);
  }
  return hipGetLastError();
}

hipError_t launch_ordered_update(const void* Q, const void* B, void* W, void* Wt, void* H, int64_t m, int64_t n,
                                 int l, int k, int e, double* part, double* vec, int dt, hipStream_t s) {
  if (l < 1 || l > LMAX || k < 1 || k > KMAX || e < 0 || e >= 2 * k) return hipErrorInvalidValue;
  if (dt == 0)
    return ordered_t((const double*)Q, (const double*)B, (double*)W, (double*)Wt, (double*)H, m, n, l, k, e, part,
                     vec, s);
  return ordered_t((const float*)Q, (const float*)B, (float*)W, (float*)Wt, (float*)H, m, n, l, k, e, part, vec, s);
}

}  // namespace rnmf

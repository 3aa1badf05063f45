// Reverse mode through unrolled compressed-HALS sweeps (Algorithm 1's sweep,
// Sec. 3.2, with the basis Q held fixed; S = W^T W, rows of H first).  All
// adjoints are FP64; the forward states are in the factor type T.
//
// One sweep maps (W, W~, H) to (W', W~', H'):
//   H rows j = 1..k:   a_j = (R_j - sum_{p != j} S_pj Hc_p) / S_jj,  H'_j = max(0, a_j)
//                      (R = B^T W~, S = W^T W, Hc_p the current row: new for p < j)
//   W columns j = 1..k: u_j = (T_j - sum_{p != j} V_pj W~c_p) / V_jj,
//                      W'_j = max(0, Q u_j),  W~'_j = Q^T W'_j
//                      (T = B H'^T, V = H' H'^T, W~c_p new for p < j)
// (the printed rules include the old block, whose two terms cancel, so a
// replaced block has no derivative with respect to its own old value; the
// derivative of max(0, x) is taken as 0 at 0).  The reverse pass runs the W
// columns j = k..1, moves the T and V adjoints to H' and B, runs the H rows
// j = k..1 (the columns of H are independent and run in parallel), and moves
// the S and R adjoints to W, W~ and B.  Skipped blocks (zero scale) pass their
// adjoints through unchanged.
#include "rnmf_common.h"

namespace rnmf {

namespace {

template <typename T>
__device__ __forceinline__ double ld(const T* p, int64_t i) { return (double)p[i]; }

// C (M x N, FP64) (+)= alpha * opA(A) opB(B); op(X)(i, k) = X[i * ld + k] or,
// transposed, X[k * ld + i].  One thread per output, FP64 sums in order of k.
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void ad_gemm(int64_t M, int64_t N, int64_t K, const TA* __restrict__ A,
                                               int64_t lda, int ta, const TB* __restrict__ B, int64_t ldb, int tb,
                                               double* __restrict__ C, int64_t ldc, double alpha, int acc) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= M * N) return;
  const int64_t i = e / N, j = e - (e / N) * N;
  double s = 0.0;
  for (int64_t q = 0; q < K; ++q) {
    const double a = ta ? ld(A, q * lda + i) : ld(A, i * lda + q);
    const double b = tb ? ld(B, j * ldb + q) : ld(B, q * ldb + j);
    s = fma(a, b, s);
  }
  C[i * ldc + j] = acc ? C[i * ldc + j] + alpha * s : alpha * s;
}

// Same with a wavefront per output for long sums (K large, few outputs).
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void ad_gemm_wave(int64_t M, int64_t N, int64_t K, const TA* __restrict__ A,
                                                    int64_t lda, int ta, const TB* __restrict__ B, int64_t ldb,
                                                    int tb, double* __restrict__ C, int64_t ldc, double alpha,
                                                    int acc) {
  const int64_t e = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= M * N) return;
  const int64_t i = e / N, j = e - (e / N) * N;
  double s = 0.0;
  for (int64_t q = lane; q < K; q += 64) {
    const double a = ta ? ld(A, q * lda + i) : ld(A, i * lda + q);
    const double b = tb ? ld(B, j * ldb + q) : ld(B, q * ldb + j);
    s = fma(a, b, s);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) C[i * ldc + j] = acc ? C[i * ldc + j] + alpha * s : alpha * s;
}

// Butterfly sum over the 64 lanes of a wavefront (every lane gets the sum).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// W column j in reverse, part 1 (rows r of a 256-row block):
//   g = gW(r, j) + Q(r, :) gWt(:, j);  gz = g if W'(r, j) > 0 else 0;
//   gW(r, j) <- 0 (the old column has no derivative here);
//   part(blk, a) = sum over the block's rows of Q(r, a) gz(r).  For the
//   partial the workgroup splits into 256 / l groups of l threads; thread a
//   of group g adds rows g, g + groups, ... (reads of a row are contiguous
//   across the group), then the groups' sums are added in order.
template <typename T>
__global__ __launch_bounds__(256) void ad_wcol_a(const T* __restrict__ Q, const T* __restrict__ Wn, int64_t m,
                                                 int l, int k, int j, const double* __restrict__ V,
                                                 double* __restrict__ gW, const double* __restrict__ gWt,
                                                 double* __restrict__ part) {
  if (!(V[j * k + j] > 0.0)) return;  // skipped in the forward: adjoints pass through
  __shared__ double gwt[LMAX];
  __shared__ double gz[256];
  __shared__ double red[256];
  const int t = threadIdx.x;
  for (int a = t; a < l; a += 256) gwt[a] = gWt[(int64_t)a * k + j];
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * 256;
  const int64_t r = r0 + t;
  double z = 0.0;
  if (r < m) {
    const T* q = Q + r * l;
    double g = gW[r * k + j];
    for (int a = 0; a < l; ++a) g = fma((double)q[a], gwt[a], g);
    z = ((double)Wn[r * k + j] > 0.0) ? g : 0.0;
    gW[r * k + j] = 0.0;
  }
  gz[t] = z;
  __syncthreads();
  const int groups = 256 / l;
  const int grp = t / l, a = t - (t / l) * l;
  const int rows = (int)((m - r0) < 256 ? (m - r0) : 256);
  double s = 0.0;
  if (grp < groups) {
    const T* q = Q + r0 * l + a;
#pragma unroll 8
    for (int i = grp; i < rows; i += groups) s = fma((double)q[(int64_t)i * l], gz[i], s);
  }
  red[t] = s;
  __syncthreads();
  for (int e = t; e < l; e += 256) {
    double v = 0.0;
    for (int g2 = 0; g2 < groups; ++g2) v += red[g2 * l + e];
    part[(int64_t)blockIdx.x * l + e] = v;
  }
}

// W column j in reverse, part 2 (one workgroup of 16 wavefronts):
// gu = sum of the parts (wavefront w adds blocks w, w + 16, ..., then the 16
// sums in order); the update vector u_j; then gT(:, j) += gu / V_jj,
// gWt(:, p) -= V_pj / V_jj gu (p != j), gV(p, j) -= Wtc_p . gu / V_jj,
// gV(j, j) -= u . gu / V_jj, and gWt(:, j) <- 0.
// Wtc_p = Wt'(:, p) for p < j, Wt(:, p) for p > j.
template <typename T>
__global__ __launch_bounds__(1024) void ad_wcol_b(const T* __restrict__ Wto, const T* __restrict__ Wtn,
                                                  const double* __restrict__ Tm, const double* __restrict__ V,
                                                  int l, int k, int j, const double* __restrict__ part, int nblk,
                                                  double* __restrict__ gT, double* __restrict__ gWt,
                                                  double* __restrict__ gV) {
  const double d = V[j * k + j];
  if (!(d > 0.0)) return;
  __shared__ double sred[16][LMAX];
  __shared__ double gu[LMAX], u[LMAX], vj[KMAX];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int a = lane; a < l; a += 64) {
    double s = 0.0;
    for (int b = wv; b < nblk; b += 16) s += part[(int64_t)b * l + a];
    sred[wv][a] = s;
  }
  if (t < k) vj[t] = V[t * k + j];
  __syncthreads();
  if (t < l) {
    double s = 0.0;
    for (int w = 0; w < 16; ++w) s += sred[w][t];
    gu[t] = s;
  }
  // u(a) = (T(a, j) - sum_{p != j} V_pj Wtc(a, p)) / V_jj: one wavefront per a, lanes over p
  for (int a = wv; a < l; a += 16) {
    double v = 0.0;
    if (lane < k && lane != j)
      v = vj[lane] * (lane < j ? (double)Wtn[a * k + lane] : (double)Wto[a * k + lane]);
    v = wave_sum(v);
    if (lane == 0) u[a] = (Tm[a * k + j] - v) / d;
  }
  __syncthreads();
  for (int e = t; e < l * k; e += 1024) {
    const int a = e / k, p = e - (e / k) * k;
    if (p == j) {
      gT[a * k + j] += gu[a] / d;
      gWt[e] = 0.0;
    } else {
      gWt[e] -= vj[p] / d * gu[a];
    }
  }
  // gV(p, j): one wavefront per p, lanes over a
  for (int p = wv; p < k; p += 16) {
    double v = 0.0;
    for (int a = lane; a < l; a += 64) {
      const double w = (p == j) ? u[a] : (p < j ? (double)Wtn[a * k + p] : (double)Wto[a * k + p]);
      v = fma(w, gu[a], v);
    }
    v = wave_sum(v);
    if (lane == 0) gV[p * k + j] -= v / d;
  }
}

// H rows in reverse.  The columns of H are independent: a workgroup takes 32
// columns, stages their adjoints gH and the signs of H' in LDS, and each
// wavefront runs 8 of them with lane p holding gh_p.  For j = k..1 with
// S_jj > 0: ga = gh_j if H'(j, c) > 0 else 0; gA(j, c) = ga; gh_j <- 0;
// gh_p -= S_pj / S_jj ga (p != j).  gH(:, c) <- gh (the adjoint of the old H).
constexpr int HR_COLS = 32;

template <typename T>
__global__ __launch_bounds__(256) void ad_hrows(const T* __restrict__ Hn, const double* __restrict__ S, int64_t n,
                                                int k, double* __restrict__ gH, double* __restrict__ gA) {
  __shared__ double Ss[KMAX * KMAX];
  __shared__ double tg[KMAX][HR_COLS + 1];
  __shared__ double ta[KMAX][HR_COLS + 1];
  __shared__ unsigned char tm[KMAX][HR_COLS];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * HR_COLS;
  for (int e = t; e < k * k; e += 256) Ss[e] = S[e];
  for (int e = t; e < k * HR_COLS; e += 256) {
    const int p = e / HR_COLS, cc = e - (e / HR_COLS) * HR_COLS;
    const int64_t c = c0 + cc;
    const bool in = c < n;
    tg[p][cc] = in ? gH[(int64_t)p * n + c] : 0.0;
    tm[p][cc] = (in && (double)Hn[(int64_t)p * n + c] > 0.0) ? 1 : 0;
  }
  __syncthreads();
  for (int cc = wv; cc < HR_COLS; cc += 4) {
    double gh = lane < k ? tg[lane][cc] : 0.0;
    for (int j = k - 1; j >= 0; --j) {
      const double d = Ss[j * k + j];
      double ga = 0.0;
      if (d > 0.0) {
        const double ghj = __shfl(gh, j, 64);
        ga = tm[j][cc] ? ghj : 0.0;
        if (lane == j) gh = 0.0;
        else if (lane < k) gh = fma(-Ss[lane * k + j], ga / d, gh);
      }
      if (lane == 0) ta[j][cc] = ga;
    }
    if (lane < k) tg[lane][cc] = gh;
  }
  __syncthreads();
  for (int e = t; e < k * HR_COLS; e += 256) {
    const int p = e / HR_COLS, cc = e - (e / HR_COLS) * HR_COLS;
    const int64_t c = c0 + cc;
    if (c < n) {
      gH[(int64_t)p * n + c] = tg[p][cc];
      gA[(int64_t)p * n + c] = ta[p][cc];
    }
  }
}

// gS(p, j) = -(1 / S_jj) sum_c Hc(p, c) gA(j, c) with Hc = H' for p <= j
// (new rows, and a_j = H'_j where ga is nonzero) and H for p > j; 0 when
// S_jj = 0.  One wavefront per entry.
template <typename T>
__global__ __launch_bounds__(256) void ad_gs(const T* __restrict__ Hn, const T* __restrict__ Ho,
                                             const double* __restrict__ gA, const double* __restrict__ S, int64_t n,
                                             int k, double* __restrict__ gS) {
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= k * k) return;
  const int p = e / k, j = e - (e / k) * k;
  const double d = S[j * k + j];
  const T* Hc = (p <= j) ? Hn : Ho;
  double s = 0.0;
  for (int64_t c = lane; c < n; c += 64) s = fma((double)Hc[(int64_t)p * n + c], gA[(int64_t)j * n + c], s);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (lane == 0) gS[p * k + j] = (d > 0.0) ? -s / d : 0.0;
}

// gA(j, :) /= S_jj (0 when S_jj = 0): the adjoint of R^T row j, in place.
__global__ __launch_bounds__(256) void ad_scale_rows(double* __restrict__ gA, const double* __restrict__ S,
                                                     int64_t n, int k) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)k * n) return;
  const int j = (int)(e / n);
  const double d = S[j * k + j];
  gA[e] = (d > 0.0) ? gA[e] / d : 0.0;
}

// M = G + G^T (k x k)
__global__ __launch_bounds__(256) void ad_symm(const double* __restrict__ G, int k, double* __restrict__ M) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= k * k) return;
  const int i = e / k, j = e - (e / k) * k;
  M[e] = G[e] + G[j * k + i];
}

__global__ __launch_bounds__(256) void ad_fill(double* __restrict__ p, int64_t count, double v) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) p[e] = v;
}

template <typename T>
__global__ __launch_bounds__(256) void ad_cast(const double* __restrict__ src, int64_t count, T* __restrict__ dst) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256)
    dst[e] = (T)src[e];
}

unsigned grid_for(int64_t count) {
  int64_t b = (count + 255) / 256;
  if (b > 65535) b = 65535;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

// ---- launchers (dt: 0 = double states, 1 = float states) -------------------

template <typename TA, typename TB>
static hipError_t gemm_t(int64_t M, int64_t N, int64_t K, const TA* A, int64_t lda, int ta, const TB* B,
                         int64_t ldb, int tb, double* C, int64_t ldc, double alpha, int acc, hipStream_t s) {
  if (M * N <= 4096 && K >= 256) {
    const int64_t blocks = (M * N + 3) / 4;
    hipLaunchKernelGGL((ad_gemm_wave<TA, TB>), dim3((unsigned)blocks), dim3(256), 0, s, M, N, K, A, lda, ta, B, ldb,
                       tb, C, ldc, alpha, acc);
  } else {
    const int64_t blocks = (M * N + 255) / 256;
    hipLaunchKernelGGL((ad_gemm<TA, TB>), dim3((unsigned)blocks), dim3(256), 0, s, M, N, K, A, lda, ta, B, ldb, tb,
                       C, ldc, alpha, acc);
  }
  return hipGetLastError();
}

hipError_t ad_gemm_sd(int64_t M, int64_t N, int64_t K, const void* A, int adt, int64_t lda, int ta, const void* B,
                      int bdt, int64_t ldb, int tb, double* C, int64_t ldc, double alpha, int acc, hipStream_t s) {
  // adt / bdt: 0 = double, 1 = float
  if (adt == 0 && bdt == 0)
    return gemm_t((int64_t)M, N, K, (const double*)A, lda, ta, (const double*)B, ldb, tb, C, ldc, alpha, acc, s);
  if (adt == 0 && bdt == 1)
    return gemm_t(M, N, K, (const double*)A, lda, ta, (const float*)B, ldb, tb, C, ldc, alpha, acc, s);
  if (adt == 1 && bdt == 0)
    return gemm_t(M, N, K, (const float*)A, lda, ta, (const double*)B, ldb, tb, C, ldc, alpha, acc, s);
  return gemm_t(M, N, K, (const float*)A, lda, ta, (const float*)B, ldb, tb, C, ldc, alpha, acc, s);
}

hipError_t ad_wcol(const void* Q, const void* Wn, const void* Wto, const void* Wtn, int64_t m, int l, int k, int j,
                   const double* Tm, const double* V, double* gW, double* gWt, double* gT, double* gV, double* part,
                   int dt, hipStream_t s) {
  const int nblk = (int)((m + 255) / 256);
  if (dt == 0) {
    hipLaunchKernelGGL(ad_wcol_a<double>, dim3(nblk), dim3(256), 0, s, (const double*)Q, (const double*)Wn, m, l, k,
                       j, V, gW, gWt, part);
    hipLaunchKernelGGL(ad_wcol_b<double>, dim3(1), dim3(1024), 0, s, (const double*)Wto, (const double*)Wtn, Tm, V, l,
                       k, j, part, nblk, gT, gWt, gV);
  } else {
    hipLaunchKernelGGL(ad_wcol_a<float>, dim3(nblk), dim3(256), 0, s, (const float*)Q, (const float*)Wn, m, l, k, j,
                       V, gW, gWt, part);
    hipLaunchKernelGGL(ad_wcol_b<float>, dim3(1), dim3(1024), 0, s, (const float*)Wto, (const float*)Wtn, Tm, V, l, k,
                       j, part, nblk, gT, gWt, gV);
  }
  return hipGetLastError();
}

int ad_wcol_parts(int64_t m) { return (int)((m + 255) / 256); }

template <typename T>
static hipError_t hrows_t(const T* Hn, const double* S, int64_t n, int k, double* gH, double* gA, hipStream_t s) {
  const dim3 g((unsigned)((n + HR_COLS - 1) / HR_COLS));
  hipLaunchKernelGGL(ad_hrows<T>, g, dim3(256), 0, s, Hn, S, n, k, gH, gA);
  return hipGetLastError();
}

hipError_t ad_hrows_run(const void* Hn, const double* S, int64_t n, int k, double* gH, double* gA, int dt,
                        hipStream_t s) {
  if (k < 1 || k > KMAX) return hipErrorInvalidValue;
  return dt == 0 ? hrows_t((const double*)Hn, S, n, k, gH, gA, s) : hrows_t((const float*)Hn, S, n, k, gH, gA, s);
}

hipError_t ad_gs_run(const void* Hn, const void* Ho, const double* gA, const double* S, int64_t n, int k,
                     double* gS, int dt, hipStream_t s) {
  const unsigned blocks = (unsigned)((k * k + 3) / 4);
  if (dt == 0)
    hipLaunchKernelGGL(ad_gs<double>, dim3(blocks), dim3(256), 0, s, (const double*)Hn, (const double*)Ho, gA, S, n,
                       k, gS);
  else
    hipLaunchKernelGGL(ad_gs<float>, dim3(blocks), dim3(256), 0, s, (const float*)Hn, (const float*)Ho, gA, S, n, k,
                       gS);
  return hipGetLastError();
}

hipError_t ad_scale_rows_run(double* gA, const double* S, int64_t n, int k, hipStream_t s) {
  const int64_t blocks = ((int64_t)k * n + 255) / 256;
  hipLaunchKernelGGL(ad_scale_rows, dim3((unsigned)blocks), dim3(256), 0, s, gA, S, n, k);
  return hipGetLastError();
}

hipError_t ad_symm_run(const double* G, int k, double* M, hipStream_t s) {
  hipLaunchKernelGGL(ad_symm, dim3((unsigned)((k * k + 255) / 256)), dim3(256), 0, s, G, k, M);
  return hipGetLastError();
}

hipError_t ad_fill_run(double* p, int64_t count, double v, hipStream_t s) {
  hipLaunchKernelGGL(ad_fill, dim3(grid_for(count)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

hipError_t ad_cast_run(const double* src, int64_t count, void* dst, int dt, hipStream_t s) {
  if (dt == 0) hipLaunchKernelGGL(ad_cast<double>, dim3(grid_for(count)), dim3(256), 0, s, src, count, (double*)dst);
  else hipLaunchKernelGGL(ad_cast<float>, dim3(grid_for(count)), dim3(256), 0, s, src, count, (float*)dst);
  return hipGetLastError();
}

}  // namespace rnmf

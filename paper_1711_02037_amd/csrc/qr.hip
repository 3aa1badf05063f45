// Cholesky QR pieces for the orthonormalisation steps of the range finder
// (Sec. 2.3; Algorithm 1 uses a thin QR after every half-step).
//
// One Cholesky QR pass on a tall Y (rows x l):
//   G = Y^T Y            (FP64 accumulation; split over rows, fixed-order sum)
//   L = chol(G), L L^T = G (one workgroup, FP64, in LDS); if G is not
//                        numerically positive definite, G + s I is factored
//                        instead with the shift of Fukaya, Kannan, Nakatsukasa,
//                        Yamamoto, Yanagisawa (SIAM J. Sci. Comput. 2020),
//                        s = 11 (rows l + l (l + 1)) u ||Y||_F^2, u = 2^-53.
//   Q = Y L^{-T}         (the GEMM of the X passes, with L^{-1} packed as the
//                        transposed small operand).
// Two passes (Yamamoto, Nakatsukasa, Yanagisawa, Fukaya 2015: CholeskyQR2) give an orthonormal Q with
// R = R2 R1 having a positive diagonal: the unique thin QR of full-rank Y.
#include "rnmf_common.h"

namespace rnmf {

int gram_splits(int64_t rows, int cus) {
  int s = 2 * cus;
  int maxs = (int)(rows / 64);
  if (maxs < 1) maxs = 1;
  if (s > maxs) s = maxs;
  return s;
}

// Partial Gram over a row range: each thread accumulates 4 x 4 blocks of the
// upper block triangle.  Rows are staged through LDS in FP64.
template <typename T>
__global__ __launch_bounds__(256) void gram_kernel(const T* __restrict__ Y, int64_t rows, int l, int64_t rlen,
                                                   double* __restrict__ gpart) {
  constexpr int RC = 16;
  __shared__ double Ys[RC][LMAX + 4];
  const int lb = (l + 3) / 4;
  const int nblk = lb * (lb + 1) / 2;
  const int64_t rb = (int64_t)blockIdx.x * rlen;
  const int64_t re = (rb + rlen < rows) ? rb + rlen : rows;
  constexpr int MAXB = 3;  // blocks per thread: ceil(528 / 256) for l = 128
  int ba[MAXB], bb[MAXB];
  double acc[MAXB][16];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    int b = threadIdx.x + 256 * q;
    ba[q] = -1;
    bb[q] = -1;
    if (b < nblk) {
      // map linear index to (row block a <= column block c) in row-major upper order
      int a = 0, rem = b;
      while (rem >= lb - a) { rem -= lb - a; ++a; }
      ba[q] = a;
      bb[q] = a + rem;
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[q][e] = 0.0;
  }
  for (int64_t r0 = rb; r0 < re; r0 += RC) {
    for (int e = threadIdx.x; e < RC * (LMAX + 4); e += 256) {
      int rr = e / (LMAX + 4), c = e % (LMAX + 4);
      int64_t r = r0 + rr;
      Ys[rr][c] = (r < re && c < l) ? (double)Y[r * l + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
      if (ba[q] < 0) continue;
      const int a4 = 4 * ba[q], c4 = 4 * bb[q];
      for (int rr = 0; rr < RC; ++rr) {
        double x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) { x[u] = Ys[rr][a4 + u]; y[u] = Ys[rr][c4 + u]; }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[q][u * 4 + v] = fma(x[u], y[v], acc[q][u * 4 + v]);
      }
    }
    __syncthreads();
  }
  double* dst = gpart + (size_t)blockIdx.x * LMAX * LMAX;
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    if (ba[q] < 0) continue;
    const int a4 = 4 * ba[q], c4 = 4 * bb[q];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int a = a4 + u, c = c4 + v;
        if (a < l && c < l) dst[a * LMAX + c] = acc[q][u * 4 + v];
      }
  }
}

// G[a][c] = sum over splits of the partials (upper part), mirrored; fixed order.
__global__ __launch_bounds__(256) void gram_sum_kernel(const double* __restrict__ gpart, int splits, int l,
                                                       double* __restrict__ G) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < l * l; e += gridDim.x * blockDim.x) {
    int a = e / l, c = e % l;
    int lo = a < c ? a : c, hi = a < c ? c : a;
    // a partial holds block (ba, bb) with ba <= bb: entry (lo, hi) lives in the
    // upper block triangle unless lo and hi are in the same 4-block, where
    // both orders were written; read (lo, hi) in either case.
    double s = 0.0;
    for (int p = 0; p < splits; ++p) s += gpart[(size_t)p * LMAX * LMAX + lo * LMAX + hi];
    G[e] = s;
  }
}

hipError_t launch_gram(const void* Y, int dt, int64_t rows, int l, double* gpart, int splits, double* G,
                       hipStream_t s) {
  int64_t rlen = (rows + splits - 1) / splits;
  int rs = ceil_div(rows, rlen);
  if (dt == 0)
    hipLaunchKernelGGL(gram_kernel<double>, dim3(rs), dim3(256), 0, s, (const double*)Y, rows, l, rlen, gpart);
  else
    hipLaunchKernelGGL(gram_kernel<float>, dim3(rs), dim3(256), 0, s, (const float*)Y, rows, l, rlen, gpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int blocks = ceil_div(l * l, 256);
  hipLaunchKernelGGL(gram_sum_kernel, dim3(blocks), dim3(256), 0, s, gpart, rs, l, G);
  return hipGetLastError();
}

// Cholesky of G and the inverse of its factor, one workgroup.  A (LDS, l x l):
// lower triangle = L (strict), upper triangle = L^{-1} transposed (strict),
// with the diagonals of L and L^{-1} in dL and dX.
template <typename OT>
__global__ __launch_bounds__(256) void chol_kernel(const double* __restrict__ G, int l, int64_t rows,
                                                   OT* __restrict__ At, int lp, unsigned* ctl, int mode,
                                                   int allow_shift, unsigned* status) {
  __shared__ double A[LMAX][LMAX + 1];
  __shared__ double dL[LMAX], dX[LMAX];
  __shared__ int fail;
  const int t = threadIdx.x;
  if (mode == 2 && ctl && *ctl == 0u) {
    // no shifted pass happened: this extra pass is an exact copy
    for (int e = t; e < lp * lp; e += 256) At[e] = (OT)((e / lp == e % lp && e / lp < l) ? 1.0 : 0.0);
    return;
  }
  double trace = 0.0;
  for (int i = 0; i < l; ++i) trace += G[i * l + i];
  int shifted = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    __syncthreads();  // every thread has read `fail` of the previous attempt
    shifted = attempt;
    double shift = 0.0;
    if (attempt == 1) {
      const double u = 1.1102230246251565e-16;
      shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * u * trace;
    }
    for (int e = t; e < l * l; e += 256) {
      int i = e / l, j = e % l;
      A[i][j] = G[e] + ((i == j) ? shift : 0.0);
    }
    if (t == 0) fail = 0;
    __syncthreads();
    for (int j = 0; j < l; ++j) {
      double d = A[j][j];
      if (!(d > 0.0) || !(d < INFINITY)) {
        if (t == 0) fail = 1;
      }
      __syncthreads();
      if (fail) break;
      double r = sqrt(d);
      if (t == 0) dL[j] = r;
      for (int i = j + 1 + t; i < l; i += 256) A[i][j] /= r;
      __syncthreads();
      const int w = l - j - 1;  // trailing size
      for (int e = t; e < w * w; e += 256) {
        int i = j + 1 + e / w, p = j + 1 + e % w;
        if (p <= i) A[i][p] -= A[i][j] * A[p][j];
      }
      __syncthreads();
    }
    if (!fail) break;
    if (attempt == 0 && !allow_shift) break;
  }
  if (fail) {
    if (t == 0) atomicOr(status, ST_NOT_SPD);
    // leave the packed operand as zero so that downstream results are inert
    for (int e = t; e < lp * lp; e += 256) At[e] = (OT)0;
    return;
  }
  if (shifted && t == 0) {
    atomicOr(status, ST_SHIFTED);
    if (ctl) atomicOr(ctl, 1u);
  }
  // L^{-1}: row by row, X[i][c] = -(sum_{p=c}^{i-1} L[i][p] X[p][c]) / L[i][i]
  for (int i = 0; i < l; ++i) {
    if (t == 0) dX[i] = 1.0 / dL[i];
    for (int c = t; c < i; c += 256) {
      double s = A[i][c] * dX[c];
      for (int p = c + 1; p < i; ++p) s += A[i][p] * A[c][p];
      A[c][i] = -s / dL[i];
    }
    __syncthreads();
  }
  // At[c][k] = L^{-1}[c][k] for k <= c, zero elsewhere (lp x lp, packed)
  for (int e = t; e < lp * lp; e += 256) {
    int c = e / lp, k = e % lp;
    double v = 0.0;
    if (c < l && k < l) {
      if (k == c) v = dX[c];
      else if (k < c) v = A[k][c];
    }
    At[e] = (OT)v;
  }
}

hipError_t launch_chol(double* G, int l, int64_t rows, void* At, int lp, int cdt, unsigned* ctl, int pass,
                       int allow_shift, unsigned* status, hipStream_t s) {
  if (cdt == 0)
    hipLaunchKernelGGL(chol_kernel<double>, dim3(1), dim3(256), 0, s, G, l, rows, (double*)At, lp, ctl, pass,
                       allow_shift, status);
  else
    hipLaunchKernelGGL(chol_kernel<float>, dim3(1), dim3(256), 0, s, G, l, rows, (float*)At, lp, ctl, pass,
                       allow_shift, status);
  return hipGetLastError();
}

}  // namespace rnmf

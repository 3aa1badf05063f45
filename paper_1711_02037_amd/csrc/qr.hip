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
  int s = cus;
  int maxs = (int)(rows / 64);
  if (maxs < 1) maxs = 1;
  if (s > maxs) s = maxs;
  return s;
}

// Partial Gram over a row range: each thread accumulates 4 x 4 blocks of the
// upper block triangle.  Rows are staged through LDS in FP64.
template <typename T>
__global__ __launch_bounds__(256) void gram_kernel(const T* __restrict__ Y, int64_t rows, int l, int64_t rlen,
                                                   double* __restrict__ gpart, const unsigned* skip) {
  if (skip && *skip == 0u) return;
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

// G[a][c] = sum over splits of the partials (upper part), mirrored.  A block
// handles 32 entries; its eight thread groups add every eighth split, then the
// eight group sums are added in group order (a fixed order).
__global__ __launch_bounds__(256) void gram_sum_kernel(const double* __restrict__ gpart, int splits, int l,
                                                       double* __restrict__ G, const unsigned* skip) {
  if (skip && *skip == 0u) return;
  __shared__ double red[8][32];
  const int el = threadIdx.x & 31, grp = threadIdx.x >> 5;
  const int e = blockIdx.x * 32 + el;
  double s = 0.0;
  if (e < l * l) {
    const int a = e / l, c = e - (e / l) * l;
    const int lo = a < c ? a : c, hi = a < c ? c : a;
    // entry (lo, hi) lies in the upper block triangle that every partial holds
    const double* src = gpart + (size_t)lo * LMAX + hi;
#pragma unroll 8
    for (int p = grp; p < splits; p += 8) s += src[(size_t)p * LMAX * LMAX];
  }
  red[grp][el] = s;
  __syncthreads();
  if (grp == 0 && e < l * l) {
    double t = red[0][el];
#pragma unroll
    for (int g = 1; g < 8; ++g) t += red[g][el];
    G[e] = t;
  }
}

hipError_t launch_gram(const void* Y, int dt, int64_t rows, int l, double* gpart, int splits, double* G,
                       hipStream_t s, const unsigned* skip) {
  int64_t rlen = (rows + splits - 1) / splits;
  int rs = ceil_div(rows, rlen);
  if (dt == 0)
    hipLaunchKernelGGL(gram_kernel<double>, dim3(rs), dim3(256), 0, s, (const double*)Y, rows, l, rlen, gpart, skip);
  else
    hipLaunchKernelGGL(gram_kernel<float>, dim3(rs), dim3(256), 0, s, (const float*)Y, rows, l, rlen, gpart, skip);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_sum_kernel, dim3(ceil_div(l * l, 32)), dim3(256), 0, s, gpart, rs, l, G, skip);
  return hipGetLastError();
}

hipError_t launch_gram_sum(const double* gpart, int splits, int l, double* G, hipStream_t s) {
  hipLaunchKernelGGL(gram_sum_kernel, dim3(ceil_div(l * l, 32)), dim3(256), 0, s, gpart, splits, l, G,
                     (const unsigned*)nullptr);
  return hipGetLastError();
}

// Cholesky of G and the inverse of its factor, one workgroup, FP64 in LDS,
// right-looking in blocks of CB columns.  Storage in A: the strict lower
// triangle holds L, the strict upper triangle holds X = L^{-1} transposed
// (X(i,c) at A[c][i], c < i); dL and dX hold the diagonals.  X starts as I.
// For each block b (rows and columns jb .. jb + nb - 1):
//   1. wave 0 factors the diagonal block (unblocked, no workgroup barrier);
//   2. threads by row solve the panel below, L(i,b) = A(i,b) L(b,b)^{-T},
//      and threads by column finish the block rows of X (forward
//      substitution with L(b,b) on what earlier blocks left in them);
//   3. rank-nb updates of the trailing part of A and of the X rows below.
// Three workgroup barriers per block instead of two per column.
__device__ __forceinline__ void wave_lds_fence() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wave's LDS writes are done
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <typename OT>
__global__ __launch_bounds__(256) void chol_kernel(const double* __restrict__ G, int l, int64_t rows,
                                                   OT* __restrict__ At, int lp, unsigned* ctl, int mode,
                                                   int allow_shift, unsigned* status) {
  constexpr int CB = 8;
  __shared__ double A[LMAX][LMAX + 1];
  __shared__ double dL[LMAX], dX[LMAX];
  __shared__ int fail_s;
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  if (mode == 2 && ctl && *ctl == 0u) return;  // no shifted pass happened: nothing to do
  bool fail = false;
  int shifted = 0;
  for (int attempt = (allow_shift == 2) ? 1 : 0; attempt < 2; ++attempt) {
    shifted = attempt;
    // eight loads in flight per thread (a plain loop waits for each in turn);
    // indices past the end read the last entry, which is not stored
    for (int e0 = t; e0 < l * l; e0 += 256 * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256;
        v[u] = G[e < l * l ? e : l * l - 1];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256;
        if (e < l * l) {
          const int i = e / l, j = e - (e / l) * l;
          A[i][j] = (j <= i) ? v[u] : 0.0;
        }
      }
    }
    for (int i = t; i < l; i += 256) dX[i] = 1.0;
    if (t == 0) fail_s = 0;
    fail = false;
    __syncthreads();
    if (attempt == 1) {
      double trace = 0.0;
      for (int i = 0; i < l; ++i) trace += A[i][i];
      const double u = 1.1102230246251565e-16;
      const double shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * u * trace;
      __syncthreads();
      for (int i = t; i < l; i += 256) A[i][i] += shift;
      __syncthreads();
    }
    for (int jb = 0; jb < l; jb += CB) {
      const int nb = (l - jb < CB) ? l - jb : CB;
      const int je = jb + nb;
      // 1. diagonal block by wave 0
      if (wave == 0) {
        for (int jj = jb; jj < je; ++jj) {
          const double d = A[jj][jj];
          if (!(d > 0.0) || !(d < INFINITY)) {  // uniform across the wave
            if (lane == 0) fail_s = 1;
            break;
          }
          const double r = sqrt(d), ri = 1.0 / r;
          const int ii = jj + 1 + lane;
          if (ii < je) A[ii][jj] *= ri;
          if (lane == 0) dL[jj] = r;
          wave_lds_fence();
          // within-block trailing update: pairs (ii, pp), jj < pp <= ii < je
          const int w = je - jj - 1;
          for (int q = lane; q < w * w; q += 64) {
            const int a = jj + 1 + q / w, b = jj + 1 + q - (q / w) * w;
            if (b <= a) A[a][b] -= A[a][jj] * A[b][jj];
          }
          wave_lds_fence();
        }
      }
      __syncthreads();
      if (fail_s) { fail = true; break; }
      // 2a. panel rows i >= je (threads t < 128): forward substitution with L(b,b)
      if (t < 128) {
        const int i = je + t;
        if (i < l) {
          for (int jj = jb; jj < je; ++jj) {
            double x = A[i][jj];
            for (int p = jb; p < jj; ++p) x -= A[i][p] * A[jj][p];
            A[i][jj] = x / dL[jj];
          }
        }
      } else {
        // 2b. block rows of X, column c < je (threads t >= 128): row jj of X
        // becomes (X(jj,:) - sum_{jb <= p < jj} L(jj,p) X(p,:)) / L(jj,jj)
        const int c = t - 128;
        if (c < je) {
          for (int jj = (c > jb ? c : jb); jj < je; ++jj) {
            double x = (jj == c) ? dX[jj] : A[c][jj];
            for (int p = (c > jb ? c : jb); p < jj; ++p) {
              const double xp = (p == c) ? dX[p] : A[c][p];
              x -= A[jj][p] * xp;
            }
            x /= dL[jj];
            if (jj == c) dX[jj] = x;
            else A[c][jj] = x;
          }
        }
      }
      __syncthreads();
      // 3. rank-nb updates below the block: A(i,p) for je <= p <= i, and X(i,c)
      //    for i >= je, c < je
      const int w = l - je;
      const int na = w * (w + 1) / 2, nx = w * je;
      for (int q = t; q < na + nx; q += 256) {
        if (q < na) {
          // q -> (i, p) with p <= i, row-major over the lower triangle
          int i = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
          while ((i + 1) * (i + 2) / 2 <= q) ++i;
          while (i * (i + 1) / 2 > q) --i;
          const int pp = q - i * (i + 1) / 2;
          const int ri = je + i, rp = je + pp;
          double acc = A[ri][rp];
          for (int cc = jb; cc < je; ++cc) acc -= A[ri][cc] * A[rp][cc];
          A[ri][rp] = acc;
        } else {
          const int e = q - na;
          const int i = je + e / je, c = e - (e / je) * je;
          double acc = A[c][i];
          for (int qq = (c > jb ? c : jb); qq < je; ++qq) {
            const double xq = (qq == c) ? dX[qq] : A[c][qq];
            acc -= A[i][qq] * xq;
          }
          A[c][i] = acc;
        }
      }
      __syncthreads();
    }
    if (!fail) break;
    if (!allow_shift) break;
    __syncthreads();
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
  // At[c][k] = X(c, k) for k <= c, zero elsewhere (lp x lp, packed)
  for (int e = t; e < lp * lp; e += 256) {
    const int c = e / lp, kk = e - (e / lp) * lp;
    double v = 0.0;
    if (c < l && kk < l) {
      if (kk == c) v = dX[c];
      else if (kk < c) v = A[kk][c];
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

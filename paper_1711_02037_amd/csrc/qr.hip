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

// Partial Gram over a row range.  The 4 x 4 blocks of the upper block
// triangle are spread over the 512 threads; when there are fewer blocks than
// threads, NG row groups share each block (rows rg, rg + NG, ...) and their
// partials are added in group order at the end.  Rows are staged through LDS
// in FP64, RC rows at a time, and the next chunk is loaded into registers
// while the current one is used, so the loads of a chunk are in flight
// together instead of one short chunk per round trip.
constexpr int GRAM_NT = 512;
constexpr int GRAM_PF = 24;  // staged values per thread: RC * ldl <= GRAM_NT * GRAM_PF

int gram_ldl(int l) { return ((l + 3) / 4) * 4; }
int gram_rc(int l) {
  int rc = (GRAM_NT * GRAM_PF) / gram_ldl(l);
  if (rc > 128) rc = 128;
  return rc & ~7;
}

template <typename T>
__global__ __launch_bounds__(GRAM_NT) void gram_kernel(const T* __restrict__ Y, int64_t rows, int l, int64_t rlen,
                                                       int RC, double* __restrict__ gpart, const unsigned* skip) {
  if (skip && *skip == 0u) return;
  extern __shared__ __align__(16) double Ys[];  // RC x ldl
  const int t = threadIdx.x;
  const int ldl = ((l + 3) / 4) * 4;
  const int lb = ldl / 4;
  const int nblk = lb * (lb + 1) / 2;
  const int NG = (GRAM_NT / nblk > 1) ? GRAM_NT / nblk : 1;  // row groups per block
  const int64_t rb = (int64_t)blockIdx.x * rlen;
  const int64_t re = (rb + rlen < rows) ? rb + rlen : rows;
  // blocks of this thread: one per row group when NG > 1, else up to two
  int ba[2] = {-1, -1}, bb[2] = {-1, -1};
  const int rg = (NG > 1) ? t / nblk : 0;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int b = (NG > 1) ? ((q == 0 && rg < NG) ? t % nblk : -1) : t + q * GRAM_NT;
    if (b >= 0 && b < nblk) {
      int a = 0, rem = b;
      while (rem >= lb - a) { rem -= lb - a; ++a; }
      ba[q] = a;
      bb[q] = a + rem;
    }
  }
  double acc[2][16];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[q][e] = 0.0;
  // element e of a chunk: row e / ldl, column e % ldl (columns >= l are zero)
  T pf[GRAM_PF];
  auto fetch = [&](int64_t r0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < GRAM_PF; ++u) {
      const int e = t + u * GRAM_NT;
      const int rr = e / ldl, c = e - (e / ldl) * ldl;
      const int64_t r = r0 + rr;
      pf[u] = (rr < RC && r < re && c < l) ? Y[r * l + c] : (T)0;
    }
  };
  fetch(rb);
  for (int64_t r0 = rb; r0 < re; r0 += RC) {
#pragma unroll
    for (int u = 0; u < GRAM_PF; ++u) {
      const int e = t + u * GRAM_NT;
      if (e < RC * ldl) Ys[e] = (double)pf[u];
    }
    __syncthreads();
    if (r0 + RC < re) fetch(r0 + RC);
    const int nr = (re - r0 < RC) ? (int)(re - r0) : RC;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (ba[q] < 0) continue;
      const double* xa = Ys + 4 * ba[q];
      const double* xc = Ys + 4 * bb[q];
      for (int rr = rg; rr < nr; rr += NG) {
        const double2 x01 = *(const double2*)(xa + rr * ldl), x23 = *(const double2*)(xa + rr * ldl + 2);
        const double2 y01 = *(const double2*)(xc + rr * ldl), y23 = *(const double2*)(xc + rr * ldl + 2);
        const double x[4] = {x01.x, x01.y, x23.x, x23.y}, y[4] = {y01.x, y01.y, y23.x, y23.y};
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[q][u * 4 + v] = fma(x[u], y[v], acc[q][u * 4 + v]);
      }
    }
    __syncthreads();
  }
  double* dst = gpart + (size_t)blockIdx.x * LMAX * LMAX;
  if (NG > 1) {
    // fixed-order sum of the row groups' partials through LDS (nblk x 16 doubles)
    for (int gi = 0; gi < NG; ++gi) {
      if (rg == gi && ba[0] >= 0) {
        const int b = t % nblk;
#pragma unroll
        for (int e = 0; e < 16; ++e) Ys[b * 16 + e] = (gi == 0) ? acc[0][e] : Ys[b * 16 + e] + acc[0][e];
      }
      __syncthreads();
    }
    if (t < nblk) {
      int a = 0, rem = t;
      while (rem >= lb - a) { rem -= lb - a; ++a; }
      const int a4 = 4 * a, c4 = 4 * (a + rem);
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int aa = a4 + u, cc = c4 + v;
          if (aa < l && cc < l) dst[aa * LMAX + cc] = Ys[t * 16 + u * 4 + v];
        }
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
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
  const int rc = gram_rc(l);
  // chunk staging, and the NG x nblk x 16 partial sums at the end
  const int lb = gram_ldl(l) / 4, nblk = lb * (lb + 1) / 2;
  size_t lds = (size_t)rc * gram_ldl(l) * 8;
  if ((size_t)nblk * 16 * 8 > lds) lds = (size_t)nblk * 16 * 8;
  if (dt == 0) {
    hipError_t e = hipFuncSetAttribute((const void*)gram_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gram_kernel<double>, dim3(rs), dim3(GRAM_NT), lds, s, (const double*)Y, rows, l, rlen, rc,
                       gpart, skip);
  } else {
    hipError_t e = hipFuncSetAttribute((const void*)gram_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gram_kernel<float>, dim3(rs), dim3(GRAM_NT), lds, s, (const float*)Y, rows, l, rlen, rc,
                       gpart, skip);
  }
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

// Cholesky of G and the inverse of its factor in one workgroup, unblocked and
// right-looking, with every entry held in a register of one thread for the
// whole factorisation.  The entries are the lower triangle of the trailing
// matrix A (initially G) and the lower triangle of Y (initially I), which
// becomes X = L^{-1}.  At step j, with d = A(j,j):
//   A(i,p) -= A(i,j) A(p,j) / d     for j < p <= i  (trailing update)
//   Y(i,c) -= A(i,j) Y(j,c) / d     for c <= j < i  (forward substitution)
// and X(j,c) = Y(j,c) / sqrt(d) once row j of Y is final.  Column j of A and
// row j of Y are the only values a step needs from other threads: their
// owners publish them to LDS (double-buffered) right after their own update
// of the previous step, so each step costs one workgroup barrier.
// Entries are ranked by the last step that updates them (A(i,p): p - 1,
// Y(i,c): i - 1), latest first, and entry rank e goes to thread e mod NT,
// slot e div NT: a thread's slots become idle in order, so its loop over
// slots stops at the first idle one, at about the same slot across a wave.
// With l + 1 entries per key the rank has a closed form, no sort is needed.
constexpr int CHOL_NT = 1024;

template <typename OT, int CHOL_MAXS>  // CHOL_MAXS: slots per thread, >= l (l + 1) / CHOL_NT
__global__ __launch_bounds__(CHOL_NT) void chol_inv_kernel(const double* __restrict__ G, int l, int64_t rows,
                                                         OT* __restrict__ At, int lp, unsigned* ctl, int mode,
                                                         int allow_shift, unsigned* status) {
  __shared__ double vcol[2][LMAX];  // column j of A (rows i >= j)
  __shared__ double yrow[2][LMAX];  // row j of Y (columns c <= j)
  __shared__ double rinv[LMAX];     // 1 / sqrt(d_j)
  __shared__ double trace_s;
  const int t = threadIdx.x;
  if (mode == 2 && ctl && *ctl == 0u) return;  // no shifted pass happened: nothing to do
  const int NE = l * (l + 1);
  // slot code: (key + 1) << 17 | type << 16 | i << 8 | c  (type 0: A, 1: Y); -1: no entry
  int code[CHOL_MAXS];
#pragma unroll
  for (int s2 = 0; s2 < CHOL_MAXS; ++s2) {
    const int e = t + s2 * CHOL_NT;
    code[s2] = -1;
    if (e < NE) {
      const int p = e / (l + 1), r = e - (e / (l + 1)) * (l + 1);
      const int b = l - 1 - p;  // bucket: entries whose last step is b - 1
      if (r < l - b) code[s2] = (b << 17) | (0 << 16) | ((b + r) << 8) | b;          // A(b + r, b)
      else code[s2] = (b << 17) | (1 << 16) | (b << 8) | (r - (l - b));               // Y(b, r - (l - b))
    }
  }
  // zero the parts of the packed operand that no entry writes
  for (int e = t; e < lp * lp; e += CHOL_NT) {
    const int c = e / lp, kk = e - (e / lp) * lp;
    if (!(c < l && kk <= c)) At[e] = (OT)0;
  }
  bool fail = false;
  int shifted = 0;
  double v[CHOL_MAXS];
  for (int attempt = (allow_shift == 2) ? 1 : 0; attempt < 2; ++attempt) {
    shifted = attempt;
    double shift = 0.0;
    if (attempt == 1) {
      if (t == 0) {
        double tr = 0.0;
        for (int i = 0; i < l; ++i) tr += G[i * l + i];
        trace_s = tr;
      }
      __syncthreads();
      const double u = 1.1102230246251565e-16;
      shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * u * trace_s;
    }
#pragma unroll
    for (int s2 = 0; s2 < CHOL_MAXS; ++s2) {
      v[s2] = 0.0;
      const int cd = code[s2];
      if (cd >= 0) {
        const int ty = (cd >> 16) & 1, i = (cd >> 8) & 0xFF, c = cd & 0xFF;
        if (ty == 0) v[s2] = G[i * l + c] + (i == c ? shift : 0.0);
        else v[s2] = (i == c) ? 1.0 : 0.0;
        // publish column 0 of A and row 0 of Y
        if (ty == 0 && c == 0) vcol[0][i] = v[s2];
        if (ty == 1 && i == 0) yrow[0][c] = v[s2];
      }
    }
    __syncthreads();
    fail = false;
    for (int j = 0; j < l; ++j) {
      const int b = j & 1, nb = b ^ 1;
      const double d = vcol[b][j];
      if (!(d > 0.0) || !(d < INFINITY)) { fail = true; break; }  // the same value in every thread
      const double ri = 1.0 / sqrt(d);
      const double dinv = ri * ri;
      if (t == 0) rinv[j] = ri;
#pragma unroll
      for (int s2 = 0; s2 < CHOL_MAXS; ++s2) {
        const int cd = code[s2];
        if ((cd >> 17) <= j) break;  // key < j: this slot and the later ones are done (or empty)
        const int ty = (cd >> 16) & 1, i = (cd >> 8) & 0xFF, c = cd & 0xFF;
        const double a = vcol[b][i] * dinv;
        if (ty == 0) {
          v[s2] = fma(-a, vcol[b][c], v[s2]);  // c > j
          if (c == j + 1) vcol[nb][i] = v[s2];
        } else {
          if (c <= j) v[s2] = fma(-a, yrow[b][c], v[s2]);  // i > j
          if (i == j + 1) yrow[nb][c] = v[s2];
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
    for (int e = t; e < lp * lp; e += CHOL_NT) At[e] = (OT)0;
    return;
  }
  // At[c][k] = X(c, k) = Y(c, k) / sqrt(d_c) for k <= c
#pragma unroll
  for (int s2 = 0; s2 < CHOL_MAXS; ++s2) {
    const int cd = code[s2];
    if (cd >= 0 && ((cd >> 16) & 1)) {
      const int i = (cd >> 8) & 0xFF, c = cd & 0xFF;
      At[(size_t)i * lp + c] = (OT)(v[s2] * rinv[i]);
    }
  }
  if (shifted && t == 0) {
    atomicOr(status, ST_SHIFTED);
    if (ctl) atomicOr(ctl, 1u);
  }
}

hipError_t launch_chol(double* G, int l, int64_t rows, void* At, int lp, int cdt, unsigned* ctl, int pass,
                       int allow_shift, unsigned* status, hipStream_t s) {
  const int ne = l * (l + 1);
#define CHOL_LAUNCH(OT, S)                                                                                  \
  hipLaunchKernelGGL((chol_inv_kernel<OT, S>), dim3(1), dim3(CHOL_NT), 0, s, G, l, rows, (OT*)At, lp, ctl, pass, \
                     allow_shift, status)
  if (cdt == 0) {
    if (ne <= 5 * CHOL_NT) CHOL_LAUNCH(double, 5);
    else if (ne <= 10 * CHOL_NT) CHOL_LAUNCH(double, 10);
    else CHOL_LAUNCH(double, 17);
  } else {
    if (ne <= 5 * CHOL_NT) CHOL_LAUNCH(float, 5);
    else if (ne <= 10 * CHOL_NT) CHOL_LAUNCH(float, 10);
    else CHOL_LAUNCH(float, 17);
  }
#undef CHOL_LAUNCH
  return hipGetLastError();
}

}  // namespace rnmf

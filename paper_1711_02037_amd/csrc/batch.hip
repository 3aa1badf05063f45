// Batched randomized HALS (Algorithm 1 for many independent problems) in one
// persistent launch.  Every workgroup takes whole problems from a work queue
// (an atomic counter over descriptors sorted by estimated cost, largest
// first) and runs the whole method for each on its own:
//   Y = X Omega; Q = qr(Y); q times { Z = X^T Q, Q_n = qr(Z), Y = X Q_n,
//   Q = qr(Y) }; B^T = X^T Q; W~ = Q^T W0; nsweeps compressed HALS sweeps
//   (H rows, then W columns with lift, clip and map-back); ||X - W H||_F.
// Nothing is shared between workgroups but the counter, so no workgroup ever
// waits for another.  QR is Cholesky QR2 (FP64 Gram and Cholesky with the
// inverse fused; a shifted pass and a third pass when the Gram is not
// numerically positive definite).  X passes: 4 x 4 register tiles per thread,
// FP32 products summed in FP32 over a chunk and in FP64 across chunks.
// Sweeps: W~, T, V, S in LDS; Q streamed in 256-row tiles through LDS; H
// rows in FP64 (one wavefront per column of H).
#include "rnmf.h"
#include "rnmf_common.h"

namespace rnmf {

namespace {

constexpr int BT = 256;   // threads per workgroup
constexpr int BLM = 64;   // largest sketch width
constexpr int BKM = 32;   // largest rank
constexpr int NCX = 32;   // X columns per chunk (X A pass)
constexpr int MTZ = 32;   // X rows per chunk (X^T Q pass)
constexpr int GT = 64;    // rows per tile (Grams, init, error)
constexpr int RQT = 256;  // Q rows per tile (W phase)
constexpr int P1 = BLM + 1;

// LDS carving (floats): sweep state, then a scratch region reused by phases.
constexpr int OFF_WT = 0;                        // W~: BLM x BKM
constexpr int OFF_T = OFF_WT + BLM * BKM;        // T: BLM x BKM
constexpr int OFF_V = OFF_T + BLM * BKM;         // V: BKM x BKM
constexpr int OFF_S = OFF_V + BKM * BKM;         // S: BKM x BKM
constexpr int OFF_VEC = OFF_S + BKM * BKM;       // update vector: BLM
constexpr int OFF_WS = OFF_VEC + BLM;            // lifted column tile: RQT
constexpr int OFF_RED = OFF_WS + RQT;            // doubles: 2 x BT (2 floats each)
constexpr int OFF_SCR = OFF_RED + 2 * 2 * BT;    // scratch
// scratch users (floats from OFF_SCR)
constexpr int SCR_CHOL_A = 2 * BLM * P1 + 64;    // after G (doubles) and padding
constexpr int SCR_CHOL_D = SCR_CHOL_A + 2 * BLM * P1;
constexpr int SCR_AT = SCR_CHOL_D + 2 * 2 * BLM + 64;  // L^{-T} as floats: BLM x BLM
constexpr int SCR_FLOATS = SCR_AT + BLM * BLM;
constexpr int LDS_FLOATS = OFF_SCR + SCR_FLOATS;
static_assert(RQT * P1 <= SCR_AT, "Q tile overlaps the factor");
static_assert(4 * BLM <= 2 * BT, "map-back partials fit the reduction buffer");
static_assert(OFF_RED % 2 == 0 && OFF_SCR % 2 == 0 && SCR_CHOL_A % 2 == 0 && SCR_CHOL_D % 2 == 0, "FP64 alignment");
static_assert(NCX * 0 + 256 * (NCX + 1) + NCX * BLM <= SCR_FLOATS, "X A tiles");
static_assert(MTZ * (4 * 64 + 1) + MTZ * BLM <= SCR_FLOATS, "X^T Q tiles");

struct BDesc {
  rnmf_problem p;
  int32_t idx;  // position in the caller's array
  int32_t tc;   // X-pass column groups: 4, 8 or 16 (4 x 4 per thread)
};

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ float clipf(float x) { return x > 0.f ? x : 0.f; }

// Y (m x l) = X (m x n) A (n x l).  Thread (ti, tj): rows ti + tr * i,
// columns 4 tj + u.
__device__ void xa_pass(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n, const float* __restrict__ A,
                        int l, float* __restrict__ Y, int tc, float* scr) {
  const int t = threadIdx.x;
  const int tr = BT / tc, RT = 4 * tr, LC = 4 * tc;
  float* Xs = scr;                      // RT x (NCX + 1)
  float* As = scr + RT * (NCX + 1);     // NCX x LC
  const int ti = t % tr, tj = t / tr;
  for (int64_t r0 = 0; r0 < m; r0 += RT) {
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[i][u] = 0.0;
    for (int64_t c0 = 0; c0 < n; c0 += NCX) {
      for (int e = t; e < RT * NCX; e += BT) {
        const int i = e / NCX, c = e - (e / NCX) * NCX;
        const int64_t r = r0 + i, cc = c0 + c;
        Xs[i * (NCX + 1) + c] = (r < m && cc < n) ? X[r * ldx + cc] : 0.f;
      }
      for (int e = t; e < NCX * LC; e += BT) {
        const int a = e / LC, j = e - (e / LC) * LC;
        As[a * LC + j] = (c0 + a < n && j < l) ? A[(c0 + a) * l + j] : 0.f;
      }
      __syncthreads();
      float s[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) s[i][u] = 0.f;
      for (int c = 0; c < NCX; ++c) {
        float xv[4], av[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) xv[i] = Xs[(ti + tr * i) * (NCX + 1) + c];
#pragma unroll
        for (int u = 0; u < 4; ++u) av[u] = As[c * LC + tj * 4 + u];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int u = 0; u < 4; ++u) s[i][u] = fmaf(xv[i], av[u], s[i][u]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[i][u] += (double)s[i][u];
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = r0 + ti + tr * i;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = tj * 4 + u;
        if (r < m && j < l) Y[r * l + j] = (float)acc[i][u];
      }
    }
  }
  __syncthreads();  // Y is read next by other threads of the workgroup
}

// Z (n x l) = X^T Q, and optionally B = Z^T (l x n).  Thread (ti, tj): Z rows
// (X columns) c0 + ti + tz * i, columns 4 tj + u.
__device__ void xtq_pass(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n, const float* __restrict__ Q,
                         int l, float* __restrict__ Z, float* __restrict__ Bout, int tc, float* scr) {
  const int t = threadIdx.x;
  const int tz = BT / tc, NZ = 4 * tz, LC = 4 * tc;
  float* Xs = scr;                    // MTZ x (NZ + 1)
  float* Qs = scr + MTZ * (NZ + 1);   // MTZ x LC
  const int ti = t % tz, tj = t / tz;
  for (int64_t c0 = 0; c0 < n; c0 += NZ) {
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[i][u] = 0.0;
    for (int64_t r0 = 0; r0 < m; r0 += MTZ) {
      for (int e = t; e < MTZ * NZ; e += BT) {
        const int i = e / NZ, c = e - (e / NZ) * NZ;
        const int64_t r = r0 + i, cc = c0 + c;
        Xs[i * (NZ + 1) + c] = (r < m && cc < n) ? X[r * ldx + cc] : 0.f;
      }
      for (int e = t; e < MTZ * LC; e += BT) {
        const int i = e / LC, j = e - (e / LC) * LC;
        Qs[i * LC + j] = (r0 + i < m && j < l) ? Q[(r0 + i) * l + j] : 0.f;
      }
      __syncthreads();
      float s[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) s[i][u] = 0.f;
      for (int rr = 0; rr < MTZ; ++rr) {
        float xv[4], qv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) xv[i] = Xs[rr * (NZ + 1) + ti + tz * i];
#pragma unroll
        for (int u = 0; u < 4; ++u) qv[u] = Qs[rr * LC + tj * 4 + u];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int u = 0; u < 4; ++u) s[i][u] = fmaf(xv[i], qv[u], s[i][u]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[i][u] += (double)s[i][u];
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t c = c0 + ti + tz * i;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = tj * 4 + u;
        if (c < n && j < l) {
          Z[c * l + j] = (float)acc[i][u];
          if (Bout) Bout[(int64_t)j * n + c] = (float)acc[i][u];
        }
      }
    }
  }
  __syncthreads();  // Z is read next by other threads of the workgroup
}

// Cholesky of G (l x l, in LDS, pitch P1) with the inverse fused, in blocks
// of 8 columns (the scheme of the single-problem factorisation).  A holds L
// in its strict lower triangle and X = L^{-1} transposed in its strict upper
// triangle; dL, dX the diagonals.  Returns 0 (plain), 1 (after the shift) or
// 2 (not positive definite).
__device__ int chol_lds(const double* G, double* A, double* dL, double* dX, int* flag, int l, int64_t rows) {
  constexpr int CB = 8;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  for (int attempt = 0; attempt < 2; ++attempt) {
    for (int e = t; e < l * l; e += BT) {
      const int i = e / l, j = e - (e / l) * l;
      A[i * P1 + j] = (j <= i) ? G[i * P1 + j] : 0.0;
    }
    for (int i = t; i < l; i += BT) dX[i] = 1.0;
    if (t == 0) *flag = 0;
    __syncthreads();
    if (attempt == 1) {
      double trace = 0.0;
      for (int i = 0; i < l; ++i) trace += A[i * P1 + i];
      const double shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * 1.1102230246251565e-16 * trace;
      __syncthreads();
      for (int i = t; i < l; i += BT) A[i * P1 + i] += shift;
      __syncthreads();
    }
    bool fail = false;
    for (int jb = 0; jb < l; jb += CB) {
      const int je = (l - jb < CB) ? l : jb + CB;
      if (wave == 0) {
        for (int jj = jb; jj < je; ++jj) {
          const double d = A[jj * P1 + jj];
          if (!(d > 0.0) || !(d < INFINITY)) {
            if (lane == 0) *flag = 1;
            break;
          }
          const double r = sqrt(d), ri = 1.0 / r;
          const int ii = jj + 1 + lane;
          if (ii < je) A[ii * P1 + jj] *= ri;
          if (lane == 0) dL[jj] = r;
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
          __builtin_amdgcn_s_waitcnt(0xC07F);
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
          const int w = je - jj - 1;
          for (int q = lane; q < w * w; q += 64) {
            const int a = jj + 1 + q / w, b = jj + 1 + q - (q / w) * w;
            if (b <= a) A[a * P1 + b] -= A[a * P1 + jj] * A[b * P1 + jj];
          }
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
          __builtin_amdgcn_s_waitcnt(0xC07F);
          __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
      }
      __syncthreads();
      if (*flag) { fail = true; break; }
      if (t < 128) {
        const int i = je + t;
        if (i < l) {
          for (int jj = jb; jj < je; ++jj) {
            double x = A[i * P1 + jj];
            for (int p = jb; p < jj; ++p) x -= A[i * P1 + p] * A[jj * P1 + p];
            A[i * P1 + jj] = x / dL[jj];
          }
        }
      } else {
        const int c = t - 128;
        if (c < je) {
          const int s0 = c > jb ? c : jb;
          for (int jj = s0; jj < je; ++jj) {
            double x = (jj == c) ? dX[jj] : A[c * P1 + jj];
            for (int p = s0; p < jj; ++p) x -= A[jj * P1 + p] * ((p == c) ? dX[p] : A[c * P1 + p]);
            x /= dL[jj];
            if (jj == c) dX[jj] = x;
            else A[c * P1 + jj] = x;
          }
        }
      }
      __syncthreads();
      const int w = l - je, na = w * (w + 1) / 2, nx = w * je;
      for (int q = t; q < na + nx; q += BT) {
        if (q < na) {
          int i = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
          while ((i + 1) * (i + 2) / 2 <= q) ++i;
          while (i * (i + 1) / 2 > q) --i;
          const int pp = q - i * (i + 1) / 2;
          const int ri = je + i, rp = je + pp;
          double acc = A[ri * P1 + rp];
          for (int cc = jb; cc < je; ++cc) acc -= A[ri * P1 + cc] * A[rp * P1 + cc];
          A[ri * P1 + rp] = acc;
        } else {
          const int e = q - na;
          const int i = je + e / je, c = e - (e / je) * je;
          double acc = A[c * P1 + i];
          for (int qq = (c > jb ? c : jb); qq < je; ++qq) acc -= A[i * P1 + qq] * ((qq == c) ? dX[qq] : A[c * P1 + qq]);
          A[c * P1 + i] = acc;
        }
      }
      __syncthreads();
    }
    if (!fail) return attempt;
    __syncthreads();
  }
  return 2;
}

// One Cholesky QR pass on Y (rows x l, global, in place).  Returns chol_lds's code.
__device__ int cholqr_pass(float* __restrict__ Y, int64_t rows, int l, int tc, float* scr, int* flag) {
  const int t = threadIdx.x;
  double* G = (double*)scr;
  double* A = (double*)(scr + SCR_CHOL_A);
  double* dL = (double*)(scr + SCR_CHOL_D);
  double* dX = dL + BLM;
  float* At = scr + SCR_AT;
  // Gram in FP64: thread (ga, gb) owns entries (ga + 16 i, gb + 16 u)
  {
    float* Ys = scr + SCR_CHOL_A;  // GT x P1 floats; G is written only after the loop
    const int ga = t % 16, gb = t / 16;
    double g[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) g[i][u] = 0.0;
    for (int64_t r0 = 0; r0 < rows; r0 += GT) {
      for (int e = t; e < GT * l; e += BT) {
        const int i = e / l, a = e - (e / l) * l;
        Ys[i * P1 + a] = (r0 + i < rows) ? Y[(r0 + i) * l + a] : 0.f;
      }
      __syncthreads();
      for (int rr = 0; rr < GT; ++rr) {
        double ya[4], yb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int a = ga + 16 * i, b = gb + 16 * i;
          ya[i] = a < l ? (double)Ys[rr * P1 + a] : 0.0;
          yb[i] = b < l ? (double)Ys[rr * P1 + b] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int u = 0; u < 4; ++u) g[i][u] = fma(ya[i], yb[u], g[i][u]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int a = ga + 16 * i, b = gb + 16 * u;
        if (a < l && b < l) G[a * P1 + b] = g[i][u];
      }
    __syncthreads();
  }
  const int code = chol_lds(G, A, dL, dX, flag, l, rows);
  if (code == 2) return 2;
  // At(a, c) = X(c, a) = L^{-1}(c, a) for a <= c, so Q = Y At
  for (int e = t; e < l * l; e += BT) {
    const int a = e / l, c = e - (e / l) * l;
    At[a * BLM + c] = (float)((a == c) ? dX[c] : (a < c ? A[a * P1 + c] : 0.0));
  }
  __syncthreads();
  // Q = Y At in place, RT rows per tile
  {
    const int tr = BT / tc, RT = 4 * tr;
    float* Ys = scr;  // RT x P1 floats, below At
    const int ti = t % tr, tj = t / tr;
    for (int64_t r0 = 0; r0 < rows; r0 += RT) {
      for (int e = t; e < RT * l; e += BT) {
        const int i = e / l, a = e - (e / l) * l;
        Ys[i * P1 + a] = (r0 + i < rows) ? Y[(r0 + i) * l + a] : 0.f;
      }
      __syncthreads();
      float s[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) s[i][u] = 0.f;
      for (int a = 0; a < l; ++a) {
        float yv[4], av[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) yv[i] = Ys[(ti + tr * i) * P1 + a];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = tj * 4 + u;
          av[u] = c < l ? At[a * BLM + c] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int u = 0; u < 4; ++u) s[i][u] = fmaf(yv[i], av[u], s[i][u]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = r0 + ti + tr * i;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = tj * 4 + u;
          if (r < rows && c < l) Y[r * l + c] = s[i][u];
        }
      }
      __syncthreads();
    }
  }
  return code;
}

// Cholesky QR2 (a third pass after a shifted one).  Returns status bits.
__device__ unsigned cholqr2(float* Y, int64_t rows, int l, int tc, float* scr, int* flag) {
  unsigned st = 0;
  bool shifted = false;
  for (int pass = 0; pass < 3; ++pass) {
    if (pass == 2 && !shifted) break;
    const int code = cholqr_pass(Y, rows, l, tc, scr, flag);
    if (code == 2) return ST_NOT_SPD;
    if (code == 1) { shifted = true; st |= ST_SHIFTED; }
  }
  return st;
}

// S = W^T W (k x k, FP64 sums) into Ss (pitch BKM).
__device__ void gram_w(const float* __restrict__ W, int64_t m, int k, float* Ss, float* scr) {
  const int t = threadIdx.x;
  float* Wsh = scr;  // GT x (BKM + 1)
  const int gi = t % 16, gj = t / 16;
  double s[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int64_t r0 = 0; r0 < m; r0 += GT) {
    for (int e = t; e < GT * k; e += BT) {
      const int i = e / k, j = e - (e / k) * k;
      Wsh[i * (BKM + 1) + j] = (r0 + i < m) ? W[(r0 + i) * k + j] : 0.f;
    }
    __syncthreads();
    for (int rr = 0; rr < GT; ++rr) {
      double a[2], b[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int i = gi + 16 * u, j = gj + 16 * u;
        a[u] = i < k ? (double)Wsh[rr * (BKM + 1) + i] : 0.0;
        b[u] = j < k ? (double)Wsh[rr * (BKM + 1) + j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) s[u][v] = fma(a[u], b[v], s[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int i = gi + 16 * u, j = gj + 16 * v;
      if (i < k && j < k) Ss[i * BKM + j] = (float)s[u][v];
    }
  __syncthreads();
}

// W~ = Q^T W (l x k, FP64 sums) into Wts (pitch BKM).
__device__ void init_wt(const float* __restrict__ Q, const float* __restrict__ W, int64_t m, int l, int k, float* Wts,
                        float* scr) {
  const int t = threadIdx.x;
  float* Qsh = scr;                  // GT x P1
  float* Wsh = scr + GT * P1;        // GT x (BKM + 1)
  const int ga = t % 16, gj = t / 16;
  double s[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i) s[i][0] = s[i][1] = 0.0;
  for (int64_t r0 = 0; r0 < m; r0 += GT) {
    for (int e = t; e < GT * l; e += BT) {
      const int i = e / l, a = e - (e / l) * l;
      Qsh[i * P1 + a] = (r0 + i < m) ? Q[(r0 + i) * l + a] : 0.f;
    }
    for (int e = t; e < GT * k; e += BT) {
      const int i = e / k, j = e - (e / k) * k;
      Wsh[i * (BKM + 1) + j] = (r0 + i < m) ? W[(r0 + i) * k + j] : 0.f;
    }
    __syncthreads();
    for (int rr = 0; rr < GT; ++rr) {
      double qa[4], wj[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = ga + 16 * i;
        qa[i] = a < l ? (double)Qsh[rr * P1 + a] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int j = gj + 16 * u;
        wj[u] = j < k ? (double)Wsh[rr * (BKM + 1) + j] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 2; ++u) s[i][u] = fma(qa[i], wj[u], s[i][u]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int a = ga + 16 * i, j = gj + 16 * u;
      if (a < l && j < k) Wts[a * BKM + j] = (float)s[i][u];
    }
  __syncthreads();
}

// Rows of H (Algorithm 1, H rule with S = W^T W), one wavefront per column of
// H: lane j holds H(j, c) and the running gradient (FP64), Gauss-Seidel over j.
__device__ void h_phase(const float* __restrict__ Bt, float* __restrict__ H, int64_t n, int l, int k,
                        const float* Wts, const float* Ss) {
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int jj = lane < k ? lane : 0;
  double rinv = 0.0;
  if (lane < k) {
    const double d = (double)Ss[lane * BKM + lane];
    rinv = d > 0.0 ? 1.0 / d : 0.0;
  }
  for (int64_t c = wave; c < n; c += BT / 64) {
    double h = lane < k ? (double)H[(int64_t)lane * n + c] : 0.0;
    const float bcol = lane < l ? Bt[c * l + lane] : 0.f;
    double g = 0.0;
    for (int a = 0; a < l; ++a) g = fma((double)readlane_f(bcol, a), (double)Wts[a * BKM + jj], g);
    for (int p = 0; p < k; ++p) g = fma(-(double)Ss[p * BKM + jj], readlane_d(h, p), g);
    for (int i = 0; i < k; ++i) {
      const double rd = readlane_d(rinv, i);
      const double hi = readlane_d(h, i), gi = readlane_d(g, i);
      const double hn = (rd > 0.0) ? (double)clipf((float)fma(gi, rd, hi)) : hi;
      const double delta = hn - hi;
      if (lane == i) h = hn;
      g = fma(-(double)Ss[i * BKM + jj], delta, g);
    }
    if (lane < k) H[(int64_t)lane * n + c] = (float)h;
  }
  __syncthreads();
}

// T = B H^T (l x k) and V = H H^T (k x k) over 64-column tiles: FP32 within a
// tile, FP64 across tiles.  Threads 0..127: T entries (ga + 16 i, gj + 8 u);
// threads 128..191: V entries (vi + 8 p, vj + 8 q).
__device__ void tv_phase(const float* __restrict__ Bt, const float* __restrict__ H, int64_t n, int l, int k, float* Ts,
                         float* Vs, float* scr) {
  const int t = threadIdx.x;
  float* Zs = scr;                // 64 (columns) x P1
  float* Hs = scr + 64 * P1;      // BKM x 65
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[i][u] = 0.0;
  for (int64_t c0 = 0; c0 < n; c0 += 64) {
    for (int e = t; e < 64 * l; e += BT) {
      const int c = e / l, a = e - (e / l) * l;
      Zs[c * P1 + a] = (c0 + c < n) ? Bt[(c0 + c) * l + a] : 0.f;
    }
    for (int e = t; e < k * 64; e += BT) {
      const int j = e / 64, c = e - (e / 64) * 64;
      Hs[j * 65 + c] = (c0 + c < n) ? H[(int64_t)j * n + c0 + c] : 0.f;
    }
    __syncthreads();
    float s[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) s[i][u] = 0.f;
    if (t < 128) {
      const int ga = t % 16, gj = t / 16;
      for (int c = 0; c < 64; ++c) {
        float za[4], hj[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int a = ga + 16 * i;
          za[i] = a < l ? Zs[c * P1 + a] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = gj + 8 * u;
          hj[u] = j < k ? Hs[j * 65 + c] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int u = 0; u < 4; ++u) s[i][u] = fmaf(za[i], hj[u], s[i][u]);
      }
    } else if (t < 192) {
      const int v = t - 128, vi = v % 8, vj = v / 8;
      for (int c = 0; c < 64; ++c) {
        float hi[4], hj[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int a = vi + 8 * i, b = vj + 8 * i;
          hi[i] = a < k ? Hs[a * 65 + c] : 0.f;
          hj[i] = b < k ? Hs[b * 65 + c] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int u = 0; u < 4; ++u) s[i][u] = fmaf(hi[i], hj[u], s[i][u]);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[i][u] += (double)s[i][u];
    __syncthreads();
  }
  if (t < 128) {
    const int ga = t % 16, gj = t / 16;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int a = ga + 16 * i, j = gj + 8 * u;
        if (a < l && j < k) Ts[a * BKM + j] = (float)acc[i][u];
      }
  } else if (t < 192) {
    const int v = t - 128, vi = v % 8, vj = v / 8;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int a = vi + 8 * i, b = vj + 8 * u;
        if (a < k && b < k) Vs[a * BKM + b] = (float)acc[i][u];
      }
  }
  __syncthreads();
}

// Columns of W (Algorithm 1): update vector in the compressed space, lift and
// clip on all rows (Q streamed in RQT-row tiles), map back with FP64 sums.
__device__ void w_phase(const float* __restrict__ Q, float* __restrict__ W, int64_t m, int l, int k, float* Wts,
                        const float* Ts, const float* Vs, float* vec, float* ws, double* red, float* scr) {
  const int t = threadIdx.x;
  float* Qs = scr;  // RQT x P1
  const int a = t & 63, g = t >> 6;
  for (int j = 0; j < k; ++j) {
    const float d = Vs[j * BKM + j];
    if (!(d > 0.f)) continue;
    if (t < BLM) {
      float v = 0.f;
      if (t < l) {
        float s0 = Ts[t * BKM + j], s1 = 0.f;
        int i = 0;
        for (; i + 2 <= k; i += 2) {
          s0 = fmaf(-Wts[t * BKM + i], Vs[i * BKM + j], s0);
          s1 = fmaf(-Wts[t * BKM + i + 1], Vs[(i + 1) * BKM + j], s1);
        }
        for (; i < k; ++i) s0 = fmaf(-Wts[t * BKM + i], Vs[i * BKM + j], s0);
        v = Wts[t * BKM + j] + (s0 + s1) / d;
      }
      vec[t] = v;
    }
    __syncthreads();
    double macc = 0.0;
    for (int64_t r0 = 0; r0 < m; r0 += RQT) {
      for (int e = t; e < RQT * l; e += BT) {
        const int i = e / l, c = e - (e / l) * l;
        Qs[i * P1 + c] = (r0 + i < m) ? Q[(r0 + i) * l + c] : 0.f;
      }
      __syncthreads();
      {
        float u0 = 0.f, u1 = 0.f;
        int c = 0;
        for (; c + 2 <= l; c += 2) {
          u0 = fmaf(Qs[t * P1 + c], vec[c], u0);
          u1 = fmaf(Qs[t * P1 + c + 1], vec[c + 1], u1);
        }
        for (; c < l; ++c) u0 = fmaf(Qs[t * P1 + c], vec[c], u0);
        const float w = (r0 + t < m) ? clipf(u0 + u1) : 0.f;
        ws[t] = w;
        if (r0 + t < m) W[(r0 + t) * k + j] = w;
      }
      __syncthreads();
      if (a < l) {
        float p = 0.f;
        for (int rr = g; rr < RQT; rr += 4) p = fmaf(Qs[rr * P1 + a], ws[rr], p);
        macc += (double)p;
      }
      __syncthreads();
    }
    red[g * BLM + a] = macc;
    __syncthreads();
    if (t < l) Wts[t * BKM + j] = (float)((red[t] + red[BLM + t]) + (red[2 * BLM + t] + red[3 * BLM + t]));
    __syncthreads();
  }
}

// ||X - W H||_F^2 and ||X||_F^2 (FP64 sums, fixed order) for thread 0.
__device__ void rel_err(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n, const float* __restrict__ W,
                        const float* __restrict__ H, int k, float* scr, double* red, double* out) {
  const int t = threadIdx.x;
  float* Xs = scr;                      // 64 x 65
  float* Wsh = scr + 64 * 65;           // 64 x (BKM + 1)
  float* Hs = Wsh + 64 * (BKM + 1);     // BKM x 65
  const int ti = t % 16, tj = t / 16;
  double e2 = 0.0, x2 = 0.0;
  for (int64_t r0 = 0; r0 < m; r0 += 64) {
    for (int e = t; e < 64 * k; e += BT) {
      const int i = e / k, j = e - (e / k) * k;
      Wsh[i * (BKM + 1) + j] = (r0 + i < m) ? W[(r0 + i) * k + j] : 0.f;
    }
    for (int64_t c0 = 0; c0 < n; c0 += 64) {
      for (int e = t; e < 64 * 64; e += BT) {
        const int i = e / 64, c = e - (e / 64) * 64;
        Xs[i * 65 + c] = (r0 + i < m && c0 + c < n) ? X[(r0 + i) * ldx + c0 + c] : 0.f;
      }
      for (int e = t; e < k * 64; e += BT) {
        const int j = e / 64, c = e - (e / 64) * 64;
        Hs[j * 65 + c] = (c0 + c < n) ? H[(int64_t)j * n + c0 + c] : 0.f;
      }
      __syncthreads();
      float s[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) s[i][u] = 0.f;
      for (int j = 0; j < k; ++j) {
        float wv[4], hv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) wv[i] = Wsh[(ti + 16 * i) * (BKM + 1) + j];
#pragma unroll
        for (int u = 0; u < 4; ++u) hv[u] = Hs[j * 65 + tj + 16 * u];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int u = 0; u < 4; ++u) s[i][u] = fmaf(wv[i], hv[u], s[i][u]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double x = (double)Xs[(ti + 16 * i) * 65 + tj + 16 * u];
          const double d = x - (double)s[i][u];
          e2 += d * d;
          x2 += x * x;
        }
      __syncthreads();
    }
  }
  red[t] = e2;
  red[BT + t] = x2;
  __syncthreads();
  for (int o = BT / 2; o > 0; o >>= 1) {
    if (t < o) {
      red[t] += red[t + o];
      red[BT + t] += red[BT + t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = red[0];
    out[1] = red[BT];
  }
  __syncthreads();
}

__global__ __launch_bounds__(BT) void batch_kernel(const BDesc* __restrict__ descs, int nprob, int q, int nsweeps,
                                                   unsigned* counter, double* err, unsigned* status) {
  extern __shared__ float lds[];
  __shared__ int cur, flag;
  const int t = threadIdx.x;
  float* Wts = lds + OFF_WT;
  float* Ts = lds + OFF_T;
  float* Vs = lds + OFF_V;
  float* Ss = lds + OFF_S;
  float* vec = lds + OFF_VEC;
  float* ws = lds + OFF_WS;
  double* red = (double*)(lds + OFF_RED);
  float* scr = lds + OFF_SCR;
  while (true) {
    if (t == 0) cur = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int pi = cur;
    __syncthreads();  // every thread has read cur before thread 0 writes it again
    if (pi >= nprob) break;
    const BDesc& d = descs[pi];
    const rnmf_problem& p = d.p;
    const int64_t m = p.m, n = p.n, ldx = p.ldx;
    const int k = p.k, l = p.l, tc = d.tc;
    unsigned st = 0;
    // range finder (Algorithm 1, steps 3-8)
    xa_pass(p.X, ldx, m, n, p.Omega, l, p.Q, tc, scr);
    st |= cholqr2(p.Q, m, l, tc, scr, &flag);
    for (int it = 0; it < q && !(st & ST_NOT_SPD); ++it) {
      xtq_pass(p.X, ldx, m, n, p.Q, l, p.Z, nullptr, tc, scr);
      st |= cholqr2(p.Z, n, l, tc, scr, &flag);
      if (st & ST_NOT_SPD) break;
      xa_pass(p.X, ldx, m, n, p.Z, l, p.Q, tc, scr);
      st |= cholqr2(p.Q, m, l, tc, scr, &flag);
    }
    if (!(st & ST_NOT_SPD)) {
      // compression (step 9): B^T into Z for the sweeps, B for the caller
      xtq_pass(p.X, ldx, m, n, p.Q, l, p.Z, p.B, tc, scr);
      // initialisation (step 10)
      for (int64_t e = t; e < m * k; e += BT) p.W[e] = p.W0[e];
      for (int64_t e = t; e < (int64_t)k * n; e += BT) p.H[e] = p.H0[e];
      __syncthreads();
      init_wt(p.Q, p.W, m, l, k, Wts, scr);
      // sweeps (steps 11-22): H rows, then W columns
      for (int s = 0; s < nsweeps; ++s) {
        gram_w(p.W, m, k, Ss, scr);
        h_phase(p.Z, p.H, n, l, k, Wts, Ss);
        tv_phase(p.Z, p.H, n, l, k, Ts, Vs, scr);
        w_phase(p.Q, p.W, m, l, k, Wts, Ts, Vs, vec, ws, red, scr);
      }
      double out[2];
      rel_err(p.X, ldx, m, n, p.W, p.H, k, scr, red, out);
      if (t == 0) {
        err[2 * d.idx] = out[0];
        err[2 * d.idx + 1] = out[1];
      }
    } else if (t == 0) {
      err[2 * d.idx] = 0.0;
      err[2 * d.idx + 1] = 0.0;
    }
    if (t == 0) status[d.idx] = st;
    __syncthreads();
  }
}

}  // namespace

size_t batch_desc_bytes() { return sizeof(BDesc); }
size_t batch_lds_bytes() { return (size_t)LDS_FLOATS * sizeof(float); }

// descs: device array of nprob descriptors (BDesc layout, filled by the host
// from batch_fill_desc).
void batch_fill_desc(void* dst, const rnmf_problem& p, int idx, int tc) {
  BDesc d;
  d.p = p;
  d.idx = idx;
  d.tc = tc;
  *(BDesc*)dst = d;
}

hipError_t launch_batch(const void* descs, int nprob, int q, int nsweeps, unsigned* counter, double* err,
                        unsigned* status, int grid, hipStream_t s) {
  const size_t lds = batch_lds_bytes();
  hipError_t e = hipFuncSetAttribute((const void*)batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if ((e = launch_fill_u32(counter, 1, 0u, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(batch_kernel, dim3((unsigned)grid), dim3(BT), lds, s, (const BDesc*)descs, nprob, q, nsweeps,
                     counter, err, status);
  return hipGetLastError();
}

}  // namespace rnmf

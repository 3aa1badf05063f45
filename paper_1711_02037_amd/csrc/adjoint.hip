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

// ---- W columns in reverse: one persistent, cooperative launch per sweep ----
//
// The k column steps form a chain: step j needs gWt(:, j) after the updates of
// the steps j' > j.  Per step, with the W column's adjoint g = gW(:, j) +
// Q gWt(:, j) masked by W'(:, j) > 0:
//   gu = Q^T (masked g)                               (a sum over the m rows)
//   gWt(:, p) -= V_pj / V_jj gu  (p != j),  gWt(:, j) <- 0,  gW(:, j) <- 0.
// Workgroup g owns a slab of rows of Q and W and a replicated copy of gWt and V
// in LDS.  The l-vector gu is all-reduced in two levels over a GR x GC grid of
// workgroups: workgroup (i, c) adds the slab partials of its row i (GC
// sources), publishes that row sum, and adds the row sums of the workgroups
// (0..GR-1, c).  Every sum runs in a fixed order, so every workgroup holds the
// same gu to the last bit.  Exchange words are 64 bits, a 32-bit half of a
// double and the 32-bit epoch of the step, written and read with agent-scope
// relaxed atomics: each word carries its own readiness.  Slots alternate
// between two buffers by the parity of the step: a workgroup can run at most
// one step ahead of a reader of its slot, because its next-but-one partial
// needs that reader's next partial.  gu of every step goes to GU(:, j); the
// adjoints of T and V follow from GU in ad_wpost.  Every wait is bounded:
// past the spin limit the workgroup records ST_TIMEOUT and leaves the chain.
constexpr int WR_NT = 512;
constexpr long WR_SPIN = 1L << 22;

__device__ __forceinline__ u64 xld(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void xst(u64* p, unsigned payload, unsigned e) {
  __hip_atomic_store(p, ((u64)e << 32) | (u64)payload, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void publish(u64* slot, int a, double v, unsigned e) {
  const u64 b = (u64)__double_as_longlong(v);
  xst(slot + 2 * a, (unsigned)b, e);
  xst(slot + 2 * a + 1, (unsigned)(b >> 32), e);
}

// Sum, in source order, of element a over nsrc slots (slot s at base + s *
// stride), waiting for epoch e.  Eight sources are loaded together and only
// their stale words are polled again (sixteen at once measured slower).
__device__ double gather(const u64* base, size_t stride, int nsrc, int a, unsigned e, bool& ok) {
  constexpr int WIN = 8;
  double sum = 0.0;
  for (int s0 = 0; s0 < nsrc; s0 += WIN) {
    const int cnt = (nsrc - s0) < WIN ? (nsrc - s0) : WIN;
    u64 w[WIN][2];
#pragma unroll
    for (int q = 0; q < WIN; ++q)
      if (q < cnt) {
        w[q][0] = xld(base + (size_t)(s0 + q) * stride + 2 * a);
        w[q][1] = xld(base + (size_t)(s0 + q) * stride + 2 * a + 1);
      }
    long spins = 0;
    while (true) {
      bool all = true;
#pragma unroll
      for (int q = 0; q < WIN; ++q)
        if (q < cnt) all = all && (unsigned)(w[q][0] >> 32) == e && (unsigned)(w[q][1] >> 32) == e;
      if (all) break;
      if (!ok || ++spins > WR_SPIN) { ok = false; break; }
#pragma unroll
      for (int q = 0; q < WIN; ++q)
        if (q < cnt) {
          if ((unsigned)(w[q][0] >> 32) != e) w[q][0] = xld(base + (size_t)(s0 + q) * stride + 2 * a);
          if ((unsigned)(w[q][1] >> 32) != e) w[q][1] = xld(base + (size_t)(s0 + q) * stride + 2 * a + 1);
        }
    }
#pragma unroll
    for (int q = 0; q < WIN; ++q)
      if (q < cnt) sum += __longlong_as_double((long long)(((u64)(unsigned)w[q][1] << 32) | (u64)(unsigned)w[q][0]));
  }
  return sum;
}

// Workgroup-wide staging st(e, ld(e)) for e in [0, count): each thread takes
// eight elements per round and issues all their loads before any store, so
// the loads' latencies overlap (a plain loop waits for each load in turn).
// Loads past the end read the last element (always in bounds) and are not
// stored.
template <int NT, typename Load, typename Store>
__device__ __forceinline__ void stage(int count, Load ld_, Store st_) {
  for (int e0 = threadIdx.x; e0 < count; e0 += NT * 8) {
    decltype(ld_(0)) v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NT;
      v[u] = ld_(e < count ? e : count - 1);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NT;
      if (e < count) st_(e, v[u]);
    }
  }
}

// Workgroup barrier for LDS data only: waits for this wavefront's LDS
// operations but not for its outstanding global stores and exchange words,
// which __syncthreads() would drain.
__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt = 63, expcnt = 7, lgkmcnt = 0
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// q . w over l entries with four partial sums, added pairwise.
template <typename T>
__device__ __forceinline__ double row_dot(const T* q, const double* w, int l) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int a = 0;
  for (; a + 4 <= l; a += 4) {
    s0 = fma((double)q[a], w[a], s0);
    s1 = fma((double)q[a + 1], w[a + 1], s1);
    s2 = fma((double)q[a + 2], w[a + 2], s2);
    s3 = fma((double)q[a + 3], w[a + 3], s3);
  }
  for (; a < l; ++a) s0 = fma((double)q[a], w[a], s0);
  return (s0 + s1) + (s2 + s3);
}

// sum over rows i = first, first + step, ... < count of q[i * ld] z[i], with
// two partial sums (rows taken alternately), added at the end.
template <typename T>
__device__ __forceinline__ double col_dot(const T* q, int64_t ld, const double* z, int first, int count, int step) {
  double s0 = 0.0, s1 = 0.0;
  int i = first;
#pragma unroll 2
  for (; i + step < count; i += 2 * step) {
    s0 = fma((double)q[(int64_t)i * ld], z[i], s0);
    s1 = fma((double)q[(int64_t)(i + step) * ld], z[i + step], s1);
  }
  if (i < count) s0 = fma((double)q[(int64_t)i * ld], z[i], s0);
  return s0 + s1;
}

template <typename T>
struct WrevArgs {
  const T* Q; const T* Wn; const double* V;
  double* gW; double* gWt; double* GU;
  int64_t m; int l, k;
  int G, GR, GC; int64_t rows_per;
  u64* part; u64* rows;  // exchange slots: [2][G][2 * LMAX] words each
  unsigned* status;
};

// RES: the workgroup's slab of Q stays in LDS for the whole launch (row
// stride l | 1, odd, so that a wavefront reading one entry per row hits
// distinct banks); otherwise the slab is read from global memory at every
// step, WR_NT rows at a time.  Dot products keep four partial sums (two in
// the transposed product) so that their loads overlap.
template <typename T, bool RES>
__global__ __launch_bounds__(WR_NT) void ad_wrev_kernel(WrevArgs<T> A) {
  extern __shared__ double lds[];
  const int l = A.l, k = A.k, t = threadIdx.x, g = blockIdx.x;
  const int lq = l | 1;
  const int64_t r0 = (int64_t)g * A.rows_per;
  const int64_t r1 = (r0 + A.rows_per) < A.m ? (r0 + A.rows_per) : A.m;
  const int nrows = r1 > r0 ? (int)(r1 - r0) : 0;
  const int zn = RES ? (int)A.rows_per : WR_NT;
  double* sgwt = lds;               // l x k
  double* gu = sgwt + l * k;        // LMAX
  double* vj = gu + LMAX;           // KMAX: V(:, j) / V_jj
  double* wj = vj + KMAX;           // LMAX: gWt(:, j)
  double* red = wj + LMAX;          // WR_NT
  double* zs = red + WR_NT;         // zn
  T* tile = (T*)(zs + zn);          // RES: nrows x lq
  __shared__ int sok;
  stage<WR_NT>(l * k, [&](int e) { return A.gWt[e]; }, [&](int e, double v) { sgwt[e] = v; });
  const T* qsl = A.Q + r0 * l;
  if (RES)
    stage<WR_NT>(nrows * l, [&](int e) { return qsl[e]; },
                 [&](int e, T v) {
                   const int i = e / l, a = e - (e / l) * l;
                   tile[i * lq + a] = v;
                 });
  if (t == 0) sok = 1;
  // one slab row per thread: the next step's gW and W' entries are loaded
  // ahead, while the exchange of the current step is in flight
  const bool one = RES && nrows <= WR_NT;
  const bool own = one && t < nrows;
  const int64_t rt = r0 + t;
  int pj = k - 1;
  double pg = own ? A.gW[rt * k + pj] : 0.0;
  T pw = own ? A.Wn[rt * k + pj] : (T)0;
  // the update of gWt: thread t takes column up = t % k of rows ua, ua + ur, ...
  const int ur = WR_NT / k, ua0 = t / k, up = t - (t / k) * k;
  __syncthreads();
  const int gi = g / A.GC, gc = g - (g / A.GC) * A.GC;
  const int groups = WR_NT / l, grp = t / l, ta = t - (t / l) * l;
  const size_t slotw = 2 * LMAX;
  bool ok = true;
  unsigned step = 0;
  for (int j = k - 1; j >= 0; --j) {
    const double d = A.V[j * k + j];
    if (!(d > 0.0)) continue;  // skipped in the forward: adjoints pass through
    const unsigned e = ++step;
    const int par = (int)(e & 1u);
    if (t < k) vj[t] = A.V[t * k + j] / d;
    if (t < l) wj[t] = sgwt[t * k + j];
    lds_barrier();
    // slab partial of Q^T (masked g)
    double s = 0.0;
    if (one) {
      if (own) {
        if (pj != j) {
          pg = A.gW[rt * k + j];
          pw = A.Wn[rt * k + j];
        }
        const double gg = pg + row_dot(tile + t * lq, wj, l);
        zs[t] = ((double)pw > 0.0) ? gg : 0.0;
        A.gW[rt * k + j] = 0.0;
        if (j > 0) {
          pj = j - 1;
          pg = A.gW[rt * k + pj];
          pw = A.Wn[rt * k + pj];
        }
      }
      lds_barrier();
      if (grp < groups) s = col_dot(tile + ta, (int64_t)lq, zs, grp, nrows, groups);
    } else if (RES) {
      for (int i = t; i < nrows; i += WR_NT) {
        const int64_t r = r0 + i;
        const double gg = A.gW[r * k + j] + row_dot(tile + i * lq, wj, l);
        zs[i] = ((double)A.Wn[r * k + j] > 0.0) ? gg : 0.0;
        A.gW[r * k + j] = 0.0;
      }
      lds_barrier();
      if (grp < groups) s = col_dot(tile + ta, (int64_t)lq, zs, grp, nrows, groups);
    } else {
      for (int64_t c0 = r0; c0 < r1; c0 += WR_NT) {
        const int64_t r = c0 + t;
        double z = 0.0;
        if (r < r1) {
          const double gg = A.gW[r * k + j] + row_dot(A.Q + r * l, wj, l);
          z = ((double)A.Wn[r * k + j] > 0.0) ? gg : 0.0;
          A.gW[r * k + j] = 0.0;
        }
        zs[t] = z;
        lds_barrier();
        const int cnt = (int)((r1 - c0) < WR_NT ? (r1 - c0) : WR_NT);
        if (grp < groups) s += col_dot(A.Q + c0 * l + ta, (int64_t)l, zs, grp, cnt, groups);
        lds_barrier();
      }
    }
    red[t] = s;
    lds_barrier();
    if (t < l) {
      double v = 0.0;
      for (int g2 = 0; g2 < groups; ++g2) v += red[g2 * l + t];
      publish(A.part + ((size_t)par * A.G + g) * slotw, t, v, e);
      const double rs = gather(A.part + ((size_t)par * A.G + (size_t)gi * A.GC) * slotw, slotw, A.GC, t, e, ok);
      publish(A.rows + ((size_t)par * A.G + g) * slotw, t, rs, e);
      gu[t] = gather(A.rows + ((size_t)par * A.G + gc) * slotw, (size_t)A.GC * slotw, A.GR, t, e, ok);
      if (!ok) sok = 0;
    }
    lds_barrier();
    if (!sok) break;
    if (g == 0 && t < l) A.GU[t * k + j] = gu[t];
    if (ua0 < ur) {
      const double f = vj[up];
      for (int a = ua0; a < l; a += ur) {
        if (up == j) sgwt[a * k + up] = 0.0;
        else sgwt[a * k + up] -= f * gu[a];
      }
    }
    lds_barrier();
  }
  if (!sok) {
    if (t == 0) atomicOr(A.status, ST_TIMEOUT);
    return;
  }
  if (g == 0)
    for (int e2 = t; e2 < l * k; e2 += WR_NT) A.gWt[e2] = sgwt[e2];
}

// Adjoints of T and V from the steps' gu (one workgroup per column j):
// gT(:, j) = gu_j / V_jj;  gV(p, j) = -Wtc_p . gu_j / V_jj (p != j) and
// gV(j, j) = -u_j . gu_j / V_jj, with the update vector
// u_j = (T(:, j) - sum_{p != j} V_pj Wtc_p) / V_jj and Wtc_p = Wt'(:, p) for
// p < j, Wt(:, p) for p > j.  All zero for a skipped column.
template <typename T>
__global__ __launch_bounds__(256) void ad_wpost(const T* __restrict__ Wto, const T* __restrict__ Wtn,
                                                const double* __restrict__ Tm, const double* __restrict__ V,
                                                const double* __restrict__ GU, int l, int k, double* __restrict__ gT,
                                                double* __restrict__ gV) {
  const int j = blockIdx.x, t = threadIdx.x;
  const double d = V[j * k + j];
  __shared__ double gu[LMAX], u[LMAX];
  if (!(d > 0.0)) {
    if (t < l) gT[t * k + j] = 0.0;
    if (t < k) gV[t * k + j] = 0.0;
    return;
  }
  if (t < l) {
    gu[t] = GU[t * k + j];
    double num = Tm[t * k + j];
    for (int p = 0; p < k; ++p)
      if (p != j) num -= V[p * k + j] * (p < j ? (double)Wtn[t * k + p] : (double)Wto[t * k + p]);
    u[t] = num / d;
    gT[t * k + j] = gu[t] / d;
  }
  __syncthreads();
  if (t < k) {
    double v = 0.0;
    for (int a = 0; a < l; ++a) {
      const double w = (t == j) ? u[a] : (t < j ? (double)Wtn[a * k + t] : (double)Wto[a * k + t]);
      v = fma(w, gu[a], v);
    }
    gV[t * k + j] = -v / d;
  }
}

// H rows in reverse.  The columns of H are independent.  A workgroup takes
// 32 columns and stages their adjoints gH and the signs of H' in LDS; each
// wavefront runs 8 columns side by side (independent chains, so their
// latencies overlap), lane p holding gh_p of each.  For j = k..1 with
// S_jj > 0: ga = gh_j if H'(j, c) > 0 else 0; gA(j, c) = ga; gh_j <- 0;
// gh_p -= S_pj (ga / S_jj) (p != j).  gH(:, c) <- gh (the adjoint of the old H).
constexpr int HR_COLS = 32;
constexpr int HR_CPW = 8;  // columns per wavefront

template <typename T>
__global__ __launch_bounds__(256) void ad_hrows(const T* __restrict__ Hn, const double* __restrict__ S, int64_t n,
                                                int k, double* __restrict__ gH, double* __restrict__ gA) {
  __shared__ double Ss[KMAX * KMAX];
  __shared__ double tg[KMAX][HR_COLS + 1];
  __shared__ double ta[KMAX][HR_COLS + 1];
  __shared__ unsigned char tm[KMAX][HR_COLS];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * HR_COLS;
  stage<256>(k * k, [&](int e) { return S[e]; }, [&](int e, double v) { Ss[e] = v; });
  // columns past n read column n - 1 and are stored as zero adjoints and signs
  auto gidx = [&](int e) {
    const int p = (int)(e / HR_COLS), cc = (int)(e - (e / HR_COLS) * HR_COLS);
    const int64_t c = (c0 + cc) < n ? (c0 + cc) : (n - 1);
    return (int64_t)p * n + c;
  };
  auto inb = [&](int e) { return c0 + (e - (e / HR_COLS) * HR_COLS) < n; };
  stage<256>(k * HR_COLS, [&](int e) { return gH[gidx(e)]; },
             [&](int e, double v) { tg[e / HR_COLS][e - (e / HR_COLS) * HR_COLS] = inb(e) ? v : 0.0; });
  stage<256>(k * HR_COLS, [&](int e) { return Hn[gidx(e)]; },
             [&](int e, T v) {
               tm[e / HR_COLS][e - (e / HR_COLS) * HR_COLS] = (inb(e) && (double)v > 0.0) ? 1 : 0;
             });
  __syncthreads();
  const int cb = wv * HR_CPW;
  double gh[HR_CPW];
#pragma unroll
  for (int q = 0; q < HR_CPW; ++q) gh[q] = lane < k ? tg[lane][cb + q] : 0.0;
  for (int j = k - 1; j >= 0; --j) {
    const double d = Ss[j * k + j];
    if (!(d > 0.0)) {
      if (lane < HR_CPW) ta[j][cb + lane] = 0.0;
      continue;
    }
    const double spj = lane < k ? Ss[lane * k + j] : 0.0;
    double ga[HR_CPW];
#pragma unroll
    for (int q = 0; q < HR_CPW; ++q) {
      const double ghj = __shfl(gh[q], j, 64);
      ga[q] = tm[j][cb + q] ? ghj : 0.0;
    }
#pragma unroll
    for (int q = 0; q < HR_CPW; ++q) {
      const double f = ga[q] / d;
      gh[q] = (lane == j) ? 0.0 : fma(-spj, f, gh[q]);
    }
    if (lane < HR_CPW) {
      double v = ga[0];
#pragma unroll
      for (int q = 1; q < HR_CPW; ++q) v = (lane == q) ? ga[q] : v;
      ta[j][cb + lane] = v;
    }
  }
#pragma unroll
  for (int q = 0; q < HR_CPW; ++q)
    if (lane < k) tg[lane][cb + q] = gh[q];
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

// C (M x K, FP64) += A (M x K) Mp, with Mp the K x K factor zero-padded to
// 64 x 64 (FP64), K <= 64.  Lane j of a wavefront holds column j of Mp in
// registers; the workgroup stages 128 rows of A in LDS (row stride K | 1),
// and each wavefront runs 32 of them, two at a time, every lane reading the
// same A entries.  Row i of C is then read and written by the lanes in one
// contiguous piece.  A is finite (the states of a forward that the sweep
// kernel has checked), so a zero entry of Mp cancels any entry of A.
template <typename T>
__global__ __launch_bounds__(256) void ad_rowmat(const T* __restrict__ A, const double* __restrict__ Mp, int64_t M,
                                                 int K, double* __restrict__ C) {
  __shared__ T At[128 * (KMAX + 1)];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, kq = K | 1;
  const int64_t i0 = (int64_t)blockIdx.x * 128;
  const int rows = (M - i0) < 128 ? (int)(M - i0) : 128;
  const T* ab = A + i0 * K;
  for (int e = t; e < 128 * (KMAX + 1); e += 256) At[e] = (T)0;
  __syncthreads();
  stage<256>(rows * K, [&](int e) { return ab[e]; },
             [&](int e, T v) {
               const int r = e / K, q = e - (e / K) * K;
               At[r * kq + q] = v;
             });
  double mc[KMAX];
#pragma unroll
  for (int q = 0; q < KMAX; ++q) mc[q] = Mp[q * KMAX + lane];
  __syncthreads();
  // the sum runs over all 64 entries: reads past a row's K entries stay in
  // the tile (at most 127 * 65 + 63) and meet the zero rows q >= K of Mp;
  // they are the next row's (finite) entries or the zeros written above
  for (int r = w * 32; r < w * 32 + 32 && r < rows; r += 2) {
    const bool two = r + 1 < rows;
    const T* a0 = At + r * kq;
    const T* a1 = At + (two ? r + 1 : r) * kq;
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      s0 = fma((double)a0[q], mc[q], s0);
      s1 = fma((double)a1[q], mc[q], s1);
    }
    if (lane < K) {
      C[(i0 + r) * K + lane] += s0;
      if (two) C[(i0 + r + 1) * K + lane] += s1;
    }
  }
}

// Mp (64 x 64) = G + G^T for the k x k G, zero outside the leading k x k.
__global__ __launch_bounds__(256) void ad_symm_pad(const double* __restrict__ G, int k, double* __restrict__ Mp) {
  for (int e = threadIdx.x; e < KMAX * KMAX; e += 256) {
    const int i = e / KMAX, j = e - (e / KMAX) * KMAX;
    Mp[e] = (i < k && j < k) ? G[i * k + j] + G[j * k + i] : 0.0;
  }
}

// Partial Gram W^T W (k <= 64) of a slab of rows, FP64: the workgroup stages
// 128 rows at a time in LDS and thread (bi, bj) accumulates the 4 x 4 block
// (4 bi.., 4 bj..) over them, rows in order.  Written in the partial layout
// of the Cholesky QR Gram (entry (a, b), a <= b, at a * LMAX + b of the
// workgroup's slot), summed by launch_gram_sum.
template <typename T>
__global__ __launch_bounds__(256) void ad_wgram(const T* __restrict__ W, int64_t m, int k, int64_t rows_per,
                                                double* __restrict__ part) {
  __shared__ double tile[128 * (KMAX + 1)];
  const int t = threadIdx.x, bi = t >> 4, bj = t & 15;
  constexpr int KP = KMAX + 1;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = (r0 + rows_per) < m ? (r0 + rows_per) : m;
  const bool live = 4 * bi < k && 4 * bj < k && bi <= bj;
  double acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
  for (int64_t c0 = r0; c0 < r1; c0 += 128) {
    const int cnt = (r1 - c0) < 128 ? (int)(r1 - c0) : 128;
    // the chunk's rows are contiguous: element e is row e / k, column e % k
    const T* wb = W + c0 * k;
    stage<256>(cnt * k, [&](int e) { return wb[e]; },
               [&](int e, T v) {
                 const int r = e / k, q = e - (e / k) * k;
                 tile[r * KP + q] = (double)v;
               });
    for (int e = t; e < cnt * (KMAX - k); e += 256) {
      const int r = e / (KMAX - k), q = k + (e - (e / (KMAX - k)) * (KMAX - k));
      tile[r * KP + q] = 0.0;
    }
    __syncthreads();
    if (live)
      for (int r = 0; r < cnt; ++r) {
        const double* row = tile + r * KP;
        double u[4], v[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
          u[x] = row[4 * bi + x];
          v[x] = row[4 * bj + x];
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 4; ++y) acc[x][y] = fma(u[x], v[y], acc[x][y]);
      }
    __syncthreads();
  }
  if (live) {
    double* dst = part + (size_t)blockIdx.x * LMAX * LMAX;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int a = 4 * bi + x, b = 4 * bj + y;
        if (a < k && b < k && a <= b) dst[a * LMAX + b] = acc[x][y];
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

WrevShape plan_wrev(int64_t m, int l, int k, int dt, int cus, int max_lds) {
  WrevShape sh;
  int64_t target = (m + 63) / 64;
  if (target > cus) target = cus;
  if (target < 1) target = 1;
  sh.GC = target < 16 ? (int)target : 16;
  sh.GR = (int)(target / sh.GC);
  sh.G = sh.GR * sh.GC;
  sh.rows_per = (m + sh.G - 1) / sh.G;
  const size_t fixed = ((size_t)l * k + 2 * LMAX + KMAX + WR_NT) * sizeof(double);
  const size_t res = fixed + (size_t)sh.rows_per * sizeof(double) +
                     (size_t)sh.rows_per * (size_t)(l | 1) * (dt == 0 ? 8 : 4);
  sh.res = res + 256 <= (size_t)max_lds;  // 256 bytes left for the static flag
  sh.lds_bytes = sh.res ? res : fixed + (size_t)WR_NT * sizeof(double);
  return sh;
}

size_t wrev_ws_words(const WrevShape& sh) { return (size_t)2 * 2 * sh.G * 2 * LMAX; }

hipError_t ad_wrev(const WrevShape& sh, const void* Q, const void* Wn, const double* V, int64_t m, int l, int k,
                   double* gW, double* gWt, double* GU, u64* xbuf, unsigned* status, int dt, hipStream_t s) {
  if (l < 1 || l > LMAX || k < 1 || k > KMAX) return hipErrorInvalidValue;
  const size_t words = wrev_ws_words(sh);
  hipError_t e = launch_fill_u32((unsigned*)xbuf, words * 2, 0u, s);
  if (e != hipSuccess) return e;
  u64* part = xbuf;
  u64* rows = xbuf + words / 2;
#define WREV(TT)                                                                                       \
  {                                                                                                    \
    WrevArgs<TT> a;                                                                                    \
    a.Q = (const TT*)Q; a.Wn = (const TT*)Wn; a.V = V; a.gW = gW; a.gWt = gWt; a.GU = GU;              \
    a.m = m; a.l = l; a.k = k; a.G = sh.G; a.GR = sh.GR; a.GC = sh.GC; a.rows_per = sh.rows_per;      \
    a.part = part; a.rows = rows; a.status = status;                                                   \
    void* args[] = {&a};                                                                               \
    const void* fn = sh.res ? (const void*)ad_wrev_kernel<TT, true> : (const void*)ad_wrev_kernel<TT, false>; \
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds_bytes);        \
    if (e != hipSuccess) return e;                                                                     \
    return hipLaunchCooperativeKernel(fn, dim3(sh.G), dim3(WR_NT), args, (unsigned)sh.lds_bytes, s);   \
  }
  if (dt == 0) WREV(double) else WREV(float)
#undef WREV
}

hipError_t ad_wpost_run(const void* Wto, const void* Wtn, const double* Tm, const double* V, const double* GU,
                        int l, int k, double* gT, double* gV, int dt, hipStream_t s) {
  if (dt == 0)
    hipLaunchKernelGGL(ad_wpost<double>, dim3(k), dim3(256), 0, s, (const double*)Wto, (const double*)Wtn, Tm, V,
                       GU, l, k, gT, gV);
  else
    hipLaunchKernelGGL(ad_wpost<float>, dim3(k), dim3(256), 0, s, (const float*)Wto, (const float*)Wtn, Tm, V, GU,
                       l, k, gT, gV);
  return hipGetLastError();
}

template <typename T>
static hipError_t hrows_t(const T* Hn, const double* S, int64_t n, int k, double* gH, double* gA, hipStream_t s) {
  const dim3 g((unsigned)((n + HR_COLS - 1) / HR_COLS));
  hipLaunchKernelGGL(ad_hrows<T>, g, dim3(256), 0, s, Hn, S, n, k, gH, gA);
  return hipGetLastError();
}

int ad_wgram_splits(int64_t m, int cus) {
  int64_t g = (m + 127) / 128;
  if (g > cus) g = cus;
  return (int)(g < 1 ? 1 : g);
}

hipError_t ad_wgram_run(const void* W, int64_t m, int k, double* part, int splits, double* S, int dt, hipStream_t s) {
  if (k < 1 || k > KMAX) return hipErrorInvalidValue;
  const int64_t rows_per = (m + splits - 1) / splits;
  const int used = (int)((m + rows_per - 1) / rows_per);
  if (dt == 0) hipLaunchKernelGGL(ad_wgram<double>, dim3(used), dim3(256), 0, s, (const double*)W, m, k, rows_per, part);
  else hipLaunchKernelGGL(ad_wgram<float>, dim3(used), dim3(256), 0, s, (const float*)W, m, k, rows_per, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gram_sum(part, used, k, S, s);
}

hipError_t ad_symm_pad_run(const double* G, int k, double* Mp, hipStream_t s) {
  hipLaunchKernelGGL(ad_symm_pad, dim3(1), dim3(256), 0, s, G, k, Mp);
  return hipGetLastError();
}

hipError_t ad_rowmat_run(const void* A, const double* Mm, int64_t M, int K, double* C, int dt, hipStream_t s) {
  if (K < 1 || K > KMAX) return hipErrorInvalidValue;
  const dim3 g((unsigned)((M + 127) / 128));
  if (dt == 0) hipLaunchKernelGGL(ad_rowmat<double>, g, dim3(256), 0, s, (const double*)A, Mm, M, K, C);
  else hipLaunchKernelGGL(ad_rowmat<float>, g, dim3(256), 0, s, (const float*)A, Mm, M, K, C);
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

}  // namespace rnmf

// Compressed HALS sweeps (Sec. 3.2; Algorithm 1) as one persistent,
// cooperative kernel: every sweep of the call runs inside a single launch.
//
// Work split (G workgroups, one per compute unit, arranged as GR x GC):
//   - rows of Q and W are split into G slabs (the Q slab lives in LDS);
//   - columns of B and H are split into G slabs;
//   - the small replicated state (W~: l x k, T: l x k, V and S: k x k) is held
//     by every workgroup in LDS.
// H phase: each workgroup updates its own columns of H (rows in order j = 1..k,
//   Gauss-Seidel; one wavefront per column, lane j holds H(j,c)); no exchange.
// T = B H^T and V = H H^T: slab partials, then one device-wide all-reduce.
// W phase: for each column j in order: the l-vector update of W~(:,j), the
//   lift W(:,j) = max(0, Q W~(:,j)) on the local rows, the local partial of
//   Q^T W(:,j), and one device-wide all-reduce of that l-vector.
// S = W^T W: slab partials (register-blocked), one all-reduce.
//
// Device-wide all-reduce: partials are written as 64-bit words (32-bit payload
// | 32-bit epoch) with agent-scope relaxed atomic stores, so every word carries
// its own readiness and no separate barrier is needed.  Workgroup (i, j) first
// adds the partials of its row i, publishes the row sum, then adds the row
// sums of its column j.  Every sum runs in a fixed order, so every workgroup
// obtains bit-identical results and the kernel is deterministic.  Large
// vectors (T, V, S) use reduce-scatter by slice, a column reduce, then an
// all-gather.  Every wait is bounded: past the spin limit the kernel records
// RNMF_ERR_DEVICE_TIMEOUT and all workgroups leave.
#include "rnmf_common.h"

namespace rnmf {

namespace {

constexpr int NTH = 512;        // threads per workgroup
constexpr int LPS = LMAX;       // values per small-exchange slot
constexpr int MAXSRC = 16;      // GC, GR <= 16
constexpr long SPIN_LIMIT = 1L << 22;

__device__ __forceinline__ u64 ld_ll(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_ll(u64* p, unsigned payload, unsigned e) {
  __hip_atomic_store(p, ((u64)e << 32) | (u64)payload, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename V> struct Words { static constexpr int n = sizeof(V) / 4; };

template <typename V>
__device__ __forceinline__ unsigned payload_of(V v, int h) {
  if constexpr (sizeof(V) == 4) return __float_as_uint(v);
  else {
    u64 b = __double_as_longlong(v);
    return h ? (unsigned)(b >> 32) : (unsigned)b;
  }
}
template <typename V>
__device__ __forceinline__ V value_of(const u64* w) {
  if constexpr (sizeof(V) == 4) return __uint_as_float((unsigned)w[0]);
  else return __longlong_as_double((long long)(((u64)(unsigned)w[1] << 32) | (u64)(unsigned)w[0]));
}

template <typename V>
__device__ __forceinline__ void put(u64* base, int elem, V v, unsigned e) {
  constexpr int W = Words<V>::n;
#pragma unroll
  for (int h = 0; h < W; ++h) st_ll(base + (size_t)elem * W + h, payload_of<V>(v, h), e);
}

// Fixed-order sum over nsrc slots (slot s at base + s * stride) of element
// `elem`, waiting for epoch e on every word.  All loads are issued first.
template <typename V>
__device__ __forceinline__ V gather_sum(const u64* base, size_t stride, int nsrc, int elem, unsigned e,
                                        bool& ok) {
  constexpr int W = Words<V>::n;
  u64 w[MAXSRC][W];
#pragma unroll
  for (int s = 0; s < MAXSRC; ++s)
    if (s < nsrc)
#pragma unroll
      for (int h = 0; h < W; ++h) w[s][h] = ld_ll(base + s * stride + (size_t)elem * W + h);
  V sum = (V)0;
#pragma unroll
  for (int s = 0; s < MAXSRC; ++s) {
    if (s < nsrc) {
#pragma unroll
      for (int h = 0; h < W; ++h) {
        long spins = 0;
        while ((unsigned)(w[s][h] >> 32) != e) {
          if (!ok || ++spins > SPIN_LIMIT) { ok = false; break; }
          w[s][h] = ld_ll(base + s * stride + (size_t)elem * W + h);
        }
      }
      sum += value_of<V>(w[s]);
    }
  }
  return sum;
}

template <typename T>
struct SweepArgs {
  const T* Q; const T* B; T* W; T* Wt; T* H;
  int m, n, l, k;
  int nsweeps; double tol; int gram_mode, order;
  int G, GR, GC, rows_per, cols_per, rows_lds, lq, cb;
  int red2_elems;
  u64 *xs_part, *xs_row, *xb_part, *xb_row, *xb_fin;
  size_t lpw, cbw, csw;  // words per slot
  double* stats; unsigned* status;
};

struct Xch {
  int g, i, j;
  unsigned seq;
  unsigned small_use, big_use;
};

// All-reduce of c <= LPS values of type V held in LDS `vals` (in/out).
template <typename T, typename V>
__device__ bool allreduce_small(const SweepArgs<T>& a, Xch& x, V* vals, int c, int* abort_flag) {
  constexpr int W = Words<V>::n;
  const int t = threadIdx.x;
  const unsigned e = ++x.seq;
  const unsigned par = (x.small_use++) & 1u;
  const size_t slot = (size_t)LPS * 2;  // words per slot (room for doubles)
  u64* P = a.xs_part + ((size_t)par * a.G) * slot;
  u64* RS = a.xs_row + ((size_t)par * a.G) * slot;
  bool ok = true;
  V r = (V)0;
  if (t < c) {
    put<V>(P + (size_t)x.g * slot, t, vals[t], e);
    r = gather_sum<V>(P + (size_t)x.i * a.GC * slot, slot, a.GC, t, e, ok);
    if (a.GR > 1) {
      put<V>(RS + (size_t)x.g * slot, t, r, e);
      r = gather_sum<V>(RS + (size_t)x.j * slot, (size_t)a.GC * slot, a.GR, t, e, ok);
    }
  }
  (void)W;
  if (!ok) *abort_flag = 1;
  __syncthreads();
  if (t < c) vals[t] = r;
  __syncthreads();
  return *abort_flag == 0;
}

// All-reduce of c <= cb values of type T held in LDS `vals` (in/out).
template <typename T>
__device__ bool allreduce_big(const SweepArgs<T>& a, Xch& x, T* vals, int c, int* abort_flag) {
  const int t = threadIdx.x;
  const unsigned e = ++x.seq;
  const unsigned par = (x.big_use++) & 1u;
  const int cs = (c + a.GC - 1) / a.GC;
  const int s0 = x.j * cs;
  const int s1 = (s0 + cs < c) ? s0 + cs : c;
  u64* P = a.xb_part;
  u64* RS = a.xb_row + (size_t)par * a.G * a.csw;
  u64* FN = a.xb_fin + (size_t)par * a.G * a.csw;
  bool ok = true;
  for (int v = t; v < c; v += NTH) put<T>(P + (size_t)x.g * a.cbw, v, vals[v], e);
  __syncthreads();
  for (int v = s0 + t; v < s1; v += NTH) {
    T r = gather_sum<T>(P + (size_t)x.i * a.GC * a.cbw, a.cbw, a.GC, v, e, ok);
    if (a.GR > 1) put<T>(RS + (size_t)x.g * a.csw, v - s0, r, e);
    else put<T>(FN + (size_t)x.g * a.csw, v - s0, r, e);
  }
  if (a.GR > 1) {
    for (int v = s0 + t; v < s1; v += NTH) {
      T r = gather_sum<T>(RS + (size_t)x.j * a.csw, (size_t)a.GC * a.csw, a.GR, v - s0, e, ok);
      put<T>(FN + (size_t)x.g * a.csw, v - s0, r, e);
    }
  }
  for (int v = t; v < c; v += NTH) {
    int jj = v / cs;
    vals[v] = gather_sum<T>(FN + ((size_t)x.i * a.GC + jj) * a.csw, 0, 1, v - jj * cs, e, ok);
  }
  if (!ok) *abort_flag = 1;
  __syncthreads();
  return *abort_flag == 0;
}

template <typename T>
__device__ __forceinline__ T readlane(T v, int lane) {
  if constexpr (sizeof(T) == 4) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
  } else {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(unsigned)b, lane);
    int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
    return __longlong_as_double((long long)(((u64)(unsigned)hi << 32) | (u64)(unsigned)lo));
  }
}

template <typename T> __device__ __forceinline__ T clip0(T x) { return x > (T)0 ? x : (T)0; }

template <typename T>
__device__ __forceinline__ const T* qrow(const SweepArgs<T>& a, const T* Qs, int r0, int rr) {
  return rr < a.rows_lds ? Qs + (size_t)rr * a.lq : a.Q + (size_t)(r0 + rr) * a.l;
}

// Local Gram of the workgroup's rows of W (k x k, full), into dst (LDS).
// Rows are staged in LDS chunks; each thread owns 4 x 4 blocks of the upper
// block triangle, mirrored on the way out.
template <typename T>
__device__ void local_wgram(const SweepArgs<T>& a, int r0, int nr, T* stage, T* dst) {
  const int k = a.k, t = threadIdx.x;
  const int kb = (k + 3) / 4;
  const int nblk = kb * (kb + 1) / 2;  // <= 136 for k <= 64
  int ba = -1, bb = -1;
  if (t < nblk) {
    int q = 0, rem = t;
    while (rem >= kb - q) { rem -= kb - q; ++q; }
    ba = q;
    bb = q + rem;
  }
  double acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0.0;
  constexpr int RC = 32;
  const int kp = 4 * kb;
  for (int c0 = 0; c0 < nr; c0 += RC) {
    __syncthreads();
    for (int e = t; e < RC * kp; e += NTH) {
      int rr = e / kp, cc = e % kp;
      stage[e] = (c0 + rr < nr && cc < k) ? a.W[(size_t)(r0 + c0 + rr) * k + cc] : (T)0;
    }
    __syncthreads();
    if (ba >= 0) {
      const int rmax = (nr - c0 < RC) ? nr - c0 : RC;
      for (int rr = 0; rr < rmax; ++rr) {
        double u[4], w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          u[q] = (double)stage[rr * kp + 4 * ba + q];
          w[q] = (double)stage[rr * kp + 4 * bb + q];
        }
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[p * 4 + q] = fma(u[p], w[q], acc[p * 4 + q]);
      }
    }
  }
  __syncthreads();
  if (ba >= 0) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        int r = 4 * ba + p, c = 4 * bb + q;
        if (r < k && c < k) {
          dst[r * k + c] = (T)acc[p * 4 + q];
          if (ba != bb) dst[c * k + r] = (T)acc[p * 4 + q];
        }
      }
  }
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(NTH) void sweep_kernel(SweepArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = (T*)smem_raw;
  __shared__ int abort_flag;
  __shared__ double pg_buf[2];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int l = a.l, k = a.k;
  const int g = blockIdx.x;
  Xch x;
  x.g = g; x.i = g / a.GC; x.j = g % a.GC; x.seq = 0; x.small_use = 0; x.big_use = 0;

  const int r0 = g * a.rows_per;
  int nr = a.m - r0; if (nr > a.rows_per) nr = a.rows_per; if (nr < 0) nr = 0;
  const int c0 = g * a.cols_per;
  int nc = a.n - c0; if (nc > a.cols_per) nc = a.cols_per; if (nc < 0) nc = 0;
  const int rows_in_lds = nr < a.rows_lds ? nr : a.rows_lds;

  // LDS carve-up (red2 first so that it is 8-byte aligned for the FP64 sums)
  T* red2 = smem;                                 // scratch: backward partials, W staging, pg sums
  T* Wts = red2 + a.red2_elems;                   // l x k
  T* U = Wts + (size_t)l * k;                     // [T: l x k | V: k x k | S: k x k]
  T* Tm = U;
  T* Vm = U + (size_t)l * k;
  T* Sm = Vm + (size_t)k * k;
  T* vec = Sm + (size_t)k * k;                    // LPS
  T* wcol = vec + LPS;                            // rows_per
  T* Qs = wcol + a.rows_per;                      // rows_lds x lq

  if (t == 0) abort_flag = 0;
  for (size_t e = t; e < (size_t)rows_in_lds * l; e += NTH) {
    int rr = (int)(e / l), c = (int)(e % l);
    Qs[(size_t)rr * a.lq + c] = a.Q[(size_t)(r0 + rr) * l + c];
  }
  for (int e = t; e < l * k; e += NTH) Wts[e] = a.Wt[e];
  __syncthreads();

  const bool need_S = (a.gram_mode != 1) || (a.tol > 0.0);
  const bool need_pg = a.tol > 0.0;
  const int RG = (NTH / l < 16) ? NTH / l : 16;

  // --- building blocks ------------------------------------------------------
  auto s_exchange = [&]() -> bool {
    local_wgram<T>(a, r0, nr, red2, Sm);
    return allreduce_big<T>(a, x, Sm, k * k, &abort_flag);
  };

  auto tv_exchange = [&]() -> bool {
    // T = B H^T (l x k) and V = H H^T (k x k) over this workgroup's columns
    for (int e = t; e < l * k + k * k; e += NTH) {
      double s = 0.0;
      if (e < l * k) {
        int aa = e / k, jj = e % k;
        const T* brow = a.B + (size_t)aa * a.n + c0;
        const T* hrow = a.H + (size_t)jj * a.n + c0;
        for (int c = 0; c < nc; ++c) s = fma((double)brow[c], (double)hrow[c], s);
      } else {
        int f = e - l * k, ii = f / k, jj = f % k;
        const T* h1 = a.H + (size_t)ii * a.n + c0;
        const T* h2 = a.H + (size_t)jj * a.n + c0;
        for (int c = 0; c < nc; ++c) s = fma((double)h1[c], (double)h2[c], s);
      }
      U[e] = (T)s;
    }
    __syncthreads();
    return allreduce_big<T>(a, x, U, l * k + k * k, &abort_flag);
  };

  auto h_phase = [&]() {
    // numerator Gram and scale
    const T* Snum = Sm;
    const T* Ssc = Sm;
    if (a.gram_mode != 0) {
      // W~^T W~ into the T region (T is recomputed after the H phase)
      for (int e = t; e < k * k; e += NTH) {
        int ii = e / k, jj = e % k;
        T s = (T)0;
        for (int aa = 0; aa < l; ++aa) s = fma(Wts[aa * k + ii], Wts[aa * k + jj], s);
        Tm[e] = s;
      }
      __syncthreads();
      Snum = Tm;
      if (a.gram_mode == 1) Ssc = Tm;
    }
    // FP64 arithmetic: the update cancels R against H^T S, and S is the Gram
    // of a nonnegative factor, so its rounding is amplified.
    for (int cc = wave; cc < nc; cc += NTH / 64) {
      const int c = c0 + cc;
      const int jj = lane < k ? lane : 0;
      double R = 0.0;
      for (int aa = 0; aa < l; ++aa) R = fma((double)a.B[(size_t)aa * a.n + c], (double)Wts[aa * k + jj], R);
      double h = (double)a.H[(size_t)jj * a.n + c];
      double gsum = R;
      for (int ii = 0; ii < k; ++ii) gsum = fma(-(double)Snum[ii * k + jj], readlane<double>(h, ii), gsum);
      for (int ii = 0; ii < k; ++ii) {
        const double d = (double)Ssc[ii * k + ii];
        if (d > 0.0) {
          const double hi = readlane<double>(h, ii);
          const double gi = readlane<double>(gsum, ii);
          // the new row is rounded to the storage type before it is used
          const double hn = (double)clip0<T>((T)(hi + gi / d));
          const double delta = hn - hi;
          if (lane == ii) h = hn;
          gsum = fma(-(double)Snum[ii * k + jj], delta, gsum);
        }
      }
      if (lane < k) a.H[(size_t)lane * a.n + c] = (T)h;
    }
    __syncthreads();
  };

  auto w_phase = [&]() -> bool {
    for (int jj = 0; jj < k; ++jj) {
      const T d = Vm[jj * k + jj];
      if (!(d > (T)0)) continue;
      if (t < l) {
        T s = Tm[t * k + jj];
        for (int ii = 0; ii < k; ++ii) s = fma(-Wts[t * k + ii], Vm[ii * k + jj], s);
        vec[t] = Wts[t * k + jj] + s / d;
      }
      __syncthreads();
      for (int rr = t; rr < nr; rr += NTH) {
        const T* q = qrow<T>(a, Qs, r0, rr);
        T u = (T)0;
        for (int aa = 0; aa < l; ++aa) u = fma(q[aa], vec[aa], u);
        const T w = clip0<T>(u);
        wcol[rr] = w;
        a.W[(size_t)(r0 + rr) * k + jj] = w;
      }
      __syncthreads();
      if (t < RG * l) {
        const int aa = t % l, rg = t / l;
        T s = (T)0;
        for (int rr = rg; rr < nr; rr += RG) s = fma(qrow<T>(a, Qs, r0, rr)[aa], wcol[rr], s);
        red2[rg * LPS + aa] = s;
      }
      __syncthreads();
      if (t < l) {
        T s = (T)0;
        for (int rg = 0; rg < RG; ++rg) s += red2[rg * LPS + t];
        vec[t] = s;
      }
      __syncthreads();
      if (!allreduce_small<T, T>(a, x, vec, l, &abort_flag)) return false;
      if (t < l) {
        Wts[t * k + jj] = vec[t];
        if (g == 0 && !(vec[t] == vec[t])) atomicOr(a.status, ST_NONFINITE_SWEEP);
      }
      __syncthreads();
    }
    return true;
  };

  // projected gradient norm^2 on X^ = Q B (factor 2 dropped)
  auto pgrad = [&](double& out) -> bool {
    double s = 0.0;
    for (int e = t; e < nr * k; e += NTH) {
      int rr = e / k, cc = e % k;
      const T* wr = a.W + (size_t)(r0 + rr) * k;
      const T* q = qrow<T>(a, Qs, r0, rr);
      T gval = (T)0;
      for (int ii = 0; ii < k; ++ii) gval = fma(wr[ii], Vm[ii * k + cc], gval);
      for (int aa = 0; aa < l; ++aa) gval = fma(-q[aa], Tm[aa * k + cc], gval);
      T p = wr[cc] > (T)0 ? gval : (gval < (T)0 ? gval : (T)0);
      s += (double)p * (double)p;
    }
    for (int e = t; e < nc * k; e += NTH) {
      int cc = e / k, jj = e % k;
      const int c = c0 + cc;
      T gval = (T)0;
      for (int ii = 0; ii < k; ++ii) gval = fma(Sm[jj * k + ii], a.H[(size_t)ii * a.n + c], gval);
      for (int aa = 0; aa < l; ++aa) gval = fma(-Wts[aa * k + jj], a.B[(size_t)aa * a.n + c], gval);
      T hv = a.H[(size_t)jj * a.n + c];
      T p = hv > (T)0 ? gval : (gval < (T)0 ? gval : (T)0);
      s += (double)p * (double)p;
    }
    // workgroup reduction in fixed order through LDS (red2 as doubles)
    double* rd = (double*)red2;
    __syncthreads();
    rd[t] = s;
    __syncthreads();
    for (int o = NTH / 2; o > 0; o >>= 1) {
      if (t < o) rd[t] += rd[t + o];
      __syncthreads();
    }
    if (t == 0) pg_buf[0] = rd[0];
    __syncthreads();
    if (!allreduce_small<T, double>(a, x, pg_buf, 1, &abort_flag)) return false;
    out = pg_buf[0];
    return true;
  };

  // --- prologue -------------------------------------------------------------
  bool alive = true;
  double pg0 = 0.0, pg = 0.0;
  int done = 0;
  if (need_S) alive = s_exchange();
  if (alive && (need_pg || a.order == 1)) alive = tv_exchange();
  if (alive && need_pg) { alive = pgrad(pg0); pg = pg0; }

  // --- sweeps ---------------------------------------------------------------
  for (int sw = 0; alive && sw < a.nsweeps; ++sw) {
    if (a.order == 0) {
      h_phase();
      alive = tv_exchange();
      if (alive) alive = w_phase();
      if (alive && need_S) alive = s_exchange();
    } else {
      alive = w_phase();
      if (alive && need_S) alive = s_exchange();
      if (alive) { h_phase(); alive = tv_exchange(); }
    }
    if (!alive) break;
    ++done;
    if (need_pg) {
      alive = pgrad(pg);
      if (!alive) break;
      if (pg < a.tol * pg0) break;
    }
  }

  if (!alive) {
    if (t == 0) atomicOr(a.status, ST_TIMEOUT);
    return;
  }
  if (g == 0) {
    for (int e = t; e < l * k; e += NTH) a.Wt[e] = Wts[e];
    if (t == 0 && a.stats) {
      a.stats[0] = (double)done;
      a.stats[1] = pg0;
      a.stats[2] = pg;
    }
  }
}

}  // namespace

SweepShape plan_sweep(int64_t m, int64_t n, int l, int k, int dt, const Dev& d) {
  SweepShape sh;
  int gmax = d.cus < 256 ? d.cus : 256;
  int G = 1;
  while (G * 2 <= gmax && ceil_div(m, G * 2) >= 16) G *= 2;
  sh.G = G;
  sh.GC = G < 16 ? G : 16;
  sh.GR = G / sh.GC;
  sh.rows_per = ceil_div(m, G);
  sh.cols_per = ceil_div(n, G);
  sh.cb = l * k + k * k;
  sh.nt = NTH;
  const size_t es = dt == 0 ? 8 : 4;
  const int lq = l | 1;
  // Wts + U + vec + wcol + red2 (also the W staging area: 32 x 4*ceil(k/4))
  size_t red2 = 16 * (size_t)LPS;
  size_t stage = 32 * (size_t)(4 * ((k + 3) / 4));
  if (stage > red2) red2 = stage;
  if ((size_t)NTH * 8 / es > red2) red2 = (size_t)NTH * 8 / es;  // pg reduction as doubles
  red2 = round_up(red2, 4);
  sh.red2_elems = (int)red2;
  size_t fixed = ((size_t)l * k + (size_t)l * k + 2 * (size_t)k * k + LPS + sh.rows_per + red2) * es;
  size_t budget = (size_t)d.max_lds - 1024;  // static shared + alignment slack
  size_t qrows = fixed < budget ? (budget - fixed) / ((size_t)lq * es) : 0;
  sh.rows_lds = (int)((size_t)sh.rows_per < qrows ? sh.rows_per : qrows);
  sh.lds_bytes = fixed + (size_t)sh.rows_lds * lq * es;
  return sh;
}

size_t sweep_ws_words(const SweepShape& sh, int l) {
  (void)l;
  size_t slot = (size_t)LPS * 2;
  size_t cs = (size_t)((sh.cb + sh.GC - 1) / sh.GC) * 2;
  return 2 * 2 * (size_t)sh.G * slot + (size_t)sh.G * (size_t)sh.cb * 2 + 2 * 2 * (size_t)sh.G * cs;
}

hipError_t launch_sweep(const SweepShape& sh, int dt, const void* Q, const void* B, void* W, void* Wt, void* H,
                        int64_t m, int64_t n, int l, int k, int nsweeps, double tol, int gram_mode, int order,
                        u64* xbuf, double* stats, unsigned* status, hipStream_t s) {
  size_t words = sweep_ws_words(sh, l);
  hipError_t e = launch_fill_u32((unsigned*)xbuf, words * 2, 0u, s);
  if (e != hipSuccess) return e;
  size_t slot = (size_t)LPS * 2;
  size_t cbw = (size_t)sh.cb * 2;
  size_t csw = (size_t)((sh.cb + sh.GC - 1) / sh.GC) * 2;
  u64* p = xbuf;
  u64* xs_part = p; p += 2 * (size_t)sh.G * slot;
  u64* xs_row = p; p += 2 * (size_t)sh.G * slot;
  u64* xb_part = p; p += (size_t)sh.G * cbw;
  u64* xb_row = p; p += 2 * (size_t)sh.G * csw;
  u64* xb_fin = p;
#define FILL_ARGS(TT)                                                                            \
  SweepArgs<TT> a;                                                                               \
  a.Q = (const TT*)Q; a.B = (const TT*)B; a.W = (TT*)W; a.Wt = (TT*)Wt; a.H = (TT*)H;            \
  a.m = (int)m; a.n = (int)n; a.l = l; a.k = k;                                                  \
  a.nsweeps = nsweeps; a.tol = tol; a.gram_mode = gram_mode; a.order = order;                   \
  a.G = sh.G; a.GR = sh.GR; a.GC = sh.GC; a.rows_per = sh.rows_per; a.cols_per = sh.cols_per;  \
  a.rows_lds = sh.rows_lds; a.lq = l | 1; a.cb = sh.cb; a.red2_elems = sh.red2_elems;             \
  a.xs_part = xs_part; a.xs_row = xs_row; a.xb_part = xb_part; a.xb_row = xb_row;              \
  a.xb_fin = xb_fin; a.lpw = slot; a.cbw = cbw; a.csw = csw; a.stats = stats; a.status = status;
  if (dt == 0) {
    FILL_ARGS(double);
    void* args[] = {&a};
    e = hipFuncSetAttribute((const void*)sweep_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sh.lds_bytes);
    if (e != hipSuccess) return e;
    return hipLaunchCooperativeKernel((const void*)sweep_kernel<double>, dim3(sh.G), dim3(NTH), args,
                                      (unsigned)sh.lds_bytes, s);
  } else {
    FILL_ARGS(float);
    void* args[] = {&a};
    e = hipFuncSetAttribute((const void*)sweep_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sh.lds_bytes);
    if (e != hipSuccess) return e;
    return hipLaunchCooperativeKernel((const void*)sweep_kernel<float>, dim3(sh.G), dim3(NTH), args,
                                      (unsigned)sh.lds_bytes, s);
  }
#undef FILL_ARGS
}

}  // namespace rnmf

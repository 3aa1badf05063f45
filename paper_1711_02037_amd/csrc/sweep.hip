// Compressed HALS sweeps (Sec. 3.2; Algorithm 1) as one persistent,
// cooperative kernel: every sweep of the call runs inside a single launch.
//
// Work split (G workgroups, one per compute unit, arranged as GR x GC):
//   - rows of Q and W are split into G slabs (the Q slab lives in registers,
//     or in LDS when it is too tall or wide for them; the W rows live in LDS,
//     or stay in global memory when they do not fit there);
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
// Regularized rules (Sec. 3.4): the ridge weight is added to the scales and
// subtracts alpha * (old block) in the numerators; the LASSO weight is
// subtracted from the H numerators and, for W, from the lifted column before
// the clip (beta_w / (V_jj + alpha_w)).  With zero weights every added term
// is an exact zero.
//
// Device-wide all-reduce: partials are written as 64-bit words (32-bit payload
// | 32-bit epoch) with agent-scope relaxed atomic stores, so every word carries
// its own readiness and no separate barrier is needed.  The per-column
// l-vector of the W phase goes through block owners (one workgroup sums each
// 16-word block over all partial slots and publishes copies of the totals);
// large vectors (T, V, S) through slice owners (reduce-scatter, then every
// workgroup reads all totals); the projected-gradient sum through a row, then
// column, two-hop scheme.  Every sum runs in a fixed order, so every
// workgroup obtains bit-identical results and the kernel is deterministic.
// Every wait is bounded: past the spin limit the kernel records
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
// `elem`, waiting for epoch e on every word.  Sources are taken in windows of
// WN: the window's loads are issued together and only its stale words are
// polled again, so a window costs about one round trip once its data has
// landed.  Polling every source at once loads the memory system enough to
// slow the whole device down; polling one source at a time pays a round trip
// per source.
template <typename V>
__device__ __forceinline__ V gather_sum(const u64* base, size_t stride, int nsrc, int elem, unsigned e,
                                        bool& ok) {
  constexpr int W = Words<V>::n;
  constexpr int WN = (W == 1) ? 8 : 4;
  V sum = (V)0;
  for (int s0 = 0; s0 < nsrc; s0 += WN) {
    u64 w[WN][W];
#pragma unroll
    for (int q = 0; q < WN; ++q)
      if (s0 + q < nsrc)
#pragma unroll
        for (int h = 0; h < W; ++h) w[q][h] = ld_ll(base + (s0 + q) * stride + (size_t)elem * W + h);
    long spins = 0;
    while (true) {
      bool all = true;
#pragma unroll
      for (int q = 0; q < WN; ++q)
        if (s0 + q < nsrc)
#pragma unroll
          for (int h = 0; h < W; ++h) all = all && ((unsigned)(w[q][h] >> 32) == e);
      if (all) break;
      if (!ok || ++spins > SPIN_LIMIT) { ok = false; break; }
#pragma unroll
      for (int q = 0; q < WN; ++q)
        if (s0 + q < nsrc)
#pragma unroll
          for (int h = 0; h < W; ++h)
            if ((unsigned)(w[q][h] >> 32) != e) w[q][h] = ld_ll(base + (s0 + q) * stride + (size_t)elem * W + h);
    }
#pragma unroll
    for (int q = 0; q < WN; ++q)
      if (s0 + q < nsrc) sum += value_of<V>(w[q]);
  }
  return sum;
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations
// (lgkmcnt) but not for its outstanding global stores, which a full
// __syncthreads() would drain (vmcnt also counts stores on this architecture).
// Use __syncthreads() where a thread reads global data another thread of the
// workgroup wrote.
__device__ __forceinline__ void lds_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt = 63, expcnt = 7, lgkmcnt = 0
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <typename T>
struct SweepArgs {
  const T* Q; const T* B; T* W; T* Wt; T* H;
  int m, n, l, k;
  int nsweeps; double tol; int gram_mode, order;
  double aw, ah, bw, bh;  // ridge (alpha) and LASSO (beta) weights
  int G, GR, GC, rows_per, cols_per, rows_lds, lq, cb;
  int xown;              // the last xown workgroups own the per-column exchange blocks
  int red2_elems;
  int alias_sv;          // S shares V's LDS slot (no projected gradient needed)
  u64* trace;            // optional phase timestamps (workgroup 0, first sweep)
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
__device__ __forceinline__ bool allreduce_small(const SweepArgs<T>& a, Xch& x, V* vals, int c, int* abort_flag) {
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
  if (!ok) *abort_flag = 1;
  lds_sync();
  if (t < c) vals[t] = r;
  lds_sync();
  return *abort_flag == 0;
}

// All-reduce of c <= cb values of type T held in LDS `vals` (in/out), by
// slice owners.  Every source workgroup stores its c partial sums in its
// slot; workgroup g then owns the slice [g cs, g cs + cs) (cs = ceil(c / G)):
// thread (group sg, element ei) loads element ei from the slots sg, sg + SG,
// ... (up to 16 words in flight), the group sums go through LDS and are added
// in group order, and the slice totals are stored once.  Finally every
// workgroup reads all c totals.  Each total is formed by one workgroup in a
// fixed order, so all workgroups receive bit-identical values.  The dedicated
// exchange owners (no rows or columns) add nothing and store no partials.
// `red` is LDS scratch of at least NTH values.
template <typename T>
__device__ __forceinline__ bool allreduce_big(const SweepArgs<T>& a, Xch& x, T* vals, int c, T* red,
                                              int* abort_flag) {
  constexpr int W = Words<T>::n;
  constexpr int MAXL = 16 / W;  // source slots per thread per round
  const int t = threadIdx.x;
  const unsigned e = ++x.seq;
  const unsigned par = (x.big_use++) & 1u;
  const int G = a.G, Gs = a.G - a.xown;
  const int cs = (c + G - 1) / G;
  const u64* P = a.xb_part;
  u64* FN = a.xb_fin + (size_t)par * G * a.csw;  // slice totals: element v at word v * W
  bool ok = true;
  if (x.g < Gs)
    for (int v = t; v < c; v += NTH) put<T>(a.xb_part + (size_t)x.g * a.cbw, v, vals[v], e);
  const int v0 = x.g * cs, v1 = (v0 + cs < c) ? v0 + cs : c;
  for (int b0 = v0; b0 < v1; b0 += NTH) {
    const int cc = (v1 - b0 < NTH) ? v1 - b0 : NTH;
    const int sgc = NTH / cc;
    const int ei = t % cc, sg = t / cc;
    if (sg < sgc) {
      T acc = (T)0;
      for (int r0 = sg; r0 < Gs; r0 += sgc * MAXL) {
        u64 w[MAXL][W];
#pragma unroll
        for (int q = 0; q < MAXL; ++q) {
          const int src = r0 + q * sgc;
#pragma unroll
          for (int h = 0; h < W; ++h)
            w[q][h] = src < Gs ? ld_ll(P + (size_t)src * a.cbw + (size_t)(b0 + ei) * W + h) : ((u64)e << 32);
        }
        long spins = 0;
        while (true) {
          bool all = true;
#pragma unroll
          for (int q = 0; q < MAXL; ++q)
#pragma unroll
            for (int h = 0; h < W; ++h) all = all && ((unsigned)(w[q][h] >> 32) == e);
          if (all) break;
          if (!ok || ++spins > SPIN_LIMIT) { ok = false; break; }
#pragma unroll
          for (int q = 0; q < MAXL; ++q)
#pragma unroll
            for (int h = 0; h < W; ++h)
              if ((unsigned)(w[q][h] >> 32) != e)
                w[q][h] = ld_ll(P + (size_t)(r0 + q * sgc) * a.cbw + (size_t)(b0 + ei) * W + h);
        }
#pragma unroll
        for (int q = 0; q < MAXL; ++q) acc += value_of<T>(w[q]);
      }
      red[sg * cc + ei] = acc;
    }
    lds_sync();
    if (t < cc) {
      T tot = (T)0;
      for (int q = 0; q < sgc; ++q) tot += red[q * cc + t];
      put<T>(FN, b0 + t, tot, e);
    }
    lds_sync();  // red is reused
  }
  // all totals: PB elements per thread in flight
  constexpr int PB = 8;
  for (int u0 = t; u0 < c; u0 += NTH * PB) {
    u64 w[PB][W];
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      const int v = u0 + b * NTH;
#pragma unroll
      for (int h = 0; h < W; ++h) w[b][h] = v < c ? ld_ll(FN + (size_t)v * W + h) : ((u64)e << 32);
    }
    long spins = 0;
    while (true) {
      bool all = true;
#pragma unroll
      for (int b = 0; b < PB; ++b)
#pragma unroll
        for (int h = 0; h < W; ++h) all = all && ((unsigned)(w[b][h] >> 32) == e);
      if (all) break;
      if (!ok || ++spins > SPIN_LIMIT) { ok = false; break; }
#pragma unroll
      for (int b = 0; b < PB; ++b)
#pragma unroll
        for (int h = 0; h < W; ++h)
          if ((unsigned)(w[b][h] >> 32) != e) w[b][h] = ld_ll(FN + (size_t)(u0 + b * NTH) * W + h);
    }
#pragma unroll
    for (int b = 0; b < PB; ++b) {
      const int v = u0 + b * NTH;
      if (v < c) vals[v] = value_of<T>(w[b]);
    }
  }
  if (!ok) *abort_flag = 1;
  lds_sync();
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

// FP64 matrix cores: v_mfma_f64_16x16x4f64 multiplies a 16 x 4 tile by a
// 4 x 16 tile; lane (i, g) = (lane % 16, lane / 16) supplies A[i][g] and
// B[g][i] and receives D[g + 4e][i] in element e (rows interleaved by 4,
// unlike the FP32 and BF16 forms, whose element e is row 4g + e; checked on
// gfx950 with distinct entries).
typedef double dx4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ dx4 mfma_f64(double a, double b, dx4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Cross-lane sums on the VALU (no LDS round trip).  sum8: over the 8 lanes of
// an aligned group (lane ^ 1, ^ 2, ^ 4 by DPP quad permutes and the half-row
// mirror).  sum_stride8: over the 8 lanes with equal lane % 8 (lane ^ 8 by a
// DPP row rotation, ^ 16 and ^ 32 by the permlane swaps of gfx950).  Every
// lane of a group obtains the bit-identical sum.
template <int CTRL>
__device__ __forceinline__ unsigned dpp32(unsigned x) {
  return (unsigned)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, true);
}
template <int CTRL, typename T>
__device__ __forceinline__ T dpp_mov(T x) {
  if constexpr (sizeof(T) == 4) {
    return __uint_as_float(dpp32<CTRL>(__float_as_uint(x)));
  } else {
    const u64 b = (u64)__double_as_longlong(x);
    const u64 lo = dpp32<CTRL>((unsigned)b), hi = dpp32<CTRL>((unsigned)(b >> 32));
    return __longlong_as_double((long long)(lo | (hi << 32)));
  }
}
template <typename T>
__device__ __forceinline__ T swap_sum16(T x) {
  if constexpr (sizeof(T) == 4) {
    auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
  } else {
    const u64 b = (u64)__double_as_longlong(x);
    auto pl = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
    auto ph = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    const double a0 = __longlong_as_double((long long)((u64)pl[0] | ((u64)ph[0] << 32)));
    const double a1 = __longlong_as_double((long long)((u64)pl[1] | ((u64)ph[1] << 32)));
    return a0 + a1;
  }
}
template <typename T>
__device__ __forceinline__ T swap_sum32(T x) {
  if constexpr (sizeof(T) == 4) {
    auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
  } else {
    const u64 b = (u64)__double_as_longlong(x);
    auto pl = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
    auto ph = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
    const double a0 = __longlong_as_double((long long)((u64)pl[0] | ((u64)ph[0] << 32)));
    const double a1 = __longlong_as_double((long long)((u64)pl[1] | ((u64)ph[1] << 32)));
    return a0 + a1;
  }
}
template <typename T>
__device__ __forceinline__ T sum8(T x) {
  x = x + dpp_mov<0xB1>(x);    // quad_perm [1,0,3,2]
  x = x + dpp_mov<0x4E>(x);    // quad_perm [2,3,0,1]
  return x + dpp_mov<0x141>(x);  // row_half_mirror
}
template <typename T>
__device__ __forceinline__ T sum_stride8(T x) {
  x = x + dpp_mov<0x128>(x);   // row_ror:8
  return swap_sum32(swap_sum16(x));
}

template <typename T> __device__ __forceinline__ T clip0(T x) { return x > (T)0 ? x : (T)0; }

// Per-column all-reduce by block owners.  The l-vector is cut into blocks of
// 16 words (one 128-byte line of a slot: 16 / W elements); block b has one
// owner workgroup, which sums the block over all G partial slots and
// publishes the totals in C copies (every other workgroup reads copy g mod C).
// Thread t of the owner takes element t mod EPB of the block from slots
// t / EPB + i * (NTH / EPB), so the loads of one wave cover whole lines and
// all of them are in flight together.  The sum runs in a fixed order (over i,
// across the lanes holding the same element, then over the waves), so every
// reader receives bit-identical totals whatever the arrival order.  Against
// a two-hop exchange in which every workgroup gathers from 16 slots twice,
// this moves about 1/14 of the polling traffic and takes one owner hop and one
// reader hop.
//
// Slot of copy c in the totals region (2 KB slots).  With room (the region
// holds at least 2 C + 2 slots) the copies sit in pairs on the upper 4 KB of
// successive 8 KB spans: at 100,000 x 5,000, k = 50 on 256 workgroups, 200
// sweeps take 58.8 ms this way against 59.7 ms with the copies packed from the
// start of the region (59.4 ms on the lower halves, 60.0 ms one per 16 KB).
__device__ __forceinline__ int copy_slot(int c, bool spread) {
  return spread ? 4 * (c >> 1) + 2 + (c & 1) : c;
}
template <typename T>
__device__ __forceinline__ void owner_block(const u64* P, u64* R, int G, size_t slot, int l, int b, int C,
                                            bool spread, unsigned e, T* red, bool& ok) {
  constexpr int W = Words<T>::n;
  constexpr int EPB = 16 / W;
  constexpr int SS = NTH / EPB;
  constexpr int MAXI = 256 / SS;  // G <= 256
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int ein = t % EPB, el = b * EPB + ein;
  const bool live = el < l;
  const int s0 = t / EPB;
  u64 w[MAXI][W];
#pragma unroll
  for (int i = 0; i < MAXI; ++i) {
    const int src = s0 + i * SS;
    const bool act = live && src < G;
#pragma unroll
    for (int h = 0; h < W; ++h)
      w[i][h] = act ? ld_ll(P + (size_t)src * slot + (size_t)el * W + h) : ((u64)e << 32);
  }
  long spins = 0;
  while (true) {
    bool all = true;
#pragma unroll
    for (int i = 0; i < MAXI; ++i)
#pragma unroll
      for (int h = 0; h < W; ++h) all = all && ((unsigned)(w[i][h] >> 32) == e);
    if (all) break;
    if (!ok || ++spins > SPIN_LIMIT) { ok = false; break; }
#pragma unroll
    for (int i = 0; i < MAXI; ++i)
#pragma unroll
      for (int h = 0; h < W; ++h)
        if ((unsigned)(w[i][h] >> 32) != e) w[i][h] = ld_ll(P + (size_t)(s0 + i * SS) * slot + (size_t)el * W + h);
  }
  T acc = (T)0;
#pragma unroll
  for (int i = 0; i < MAXI; ++i) acc += value_of<T>(w[i]);
  if constexpr (W == 1) acc = swap_sum32(swap_sum16(acc));  // lanes with equal lane % 16
  else acc = sum_stride8(acc);                                // lanes with equal lane % 8
  if (lane < EPB) red[wave * EPB + lane] = acc;
  lds_sync();
  if (t < C * EPB) {
    const int cp = t / EPB, ei = t % EPB;
    if (b * EPB + ei < l) {
      T tot = (T)0;
#pragma unroll
      for (int wv = 0; wv < NTH / 64; ++wv) tot += red[wv * EPB + ei];
      put<T>(R + (size_t)copy_slot(cp, spread) * slot, b * EPB + ei, tot, e);
    }
  }
  lds_sync();
}

// Maps a linear block index to (row block, column block) of the upper block
// triangle of an nb x nb block matrix, in row-major order.
__device__ __forceinline__ void upper_block(int b, int nb, int& r, int& c) {
  int q = 0, rem = b;
  while (rem >= nb - q) { rem -= nb - q; ++q; }
  r = q;
  c = q + rem;
}

// Register-resident Q slab (REGQ): thread (wave w, lane L) owns rows
// {8w + L/8 + 64 i : i < RQ} and columns {CQ (L % 8) + s : s < CQ} of the slab.
constexpr int RQ = 7;       // at most 448 rows per workgroup
constexpr int CQMAX = 12;   // at most 8 x 12 = 96 columns (FP32; FP64 takes 9, 72 columns)

// WG (with REGQ): the W rows stay in global memory (each workgroup owns rows
// r0 .. r0 + nr - 1 of W, which no other workgroup touches during the
// launch); the W phase stores W(r, j) there and S = W^T W is formed after the
// W phase from those rows, like the LDS-slab path.  This frees the LDS the
// rows would take, for tall inputs at larger k.
template <typename T, bool REGQ, int CQ, bool WG>
__global__ __launch_bounds__(NTH) void sweep_kernel(SweepArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* smem = (T*)smem_raw;
  __shared__ int abort_flag;
  __shared__ double pg_buf[2];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int l = a.l, k = a.k, n = a.n;
  const int g = blockIdx.x;
  Xch x;
  x.g = g; x.i = g / a.GC; x.j = g % a.GC; x.seq = 0; x.small_use = 0; x.big_use = 0;

  const int r0 = g * a.rows_per;
  int nr = a.m - r0; if (nr > a.rows_per) nr = a.rows_per; if (nr < 0) nr = 0;
  const int c0 = g * a.cols_per;
  int nc = a.n - c0; if (nc > a.cols_per) nc = a.cols_per; if (nc < 0) nc = 0;
  const int nrl = nr < a.rows_lds ? nr : a.rows_lds;  // rows whose Q lives in LDS
  const bool xowner_wg = a.xown > 0 && g >= a.G - a.xown;  // dedicated exchange owner (no rows)
  const int lq = a.lq;

  // LDS carve-up (red2 first so that it is 8-byte aligned for the FP64 sums)
  T* red2 = smem;                                 // scratch: backward partials, staging, pg sums
  T* Wts = red2 + a.red2_elems;                   // l x k
  T* U = Wts + (size_t)l * k;                     // [T: l x k | V: k x k | S: k x k]
  T* Tm = U;
  T* Vm = U + (size_t)l * k;
  T* Sm = a.alias_sv ? Vm : Vm + (size_t)k * k;   // S and V are never live together without pg
  T* vec = Vm + (size_t)k * k * (a.alias_sv ? 1 : 2);  // LPS
  T* wcol = vec + LPS;                            // rows_per
  T* Qs = wcol + a.rows_per;                      // rows_lds x lq
  // with the Q slab in registers, LDS also holds this workgroup's rows of W
  // and columns of B and H for the whole launch
  const int cp = a.cols_per;
  T* Ws = Qs + (size_t)a.rows_lds * lq;           // (rows_per + 1) x k (REGQ; the last row is a sink)
  T* Bs = Ws + (WG ? (size_t)0 : (size_t)(a.rows_per + 1) * k);  // l x cols_per   (REGQ)
  T* Hs = Bs + (size_t)l * cp;                    // k x cols_per   (REGQ)
  const T* Bp;
  T* Hp;
  int ldB;
  if constexpr (REGQ) { Bp = Bs; Hp = Hs; ldB = cp; }
  else { Bp = a.B + c0; Hp = a.H + c0; ldB = n; }
  const int ldH = ldB;

  const bool tracer = a.trace && g == 0 && t == 0;
#define TRACE(idx) \
  if (tracer) a.trace[(idx)] = __builtin_amdgcn_s_memrealtime();
  TRACE(0);
  if (t == 0) abort_flag = 0;
  const int ga = wave * 8 + (lane >> 3), gc = lane & 7;  // REGQ row group, column group
  T qreg[REGQ ? RQ : 1][REGQ ? CQ : 1];
  if constexpr (REGQ) {
#pragma unroll
    for (int i = 0; i < RQ; ++i)
#pragma unroll
      for (int s = 0; s < CQ; ++s) {
        const int rr = ga + 64 * i, aa = gc * CQ + s;
        qreg[i][s] = (rr < nr && aa < l) ? a.Q[(size_t)(r0 + rr) * l + aa] : (T)0;
      }
    if constexpr (!WG)
      for (int e = t; e < nr * k; e += NTH) Ws[e] = a.W[(size_t)r0 * k + e];
    for (int e = t; e < l * cp; e += NTH) {
      const int r = e / cp, cc = e - (e / cp) * cp;
      Bs[e] = cc < nc ? a.B[(size_t)r * n + c0 + cc] : (T)0;
    }
    for (int e = t; e < k * cp; e += NTH) {
      const int r = e / cp, cc = e - (e / cp) * cp;
      Hs[e] = cc < nc ? a.H[(size_t)r * n + c0 + cc] : (T)0;
    }
  } else {
    for (int e = t; e < nrl * l; e += NTH) {
      int rr = e / l, c = e - rr * l;
      Qs[rr * lq + c] = a.Q[(size_t)(r0 + rr) * l + c];
    }
  }
  for (int e = t; e < l * k; e += NTH) Wts[e] = a.Wt[e];
  __syncthreads();
  TRACE(1);
  bool tr_sweep = false;

  const bool need_S = (a.gram_mode != 1) || (a.tol > 0.0);
  const bool need_pg = a.tol > 0.0;
  const int RG = (NTH / l < 16) ? NTH / l : 16;
  const int kb = (k + 3) / 4, lb = (l + 3) / 4;
  // columns per chunk of the H phase's FP64 gradient block (k x hch doubles
  // at a pitch of hch + 1 in red2); below 8 the H phase takes the lane form
  int hch = (int)((size_t)a.red2_elems * sizeof(T) / 8 / (size_t)k) - 1;
  hch &= ~7;
  if (hch > 8 * ((a.cols_per + 7) / 8)) hch = 8 * ((a.cols_per + 7) / 8);

  // --- S = W^T W over this workgroup's rows (4 x 4 register blocks) --------
  // Rows are staged through LDS 32 at a time; the next chunk is loaded into
  // registers while the current one is used.
  auto local_wgram = [&]() __attribute__((always_inline)) {
    __syncthreads();  // W rows written by other threads of this workgroup
    constexpr int RC = 32, PF = (RC * KMAX + NTH - 1) / NTH;  // staged values per thread
    const int kp = 4 * kb;
    const int nblk = kb * (kb + 1) / 2;
    // NG groups of threads share the rows of a chunk (rows rg, rg + NG, ...)
    const int NG = (NTH / nblk < 8) ? NTH / nblk : 8;
    const int tb = t % nblk, rgi = t / nblk;
    int ba = -1, bb = -1;
    if (rgi < NG) upper_block(tb, kb, ba, bb);
    double acc[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = 0.0;
    T pf[PF];
    auto fetch = [&](int cstart) __attribute__((always_inline)) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int e = t + q * NTH;
        const int rr = e / kp, cc = e - (e / kp) * kp;
        pf[q] = (e < RC * kp && cstart + rr < nr && cc < k) ? a.W[(size_t)(r0 + cstart + rr) * k + cc] : (T)0;
      }
    };
    constexpr bool WLDS = REGQ && !WG;  // rows in the LDS copy Ws
    if constexpr (!WLDS) fetch(0);
    // rows come straight from the LDS copy Ws (leading dimension k) when it exists
    const int lds_ld = WLDS ? k : kp;
    for (int cs = 0; cs < nr; cs += RC) {
      const T* rows;
      if constexpr (WLDS) {
        rows = Ws + (size_t)cs * k;
      } else {
        rows = red2;
        lds_sync();
#pragma unroll
        for (int q = 0; q < PF; ++q) {
          const int e = t + q * NTH;
          if (e < RC * kp) red2[e] = pf[q];
        }
        lds_sync();
        if (cs + RC < nr) fetch(cs + RC);
      }
      if (ba >= 0) {
        const int rmax = (nr - cs < RC) ? nr - cs : RC;
        for (int rr = rgi; rr < rmax; rr += NG) {
          double u[4], w[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int c1 = 4 * ba + q, c2 = 4 * bb + q;
            u[q] = (WLDS && c1 >= k) ? 0.0 : (double)rows[rr * lds_ld + c1];
            w[q] = (WLDS && c2 >= k) ? 0.0 : (double)rows[rr * lds_ld + c2];
          }
#pragma unroll
          for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[p * 4 + q] = fma(u[p], w[q], acc[p * 4 + q]);
        }
      }
    }
    // fixed-order sum of the NG group partials through LDS (as doubles), in
    // passes of `cap` blocks so that the staging area bounds the LDS use
    lds_sync();
    double* gsum = (double*)red2;
    const int cap = (int)((size_t)a.red2_elems * sizeof(T) / 8 / 16);
    for (int b0 = 0; b0 < nblk; b0 += cap) {
      const bool mine = ba >= 0 && tb >= b0 && tb < b0 + cap;
      for (int gi = 0; gi < NG; ++gi) {
        if (rgi == gi && mine) {
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            if (gi == 0) gsum[(tb - b0) * 16 + e] = acc[e];
            else gsum[(tb - b0) * 16 + e] += acc[e];
          }
        }
        lds_sync();
      }
      if (t >= b0 && t < nblk && t < b0 + cap) {
        int pa, pb;
        upper_block(t, kb, pa, pb);
#pragma unroll
        for (int p = 0; p < 4; ++p)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = 4 * pa + p, c = 4 * pb + q;
            if (r < k && c < k) {
              const T v = (T)gsum[(t - b0) * 16 + p * 4 + q];
              Sm[r * k + c] = v;
              if (pa != pb) Sm[c * k + r] = v;
            }
          }
      }
      lds_sync();
    }
  };

  // REGQ: the W phase fills the local S column by column (s_cols marks the
  // columns done); the rest comes from the LDS copy of the W rows.
  unsigned long long s_cols = 0ull;
  auto s_exchange = [&]() __attribute__((always_inline)) -> bool {
    const unsigned long long all_cols = (k == 64) ? ~0ull : ((1ull << k) - 1ull);
    if constexpr (REGQ) {
      if ((s_cols & all_cols) != all_cols) local_wgram();
      s_cols = 0ull;
      lds_sync();
    } else {
      local_wgram();
    }
    if (tr_sweep) { TRACE(6 + 2 * k); }
    return allreduce_big<T>(a, x, Sm, k * k, red2, &abort_flag);
  };

  // --- T = B H^T and V = H H^T over this workgroup's columns ---------------
  // 4 x 4 register blocks (FP64 accumulation); B and H columns are staged
  // through LDS 8 columns at a time.
  auto tv_exchange = [&]() __attribute__((always_inline)) -> bool {
    if constexpr (REGQ) {
      // [B; H] (l + k rows) times H^T over this workgroup's nc columns on FP64
      // matrix cores: rows below l give T = B H^T, the rest V = H H^T (its
      // upper triangle, mirrored); one 16 x 16 output tile per wave at a time
      lds_sync();
      if (tr_sweep) { TRACE(124); }
      const int fi = lane & 15, fg = lane >> 4;
      const int MT = (l + k + 15) / 16, NTt = (k + 15) / 16, KS = (nc + 3) / 4;
      for (int tile = wave; tile < MT * NTt; tile += NTH / 64) {
        const int mt = tile / NTt, nt = tile - (tile / NTt) * NTt;
        const int ra = 16 * mt + fi, cb = 16 * nt + fi;
        const bool aok = ra < l + k, bok = cb < k;
        const T* arow = ra < l ? Bs + (size_t)ra * cp : Hs + (size_t)(aok ? ra - l : 0) * cp;
        const T* brow = Hs + (size_t)(bok ? cb : 0) * cp;
        dx4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int s4 = 0; s4 < KS; ++s4) {
          const int cc = 4 * s4 + fg;
          const double av = (aok && cc < nc) ? (double)arow[cc] : 0.0;
          const double bv = (bok && cc < nc) ? (double)brow[cc] : 0.0;
          acc = mfma_f64(av, bv, acc);
        }
        if (bok) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int r = 16 * mt + fg + 4 * e;
            if (r < l) {
              Tm[r * k + cb] = (T)acc[e];
            } else if (r < l + k && r - l <= cb) {
              Vm[(r - l) * k + cb] = (T)acc[e];
              Vm[cb * k + (r - l)] = (T)acc[e];
            }
          }
        }
      }
      if (tr_sweep) { TRACE(125); }
      lds_sync();
      if (tr_sweep) { TRACE(120); }
      return allreduce_big<T>(a, x, U, l * k + k * k, red2, &abort_flag);
    }
    __syncthreads();  // H columns written by other threads of this workgroup
    constexpr int CW = 8;
    const int nbt = lb * kb;                 // blocks of T
    const int nbv = kb * (kb + 1) / 2;       // upper blocks of V
    T* Bst;
    T* Hst;
    if constexpr (REGQ) { Bst = Bs; Hst = Hs; }
    else { Bst = red2; Hst = red2 + LMAX * CW; }  // l x CW and k x CW staging
    double acc[2][16];
    int br[2], bc[2], isv[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int b = t + q * NTH;
      isv[q] = -1;
      if (b < nbt) { br[q] = b / kb; bc[q] = b - (b / kb) * kb; isv[q] = 0; }
      else if (b < nbt + nbv) { upper_block(b - nbt, kb, br[q], bc[q]); isv[q] = 1; }
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[q][e] = 0.0;
    }
    const int CWS = REGQ ? cp : CW;  // column stride of the staged slabs
    for (int cs = 0; cs < nc; cs += (REGQ ? nc : CW)) {
      const int w = REGQ ? nc : ((nc - cs < CW) ? nc - cs : CW);
      if constexpr (!REGQ) {
        lds_sync();
        for (int e = t; e < (l + k) * CW; e += NTH) {
          const int row = e / CW, cc = e - (e / CW) * CW;
          if (row < l) Bst[row * CW + cc] = cc < w ? a.B[(size_t)row * n + c0 + cs + cc] : (T)0;
          else Hst[(row - l) * CW + cc] = cc < w ? a.H[(size_t)(row - l) * n + c0 + cs + cc] : (T)0;
        }
      }
      lds_sync();
      if (tr_sweep) { TRACE(124); }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (isv[q] < 0) continue;
        const T* left = isv[q] ? Hst : Bst;
        const int rl = isv[q] ? k : l;
        for (int cc = 0; cc < w; ++cc) {
          double u[4], v[4];
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            const int r = 4 * br[q] + p, c = 4 * bc[q] + p;
            u[p] = r < rl ? (double)left[r * CWS + cc] : 0.0;
            v[p] = c < k ? (double)Hst[c * CWS + cc] : 0.0;
          }
#pragma unroll
          for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int s = 0; s < 4; ++s) acc[q][p * 4 + s] = fma(u[p], v[s], acc[q][p * 4 + s]);
        }
      }
    }
    if (tr_sweep) { TRACE(125); }
    lds_sync();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (isv[q] < 0) continue;
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int r = 4 * br[q] + p, c = 4 * bc[q] + s;
          if (c >= k) continue;
          if (!isv[q]) {
            if (r < l) Tm[r * k + c] = (T)acc[q][p * 4 + s];
          } else if (r < k) {
            Vm[r * k + c] = (T)acc[q][p * 4 + s];
            if (br[q] != bc[q]) Vm[c * k + r] = (T)acc[q][p * 4 + s];
          }
        }
    }
    // blocks beyond 2 * NTH (l = 128 and k = 64 need at most 648)
    for (int b = t + 2 * NTH; b < nbt + nbv; b += NTH) {
      int rb, cb2, vv = b >= nbt;
      if (!vv) { rb = b / kb; cb2 = b - (b / kb) * kb; } else upper_block(b - nbt, kb, rb, cb2);
      for (int p = 0; p < 4; ++p)
        for (int s = 0; s < 4; ++s) {
          const int r = 4 * rb + p, c = 4 * cb2 + s;
          if (c >= k || r >= (vv ? k : l)) continue;
          double sum = 0.0;
          for (int cc = 0; cc < nc; ++cc) {
            const double lv = vv ? (double)Hp[(size_t)r * ldH + cc] : (double)Bp[(size_t)r * ldB + cc];
            sum = fma(lv, (double)Hp[(size_t)c * ldH + cc], sum);
          }
          if (!vv) Tm[r * k + c] = (T)sum;
          else { Vm[r * k + c] = (T)sum; Vm[c * k + r] = (T)sum; }
        }
    }
    lds_sync();
    if (tr_sweep) { TRACE(120); }
    return allreduce_big<T>(a, x, U, l * k + k * k, red2, &abort_flag);
  };

  // --- H phase: this workgroup's columns of H, one wavefront per column -----
  auto h_phase = [&]() __attribute__((always_inline)) {
    const T* Snum = Sm;
    const T* Ssc = Sm;
    if (a.gram_mode != 0) {
      // W~^T W~ into the T region (T is recomputed after the H phase)
      for (int e = t; e < k * k; e += NTH) {
        int ii = e / k, jj = e % k;
        double s = 0.0;
        for (int aa = 0; aa < l; ++aa) s = fma((double)Wts[aa * k + ii], (double)Wts[aa * k + jj], s);
        Tm[e] = (T)s;
      }
      lds_sync();
      Snum = Tm;
      if (a.gram_mode == 1) Ssc = Tm;
    }
    // reciprocal scales, one per lane (0 marks a skipped row)
    double rinv_l = 0.0;
    if (lane < k) {
      const double d = (double)Ssc[lane * k + lane] + a.ah;
      rinv_l = d > 0.0 ? 1.0 / d : 0.0;
    }
    // FP64 arithmetic: the update cancels R against H^T S, and S is the Gram
    // of a nonnegative factor, so its rounding is amplified.  A wave takes up
    // to HI columns at once (columns cc, cc + 8, ...): their Gauss-Seidel
    // chains are independent, so their latencies overlap.
    constexpr int HI = 3;
    const int jj = lane < k ? lane : 0;
    if constexpr (REGQ) {
      if (hch >= 8) {
        // G = W~^T B - Snum^T H for a chunk of hch columns on FP64 matrix
        // cores (K = l + k), kept in red2 as doubles (pitch hch + 1), then
        // the row updates of each column in order.  Every lane forms the
        // candidate row value of its own row; lane ii's is the update of
        // step ii, broadcast as the change it makes.
        lds_sync();  // red2 may still be read by the exchange that precedes
        double* Gd = (double*)red2;
        const int gp = hch + 1;
        const int fi = lane & 15, fg = lane >> 4;
        const int MT = (k + 15) / 16, KS = (l + k + 3) / 4;
        for (int cs = 0; cs < nc; cs += hch) {
          const int w = (nc - cs < hch) ? nc - cs : hch;
          const int NTc = (w + 15) / 16;
          for (int tile = wave; tile < MT * NTc; tile += NTH / 64) {
            const int mt = tile / NTc, nt = tile - (tile / NTc) * NTc;
            const int jr = 16 * mt + fi, cc = 16 * nt + fi;
            const bool jok = jr < k, cok = cc < w;
            const int jc = jok ? jr : 0, ccc = cs + (cok ? cc : 0);
            dx4 acc = {0.0, 0.0, 0.0, 0.0};
            for (int s4 = 0; s4 < KS; ++s4) {
              const int kap = 4 * s4 + fg;
              double av = 0.0, bv = 0.0;
              if (kap < l) {
                av = jok ? (double)Wts[kap * k + jc] : 0.0;
                bv = cok ? (double)Bs[(size_t)kap * cp + ccc] : 0.0;
              } else if (kap < l + k) {
                av = jok ? -(double)Snum[(kap - l) * k + jc] : 0.0;
                bv = cok ? (double)Hs[(size_t)(kap - l) * cp + ccc] : 0.0;
              }
              acc = mfma_f64(av, bv, acc);
            }
            if (cok) {
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const int r = 16 * mt + fg + 4 * e;
                if (r < k) Gd[r * gp + cc] = acc[e];
              }
            }
          }
          if (tr_sweep && cs == 0) { TRACE(121); }
          lds_sync();
          if (tr_sweep && cs == 0) { TRACE(122); }
          for (int cb = wave; cb < w; cb += (NTH / 64) * HI) {
            bool live[HI];
            double h[HI], gs[HI], hn[HI];
#pragma unroll
            for (int q = 0; q < HI; ++q) {
              const int cc = cb + (NTH / 64) * q;
              live[q] = cc < w;
              const int c = live[q] ? cc : cb;
              h[q] = lane < k ? (double)Hs[(size_t)lane * cp + cs + c] : 0.0;
              gs[q] = lane < k ? Gd[lane * gp + c] - fma(a.ah, h[q], a.bh) : 0.0;
              hn[q] = h[q];
            }
            // a zero scale (rinv 0) gives the lane's own value back: change +0
            T s_nx = Snum[jj];
            for (int ii = 0; ii < k; ++ii) {
              const double sij = (double)s_nx;
              s_nx = Snum[(ii + 1 < k ? ii + 1 : ii) * k + jj];
#pragma unroll
              for (int q = 0; q < HI; ++q) {
                // the new row is rounded to the storage type before it is used
                const double cand = (double)clip0<T>((T)fma(gs[q], rinv_l, h[q]));
                const double d = readlane<double>(cand - h[q], ii);
                if (lane == ii) hn[q] = cand;
                gs[q] = fma(-sij, d, gs[q]);
              }
            }
            if (tr_sweep && cs == 0 && cb == wave) {
              if (wave == 0) { TRACE(123); }
              // wavefront 7's end of the row updates (traced launches only)
              if (a.trace && g == 0 && wave == 7 && lane == 0) a.trace[126] = __builtin_amdgcn_s_memrealtime();
            }
#pragma unroll
            for (int q = 0; q < HI; ++q)
              if (live[q] && lane < k) Hs[(size_t)lane * cp + cs + cb + (NTH / 64) * q] = (T)hn[q];
          }
          lds_sync();  // the next chunk reuses red2; the H columns are read next
        }
        return;
      }
    }
    const int l0 = l < 64 ? l : 64;
    for (int cb = wave; cb < nc; cb += (NTH / 64) * HI) {
      bool live[HI];
      T b0[HI], b1[HI];
      double h[HI], R0[HI], R1[HI];
#pragma unroll
      for (int q = 0; q < HI; ++q) {
        const int cc = cb + (NTH / 64) * q;
        live[q] = cc < nc;
        const int c = live[q] ? cc : cb;
        // lane holds B(lane, c) and B(lane + 64, c); H(lane, c)
        b0[q] = lane < l ? Bp[(size_t)lane * ldB + c] : (T)0;
        b1[q] = lane + 64 < l ? Bp[(size_t)(lane + 64) * ldB + c] : (T)0;
        h[q] = lane < k ? (double)Hp[(size_t)lane * ldH + c] : 0.0;
        R0[q] = 0.0;
        R1[q] = 0.0;
      }
      // R(c, jj) = sum_a B(a, c) W~(a, jj): four LDS reads in flight per step
      int aa = 0;
      for (; aa + 4 <= l0; aa += 4) {
        double w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) w[u] = (double)Wts[(aa + u) * k + jj];
#pragma unroll
        for (int q = 0; q < HI; ++q) {
          R0[q] = fma((double)readlane<T>(b0[q], aa), w[0], R0[q]);
          R1[q] = fma((double)readlane<T>(b0[q], aa + 1), w[1], R1[q]);
          R0[q] = fma((double)readlane<T>(b0[q], aa + 2), w[2], R0[q]);
          R1[q] = fma((double)readlane<T>(b0[q], aa + 3), w[3], R1[q]);
        }
      }
      for (; aa < l0; ++aa) {
        const double w0 = (double)Wts[aa * k + jj];
#pragma unroll
        for (int q = 0; q < HI; ++q) R0[q] = fma((double)readlane<T>(b0[q], aa), w0, R0[q]);
      }
      for (aa = 64; aa < l; ++aa) {
        const double w1 = (double)Wts[aa * k + jj];
#pragma unroll
        for (int q = 0; q < HI; ++q) R1[q] = fma((double)readlane<T>(b1[q], aa - 64), w1, R1[q]);
      }
      if (tr_sweep) { TRACE(121); }
      double g0[HI], g1[HI];
#pragma unroll
      for (int q = 0; q < HI; ++q) { g0[q] = R0[q] + R1[q]; g1[q] = 0.0; }
      int ii = 0;
      for (; ii + 4 <= k; ii += 4) {
        double sv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) sv[u] = (double)Snum[(ii + u) * k + jj];
#pragma unroll
        for (int q = 0; q < HI; ++q) {
          g0[q] = fma(-sv[0], readlane<double>(h[q], ii), g0[q]);
          g1[q] = fma(-sv[1], readlane<double>(h[q], ii + 1), g1[q]);
          g0[q] = fma(-sv[2], readlane<double>(h[q], ii + 2), g0[q]);
          g1[q] = fma(-sv[3], readlane<double>(h[q], ii + 3), g1[q]);
        }
      }
      for (; ii < k; ++ii) {
        const double s0 = (double)Snum[ii * k + jj];
#pragma unroll
        for (int q = 0; q < HI; ++q) g0[q] = fma(-s0, readlane<double>(h[q], ii), g0[q]);
      }
      // regularized numerator: - bh - ah H(lane, c); lane i's g is read only at
      // step i, while H(i, c) still holds its old value, so it is added here
      double gsum[HI];
#pragma unroll
      for (int q = 0; q < HI; ++q) gsum[q] = (g0[q] + g1[q]) - fma(a.ah, h[q], a.bh);
      if (tr_sweep) { TRACE(122); }
      // Gauss-Seidel over the rows: the scale comes from a register by lane
      // broadcast and the next S entry is loaded one step ahead, so no LDS
      // round trip sits on the chain
      // (a zero scale leaves the row unchanged: h stays, delta is +0)
      double s_cur = (double)Snum[jj];
      double s_nxt = (double)Snum[(k > 1 ? 1 : 0) * k + jj];
      for (ii = 0; ii < k; ++ii) {
        const double sij = s_cur;
        s_cur = s_nxt;
        s_nxt = (double)Snum[min(ii + 2, k - 1) * k + jj];  // two steps ahead
        const double rd = readlane<double>(rinv_l, ii);
#pragma unroll
        for (int q = 0; q < HI; ++q) {
          const double hi = readlane<double>(h[q], ii);
          const double gi = readlane<double>(gsum[q], ii);
          // the new row is rounded to the storage type before it is used
          const double hn = (rd > 0.0) ? (double)clip0<T>((T)fma(gi, rd, hi)) : hi;
          const double delta = hn - hi;
          if (lane == ii) h[q] = hn;
          gsum[q] = fma(-sij, delta, gsum[q]);
        }
      }
      if (tr_sweep) { TRACE(123); }
#pragma unroll
      for (int q = 0; q < HI; ++q)
        if (live[q] && lane < k) Hp[(size_t)lane * ldH + cb + (NTH / 64) * q] = (T)h[q];
    }
    if constexpr (REGQ) lds_sync();
    else __syncthreads();
  };

  // --- W phase: columns of W in order, one device-wide exchange each --------
  // W phase with the Q slab in registers.  Per column: lift and clip (a
  // register GEMV reduced over the 8 column-group lanes), the local map-back
  // (reduced over the row groups: the 8 of a wave by lane permutes, then the
  // waves through LDS), and one device-wide exchange of the l-vector through
  // the block owners.  While it is in flight, thread t < l forms the part of
  // the next column's update that does not involve the column being exchanged
  // (its term is added once the value arrives, so one workgroup barrier
  // separates the arrival from the next lift), and threads t >= 128 form the
  // local partial sums of S = W^T W for the finished columns.
  auto w_phase_reg = [&]() __attribute__((always_inline)) -> bool {
    constexpr int PW = 8 * CQ;         // row of the per-wave partials
    T* part = red2;                    // 8 x PW: per-wave map-back partials
    double* spart = (double*)(red2 + 8 * 8 * CQMAX + 5 * LPS);  // 2 x 384: local S partial sums
    T* ored = red2 + 8 * 8 * CQMAX + 5 * LPS + 768 * 8 / sizeof(T);  // 128: exchange owner's wave sums
    const int nblk_x = (l * Words<T>::n + 15) / 16;          // 16-word blocks of the l-vector
    const int ncopy_x = a.G < 16 ? a.G : 16;                 // copies of the totals
    const bool spread_x = a.G >= 2 * ncopy_x + 2;            // copy_slot's spread placement fits
    int jprev = -1;  // column whose S partials await their reduction
    const T aw = (T)a.aw, bw = (T)a.bw;
    // columns with a positive scale V_jj + alpha_w, as a wave-uniform bit set
    // (every wave reads the same diagonal), so that finding the next column
    // costs no LDS round trip inside the column loop
    const unsigned long long vmask =
        __builtin_amdgcn_ballot_w64(lane < k && Vm[(lane < k ? lane : 0) * (k + 1)] + aw > (T)0);
    auto next_col = [&](int j) __attribute__((always_inline)) -> int {
      const int q0 = j + 1;
      if (q0 >= k) return k;
      const unsigned long long rest = vmask >> q0;
      return rest ? q0 + __builtin_ctzll(rest) : k;
    };
    // entries of the update vector past l stay zero, so the lift reads all
    // CQ entries of its column group without a per-entry predicate
    for (int e = l + t; e < 8 * CQ; e += NTH) vec[e] = (T)0;
    int jj = next_col(-1);
    if (jj >= k) return true;
    // update vector of the first column: v = W~(:,j) + (T(:,j) - W~ V(:,j)) / V_jj
    if (t < l) {
      const T* wr = Wts + t * k;
      T s0 = Tm[t * k + jj], s1 = (T)0;
      int ii = 0;
      for (; ii + 2 <= k; ii += 2) {
        s0 = fma(-wr[ii], Vm[ii * k + jj], s0);
        s1 = fma(-wr[ii + 1], Vm[(ii + 1) * k + jj], s1);
      }
      for (; ii < k; ++ii) s0 = fma(-wr[ii], Vm[ii * k + jj], s0);
      const T wo = Wts[t * k + jj];
      vec[t] = wo + ((s0 + s1) - aw * wo) / (Vm[jj * k + jj] + aw);
    }
    lds_sync();
    while (jj < k) {
      if (!xowner_wg) {
      // lift and clip: W(r, j) = max(0, Q(r, :) v - beta_w / (V_jj + alpha_w))
      const T shift = bw / (Vm[jj * k + jj] + aw);
      T vs[CQ];
#pragma unroll
      for (int s = 0; s < CQ; ++s) vs[s] = vec[gc * CQ + s];
      T w[RQ];
#pragma unroll
      for (int i = 0; i < RQ; ++i) {
        T u0 = (T)0, u1 = (T)0;
#pragma unroll
        for (int s = 0; s + 1 < CQ; s += 2) {
          u0 = fma(qreg[i][s], vs[s], u0);
          u1 = fma(qreg[i][s + 1], vs[s + 1], u1);
        }
        if (CQ & 1) u0 = fma(qreg[i][CQ - 1], vs[CQ - 1], u0);
        w[i] = clip0<T>(sum8<T>(u0 + u1) - shift);
      }
      if (gc == 0) {
        if constexpr (WG) {
#pragma unroll
          for (int i = 0; i < RQ; ++i) {
            const int rr = ga + 64 * i;
            if (rr < nr) a.W[(size_t)(r0 + rr) * k + jj] = w[i];
          }
        } else {
          // W is written back once, at the end; rows past the slab land in the
          // sink row rows_per, or in rows nr .. rows_per - 1 that no one reads
          // (a clamp instead of a predicate per row)
#pragma unroll
          for (int i = 0; i < RQ; ++i) {
            const int rr = min(ga + 64 * i, a.rows_per);
            Ws[rr * k + jj] = w[i];
          }
        }
      }
      // local map-back partials: sum_i Q(r_i, a) w_i over this thread's rows
      T pv[CQ];
#pragma unroll
      for (int s = 0; s < CQ; ++s) {
        T p0 = (T)0, p1 = (T)0;
#pragma unroll
        for (int i = 0; i + 1 < RQ; i += 2) {
          p0 = fma(qreg[i][s], w[i], p0);
          p1 = fma(qreg[i + 1][s], w[i + 1], p1);
        }
        if (RQ & 1) p0 = fma(qreg[RQ - 1][s], w[RQ - 1], p0);
        pv[s] = sum_stride8<T>(p0 + p1);
      }
      if (lane < 8) {
#pragma unroll
        for (int s = 0; s < CQ; ++s) part[wave * PW + gc * CQ + s] = pv[s];
      }
      }  // !xowner_wg
      const int nj = next_col(jj);
      lds_sync();
      if (tr_sweep) { TRACE(5 + 2 * jj); }
      // exchange (t < l) and, meanwhile, the next update vector's partials
      const unsigned e = ++x.seq;
      const unsigned par = (x.small_use++) & 1u;
      T wt = (T)0;
      bool ok = true;
      const size_t slot = (size_t)LPS * 2;
      u64* P = a.xs_part + ((size_t)par * a.G) * slot;
      u64* RS = a.xs_row + ((size_t)par * a.G) * slot;
      T cs = (T)0;  // sum over i != jj of W~(t, i) V(i, nj): the known part of the next update
      if (t < l && !xowner_wg) {
        T s = part[t];
#pragma unroll
        for (int wv = 1; wv < 8; ++wv) s += part[wv * PW + t];
        put<T>(P + (size_t)x.g * slot, t, s, e);
        if (nj < k) {
          // row t of W~ is private to thread t during the W phase
          const T* wr = Wts + t * k;
          T c0 = (T)0, c1 = (T)0, c2 = (T)0, c3 = (T)0;
          int ii = 0;
          for (; ii + 4 <= k; ii += 4) {
            c0 = fma(ii == jj ? (T)0 : wr[ii], Vm[ii * k + nj], c0);
            c1 = fma(ii + 1 == jj ? (T)0 : wr[ii + 1], Vm[(ii + 1) * k + nj], c1);
            c2 = fma(ii + 2 == jj ? (T)0 : wr[ii + 2], Vm[(ii + 2) * k + nj], c2);
            c3 = fma(ii + 3 == jj ? (T)0 : wr[ii + 3], Vm[(ii + 3) * k + nj], c3);
          }
          for (; ii < k; ++ii) c0 = fma(ii == jj ? (T)0 : wr[ii], Vm[ii * k + nj], c0);
          cs = (c0 + c1) + (c2 + c3);
        }
      } else if (t >= 128) {
        if (need_S && !WG) {
          // local S(i, j) = sum_r W(r, i) W(r, j) for i <= j (columns i < j
          // are final): entry i, rows r = p, p + P, ... in part p
          const int h = t - 128, np = 384 / (jj + 1);
          const int i = h / np, p = h - (h / np) * np;
          // first finish the previous column (its partials are in the other buffer)
          if (jprev >= 0 && h <= jprev) {
            const int npp = 384 / (jprev + 1);
            const double* sp = spart + (jprev & 1) * 384 + h * npp;
            double s = 0.0;
            for (int q = 0; q < npp; ++q) s += sp[q];
            Sm[h * k + jprev] = (T)s;
            Sm[jprev * k + h] = (T)s;
          }
          if (i <= jj) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int r = p;
            for (; r + 3 * np < nr; r += 4 * np) {
              s0 = fma((double)Ws[r * k + i], (double)Ws[r * k + jj], s0);
              s1 = fma((double)Ws[(r + np) * k + i], (double)Ws[(r + np) * k + jj], s1);
              s2 = fma((double)Ws[(r + 2 * np) * k + i], (double)Ws[(r + 2 * np) * k + jj], s2);
              s3 = fma((double)Ws[(r + 3 * np) * k + i], (double)Ws[(r + 3 * np) * k + jj], s3);
            }
            for (; r < nr; r += np) s0 = fma((double)Ws[r * k + i], (double)Ws[r * k + jj], s0);
            spart[(jj & 1) * 384 + h] = (s0 + s1) + (s2 + s3);
          }
        }
      }
      // block owners sum the partials; every workgroup then reads the totals
      for (int b = 0; b < nblk_x; ++b) {
        const int ow = a.xown > 0 ? a.G - a.xown + b : ((nblk_x <= a.G) ? (b * a.G) / nblk_x : b % a.G);
        if (ow == g) owner_block<T>(P, RS, a.G - a.xown, slot, l, b, ncopy_x, spread_x, e, ored, ok);
      }
      if (t < l && !xowner_wg) {
        wt = gather_sum<T>(RS + (size_t)copy_slot(g % ncopy_x, spread_x) * slot, slot, 1, t, e, ok);
        Wts[t * k + jj] = wt;
        if (g == 0 && !(wt == wt)) atomicOr(a.status, ST_NONFINITE_SWEEP);
        if (nj < k) {
          const T s = fma(wt, Vm[jj * k + nj], cs);
          const T wo = Wts[t * k + nj];
          vec[t] = wo + ((Tm[t * k + nj] - s) - aw * wo) / (Vm[nj * k + nj] + aw);
        }
      }
      if constexpr (!WG) s_cols |= 1ull << jj;
      if (!ok) abort_flag = 1;
      if (tr_sweep) { TRACE(6 + 2 * jj); }
      lds_sync();
      if (abort_flag) return false;
      jprev = jj;
      jj = nj;
    }
    if (need_S && !WG && jprev >= 0) {
      const int h = t - 128;
      if (h >= 0 && h <= jprev) {
        const int npp = 384 / (jprev + 1);
        const double* sp = spart + (jprev & 1) * 384 + h * npp;
        double s = 0.0;
        for (int q = 0; q < npp; ++q) s += sp[q];
        Sm[h * k + jprev] = (T)s;
        Sm[jprev * k + h] = (T)s;
      }
      lds_sync();
    }
    return true;
  };

  auto w_phase = [&]() __attribute__((always_inline)) -> bool {
    const T aw = (T)a.aw, bw = (T)a.bw;
    for (int jj = 0; jj < k; ++jj) {
      const T d = Vm[jj * k + jj] + aw;
      if (!(d > (T)0)) continue;
      const T shift = bw / d;
      if (t < l) {
        const T* wr = Wts + t * k;
        T s0 = Tm[t * k + jj], s1 = (T)0, s2 = (T)0, s3 = (T)0;
        int ii = 0;
        for (; ii + 4 <= k; ii += 4) {
          s0 = fma(-wr[ii], Vm[ii * k + jj], s0);
          s1 = fma(-wr[ii + 1], Vm[(ii + 1) * k + jj], s1);
          s2 = fma(-wr[ii + 2], Vm[(ii + 2) * k + jj], s2);
          s3 = fma(-wr[ii + 3], Vm[(ii + 3) * k + jj], s3);
        }
        for (; ii < k; ++ii) s0 = fma(-wr[ii], Vm[ii * k + jj], s0);
        const T wo = Wts[t * k + jj];
        vec[t] = wo + (((s0 + s1) + (s2 + s3)) - aw * wo) / d;
      }
      lds_sync();
      if (tr_sweep && jj == 1) { TRACE(10 + 2 * k); }
      // lift and clip on the local rows: W(r, j) = max(0, Q(r, :) v)
      for (int rr = t; rr < nr; rr += NTH) {
        const T* q = rr < nrl ? nullptr : a.Q + (size_t)(r0 + rr) * l;
        T u0 = (T)0, u1 = (T)0, u2 = (T)0, u3 = (T)0;
        int aa = 0;
        if (rr < nrl) {
          const T* qs = Qs + rr * lq;
          for (; aa + 4 <= l; aa += 4) {
            u0 = fma(qs[aa], vec[aa], u0);
            u1 = fma(qs[aa + 1], vec[aa + 1], u1);
            u2 = fma(qs[aa + 2], vec[aa + 2], u2);
            u3 = fma(qs[aa + 3], vec[aa + 3], u3);
          }
          for (; aa < l; ++aa) u0 = fma(qs[aa], vec[aa], u0);
        } else {
          for (; aa + 4 <= l; aa += 4) {
            u0 = fma(q[aa], vec[aa], u0);
            u1 = fma(q[aa + 1], vec[aa + 1], u1);
            u2 = fma(q[aa + 2], vec[aa + 2], u2);
            u3 = fma(q[aa + 3], vec[aa + 3], u3);
          }
          for (; aa < l; ++aa) u0 = fma(q[aa], vec[aa], u0);
        }
        const T w = clip0<T>(((u0 + u1) + (u2 + u3)) - shift);
        wcol[rr] = w;
        a.W[(size_t)(r0 + rr) * k + jj] = w;
      }
      lds_sync();
      if (tr_sweep && jj == 1) { TRACE(11 + 2 * k); }
      // local part of the map-back Q^T W(:, j)
      if (t < RG * l) {
        const int aa = t % l, rg = t / l;
        T s0 = (T)0, s1 = (T)0, s2 = (T)0, s3 = (T)0;
        int rr = rg;
        for (; rr + 3 * RG < nrl; rr += 4 * RG) {
          s0 = fma(Qs[rr * lq + aa], wcol[rr], s0);
          s1 = fma(Qs[(rr + RG) * lq + aa], wcol[rr + RG], s1);
          s2 = fma(Qs[(rr + 2 * RG) * lq + aa], wcol[rr + 2 * RG], s2);
          s3 = fma(Qs[(rr + 3 * RG) * lq + aa], wcol[rr + 3 * RG], s3);
        }
        for (; rr < nrl; rr += RG) s0 = fma(Qs[rr * lq + aa], wcol[rr], s0);
        for (; rr < nr; rr += RG) s0 = fma(a.Q[(size_t)(r0 + rr) * l + aa], wcol[rr], s0);
        red2[rg * LPS + aa] = (s0 + s1) + (s2 + s3);
      }
      lds_sync();
      if (tr_sweep && jj == 1) { TRACE(12 + 2 * k); }
      if (t < l) {
        T s = (T)0;
        for (int rg = 0; rg < RG; ++rg) s += red2[rg * LPS + t];
        vec[t] = s;
      }
      lds_sync();
      if (tr_sweep) { TRACE(5 + 2 * jj); }
      if (!allreduce_small<T, T>(a, x, vec, l, &abort_flag)) return false;
      if (tr_sweep) { TRACE(6 + 2 * jj); }
      if (t < l) {
        Wts[t * k + jj] = vec[t];
        if (g == 0 && !(vec[t] == vec[t])) atomicOr(a.status, ST_NONFINITE_SWEEP);
      }
      lds_sync();
    }
    return true;
  };

  // projected gradient norm^2 on X^ = Q B (factor 2 dropped), with alpha F + beta
  // added for the regularized cost
  auto pgrad = [&](double& out) __attribute__((always_inline)) -> bool {
    __syncthreads();  // W and H written by other threads of this workgroup
    double s = 0.0;
    const T* Wrows;
    if constexpr (REGQ && !WG) Wrows = Ws;
    else Wrows = a.W + (size_t)r0 * k;
    for (int e = t; e < nr * k; e += NTH) {
      int rr = e / k, cc = e % k;
      const T* wr = Wrows + (size_t)rr * k;
      T gval = (T)0;
      for (int ii = 0; ii < k; ++ii) gval = fma(wr[ii], Vm[ii * k + cc], gval);
      if (rr < nrl) {
        for (int aa = 0; aa < l; ++aa) gval = fma(-Qs[rr * lq + aa], Tm[aa * k + cc], gval);
      } else {
        for (int aa = 0; aa < l; ++aa) gval = fma(-a.Q[(size_t)(r0 + rr) * l + aa], Tm[aa * k + cc], gval);
      }
      gval = fma((T)a.aw, wr[cc], gval) + (T)a.bw;
      T p = wr[cc] > (T)0 ? gval : (gval < (T)0 ? gval : (T)0);
      s += (double)p * (double)p;
    }
    for (int e = t; e < nc * k; e += NTH) {
      int cc = e / k, jj = e % k;
      T gval = (T)0;
      for (int ii = 0; ii < k; ++ii) gval = fma(Sm[jj * k + ii], Hp[(size_t)ii * ldH + cc], gval);
      for (int aa = 0; aa < l; ++aa) gval = fma(-Wts[aa * k + jj], Bp[(size_t)aa * ldB + cc], gval);
      T hv = Hp[(size_t)jj * ldH + cc];
      gval = fma((T)a.ah, hv, gval) + (T)a.bh;
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

  // --- schedule: every phase is instantiated once (keeps the kernel small
  // enough for the instruction cache); the order of phases is data ---------
  enum { PH_S = 0, PH_TV = 1, PH_H = 2, PH_W = 3, PH_PG = 4 };
  int pro[3], npro = 0, seq[5], nseq = 0;
  if (need_S) pro[npro++] = PH_S;
  if (need_pg || a.order == 1) pro[npro++] = PH_TV;
  if (need_pg) pro[npro++] = PH_PG;
  if (a.order == 0) {
    seq[nseq++] = PH_H; seq[nseq++] = PH_TV; seq[nseq++] = PH_W;
    if (need_S) seq[nseq++] = PH_S;
  } else {
    seq[nseq++] = PH_W;
    if (need_S) seq[nseq++] = PH_S;
    seq[nseq++] = PH_H; seq[nseq++] = PH_TV;
  }
  if (need_pg) seq[nseq++] = PH_PG;

  bool alive = true;
  double pg0 = 0.0, pg = 0.0;
  int done = 0;
  int pos = -npro;  // negative: prologue
  if (a.nsweeps <= 0 && npro == 0) pos = 0;
  while (alive && (pos < 0 || done < a.nsweeps)) {
    const int ph = pos < 0 ? pro[pos + npro] : seq[pos];
    const bool in_sweep = pos >= 0;
    tr_sweep = in_sweep && done == 0;
    switch (ph) {
      case PH_S:
        alive = s_exchange();
        if (tr_sweep) { TRACE(7 + 2 * k); }
        break;
      case PH_TV:
        alive = tv_exchange();
        if (tr_sweep) { TRACE(4); }
        break;
      case PH_H:
        h_phase();
        if (tr_sweep) { TRACE(3); }
        break;
      case PH_W:
        if constexpr (REGQ) alive = w_phase_reg();
        else alive = w_phase();
        if (tr_sweep) { TRACE(5 + 2 * k); }
        break;
      default: {
        double v = 0.0;
        alive = pgrad(v);
        if (in_sweep) pg = v;
        else { pg0 = v; pg = v; }
        break;
      }
    }
    if (!alive) break;
    ++pos;
    if (pos == 0 && !in_sweep) {
      TRACE(2);
      if (a.nsweeps <= 0) break;
    }
    if (in_sweep && pos == nseq) {
      if (tr_sweep) { TRACE(8 + 2 * k); }
      pos = 0;
      ++done;
      if (need_pg && pg < a.tol * pg0) break;
    }
  }
  tr_sweep = false;

  TRACE(9 + 2 * k);
#undef TRACE
  if (!alive) {
    if (t == 0) atomicOr(a.status, ST_TIMEOUT);
    return;
  }
  if constexpr (REGQ) {
    for (int e = t; e < k * nc; e += NTH) {
      const int r = e / nc, cc = e - (e / nc) * nc;
      a.H[(size_t)r * n + c0 + cc] = Hs[r * cp + cc];
    }
    if constexpr (!WG)
      for (int e = t; e < nr * k; e += NTH) a.W[(size_t)r0 * k + e] = Ws[e];
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

SweepShape plan_sweep(int64_t m, int64_t n, int l, int k, int dt, const Dev& d, bool need_pg) {
  SweepShape sh;
  int gmax = d.cus < 256 ? d.cus : 256;
  int G = 1;
  while (G * 2 <= gmax && ceil_div(m, G * 2) >= 16) G *= 2;
  sh.G = G;
  sh.GC = G < 16 ? G : 16;
  sh.GR = G / sh.GC;
  // with many workgroups, the per-column exchange of the register-slab W
  // phase is served by dedicated owner workgroups (one per 16-word block of
  // the l-vector) that hold no rows or columns, so that no workgroup's local
  // work sits on the exchange's critical path; dropped below if the Q slab
  // does not fit in registers
  const int xown = (G >= 64) ? (l * (dt == 0 ? 2 : 1) + 15) / 16 : 0;
  sh.xown = xown;
  sh.rows_per = ceil_div(m, G - xown);
  sh.cols_per = ceil_div(n, G - xown);
  sh.cb = l * k + k * k;
  sh.nt = NTH;
  const size_t es = dt == 0 ? 8 : 4;
  const int lq = l | 1;  // odd row stride: row-per-thread LDS reads hit distinct banks
  // Wts + U + vec + wcol + red2 (also the W staging area: 32 x 4*ceil(k/4))
  size_t red2 = 16 * (size_t)LPS;
  size_t stage = 32 * (size_t)(4 * ((k + 3) / 4));
  if (stage > red2) red2 = stage;
  if ((size_t)(LMAX + KMAX) * 8 > red2) red2 = (size_t)(LMAX + KMAX) * 8;  // T/V column staging
  if ((size_t)(8 * 8 * CQMAX + 5 * LPS) + 768 * 8 / es + 128 > red2) red2 = 8 * 8 * CQMAX + 5 * LPS + 768 * 8 / es + 128;  // W phase (REGQ)

  if ((size_t)NTH * 8 / es > red2) red2 = (size_t)NTH * 8 / es;  // pg reduction as doubles
  red2 = round_up(red2, 4);
  sh.red2_elems = (int)red2;
  // REGQ needs the W rows and the B and H columns in LDS besides the fixed part
  // (without the W rows when they stay in global memory)
  auto regq_extra_of = [&](bool wg) {
    return ((wg ? (size_t)0 : (size_t)(sh.rows_per + 1) * k) + (size_t)(l + k) * sh.cols_per) * es;
  };
  auto regq_fits_of = [&](bool wg) {
    const size_t fixed2 = ((size_t)l * k + (size_t)l * k + 2 * (size_t)k * k + LPS + sh.rows_per + red2) * es;
    return sh.rows_per <= 64 * RQ && l <= 8 * (dt == 0 ? 9 : CQMAX) && fixed2 + regq_extra_of(wg) + 1024 <= (size_t)d.max_lds;
  };
  sh.wglobal = 0;
  bool regq_fits = regq_fits_of(false);
  // the W-global variant exists for FP32 with the 12-column Q slab (l > 72)
  if (!regq_fits && dt != 0 && l > 72 && regq_fits_of(true)) {
    regq_fits = true;
    sh.wglobal = 1;
  }
  if (!regq_fits && sh.xown) {
    // without the owners the rows spread over all workgroups; the LDS-slab
    // path exchanges by the two-hop scheme over all workgroups
    sh.xown = 0;
    sh.rows_per = ceil_div(m, G);
    sh.cols_per = ceil_div(n, G);
    regq_fits = regq_fits_of(false);
  }
  const size_t regq_extra = regq_extra_of(sh.wglobal != 0);
  sh.alias_sv = (need_pg || regq_fits) ? 0 : 1;
  size_t fixed = ((size_t)l * k + (size_t)l * k + (size_t)(sh.alias_sv ? 1 : 2) * k * k + LPS + sh.rows_per + red2) * es;
  size_t budget = (size_t)d.max_lds - 1024;  // static shared + alignment slack
  size_t qrows = fixed < budget ? (budget - fixed) / ((size_t)lq * es) : 0;
  sh.regq = regq_fits ? 1 : 0;
  sh.rows_lds = sh.regq ? 0 : (int)((size_t)sh.rows_per < qrows ? sh.rows_per : qrows);
  sh.lds_bytes = fixed + (sh.regq ? regq_extra : (size_t)sh.rows_lds * lq * es);
  return sh;
}

size_t sweep_ws_words(const SweepShape& sh, int l) {
  (void)l;
  size_t slot = (size_t)LPS * 2;
  size_t cs = (size_t)((sh.cb + sh.GC - 1) / sh.GC) * 2;
  return 2 * 2 * (size_t)sh.G * slot + (size_t)sh.G * (size_t)sh.cb * 2 + 2 * 2 * (size_t)sh.G * cs;
}

hipError_t launch_sweep(const SweepShape& sh, int dt, const void* Q, const void* B, void* W, void* Wt, void* H,
                        int64_t m, int64_t n, int l, int k, int nsweeps, double tol, int gram_mode, int order, const Reg& reg,
                        u64* xbuf, double* stats, unsigned* status, u64* trace, hipStream_t s) {
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
  a.aw = reg.aw; a.ah = reg.ah; a.bw = reg.bw; a.bh = reg.bh;                                    \
  a.G = sh.G; a.GR = sh.GR; a.GC = sh.GC; a.rows_per = sh.rows_per; a.cols_per = sh.cols_per;  \
  a.rows_lds = sh.rows_lds; a.lq = l | 1; a.cb = sh.cb; a.red2_elems = sh.red2_elems;               \
  a.alias_sv = sh.alias_sv; a.trace = trace; a.xown = sh.xown;                                    \
  a.xs_part = xs_part; a.xs_row = xs_row; a.xb_part = xb_part; a.xb_row = xb_row;              \
  a.xb_fin = xb_fin; a.lpw = slot; a.cbw = cbw; a.csw = csw; a.stats = stats; a.status = status;
  if (dt == 0) {
    FILL_ARGS(double);
    void* args[] = {&a};
    const void* fn = sh.regq ? (const void*)sweep_kernel<double, true, 9, false> : (const void*)sweep_kernel<double, false, 1, false>;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds_bytes);
    if (e != hipSuccess) return e;
    return hipLaunchCooperativeKernel(fn, dim3(sh.G), dim3(NTH), args, (unsigned)sh.lds_bytes, s);
  } else {
    FILL_ARGS(float);
    void* args[] = {&a};
    const void* fn = !sh.regq ? (const void*)sweep_kernel<float, false, 1, false>
                     : (l <= 72) ? (const void*)sweep_kernel<float, true, 9, false>
                     : sh.wglobal ? (const void*)sweep_kernel<float, true, 12, true>
                                  : (const void*)sweep_kernel<float, true, 12, false>;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds_bytes);
    if (e != hipSuccess) return e;
    return hipLaunchCooperativeKernel(fn, dim3(sh.G), dim3(NTH), args, (unsigned)sh.lds_bytes, s);
  }
#undef FILL_ARGS
}

}  // namespace rnmf

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
constexpr int P1 = BLM + 1;

// LDS carving (floats): sweep state, then a scratch region reused by phases.
constexpr int OFF_WT = 0;                        // W~: BLM x BKM
constexpr int OFF_T = OFF_WT + BLM * BKM;        // T: BLM x BKM
constexpr int OFF_V = OFF_T + BLM * BKM;         // V: BKM x BKM
constexpr int OFF_S = OFF_V + BKM * BKM;         // S: BKM x BKM
constexpr int OFF_VEC = OFF_S + BKM * BKM;       // update vector: BLM
constexpr int RQW = 256;                         // most Q rows per tile (W phase)
constexpr int OFF_WS = OFF_VEC + BLM;            // lifted column tile: RQW
constexpr int OFF_RED = OFF_WS + RQW;            // doubles: 2 x BT (2 floats each)
constexpr int OFF_SCR = OFF_RED + 2 * 2 * BT;    // scratch
// scratch users (floats from OFF_SCR): the Cholesky works in place on the
// Gram (A, FP64, BLM x P1), then dL, dX, then L^{-T} as floats (BLM x BLM);
// the tiles of the other phases reuse the region from its start.
constexpr int SCR_CHOL_D = 2 * BLM * P1;
constexpr int SCR_AT = SCR_CHOL_D + 2 * 2 * BLM;
constexpr int SCR_FLOATS = SCR_AT + BLM * BLM;
constexpr int LDS_FLOATS = OFF_SCR + SCR_FLOATS;
static_assert(256 * 17 <= SCR_AT, "Cholesky QR apply tile below the factor");
static_assert(8 * BLM <= 2 * BT, "map-back partials fit the reduction buffer");
static_assert(OFF_RED % 2 == 0 && OFF_SCR % 2 == 0 && SCR_CHOL_D % 2 == 0, "FP64 alignment");
static_assert(256 * (NCX + 1) + NCX * BLM <= SCR_FLOATS, "X A tiles");
static_assert(MTZ * (4 * 64 + 1) + MTZ * BLM <= SCR_FLOATS, "X^T Q tiles");
static_assert(LDS_FLOATS * 4 <= 80 * 1024 - 256, "two workgroups per compute unit");

struct BDesc {
  rnmf_problem p;
  int32_t idx;  // position in the caller's array
  int32_t tc;   // X-pass column groups: 4, 8 or 16 (4 x 4 per thread)
  int32_t hct;  // H-phase tile: columns of B^T staged per tile (64, 128 or 256)
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

// Global memory is addressed through address-space-1 pointers: the phases
// are separate functions, and generic pointers would turn every access into a
// flat instruction (which also counts against the LDS wait counter).
typedef __attribute__((address_space(1))) const float gcf;
typedef __attribute__((address_space(1))) float gf;
template <typename T>
__device__ __forceinline__ gcf* G(const T* p) { return (gcf*)p; }
__device__ __forceinline__ gf* GW(float* p) { return (gf*)p; }

// Tile loads: every load of a thread is issued before the first one is
// waited for, so a tile costs one memory round trip, not one per element.
// Element e = t + s * BT (s < CNT) of the tile, so a tile holds at most
// CNT * BT elements (every caller sizes its tile to that); elements outside the tile
// read a valid address (the tile's first element) and are replaced by zero,
// so the loads carry no branches.
//   flat: a contiguous block of a packed matrix, base[e] for e < valid;
//         stored as rows of C at pitch dp;
//   pow2: an R x 2^lg tile of a row-major matrix with row pitch sp (2^lg <=
//         BT: a thread keeps its column and steps down BT >> lg rows).
template <int CNT>
__device__ __forceinline__ void flat_fetch(float (&v)[CNT], gcf* base, int valid, int t = threadIdx.x) {
#pragma unroll
  for (int s = 0; s < CNT; ++s) {
    const int e = t + s * BT;
    const bool ok = e < valid;
    const float x = base[ok ? e : 0];
    v[s] = ok ? x : 0.f;
  }
}
template <int CNT>
__device__ __forceinline__ void flat_store(const float (&v)[CNT], float* dst, int dp, int C, int total,
                                           int t = threadIdx.x) {
  // element t + s * BT: row i, column c; each step adds BT = qs * C + rs
  int i = t / C, c = t - (t / C) * C;
  const int qs = BT / C, rs = BT - (BT / C) * C;
#pragma unroll
  for (int s = 0; s < CNT; ++s) {
    if (t + s * BT < total) dst[i * dp + c] = v[s];
    c += rs;
    i += qs;
    if (c >= C) {
      c -= C;
      ++i;
    }
  }
}
// rows r0 .. r0 + R - 1 of a packed (rows x C) matrix into dst (pitch dp)
template <int CNT>
__device__ __forceinline__ void rows_load(float* dst, int dp, gcf* src, int64_t r0, int64_t rows, int R, int C) {
  float v[CNT];
  const int64_t left = rows - r0;
  flat_fetch<CNT>(v, src + r0 * C, (int)((left < R ? left : R) * C));
  flat_store<CNT>(v, dst, dp, C, R * C);
}
template <int CNT>
__device__ __forceinline__ void pow2_fetch(float (&v)[CNT], gcf* src, int64_t sp, int64_t r0, int64_t rows,
                                           int64_t c0, int64_t cols, int R, int lg) {
  const int t = threadIdx.x;
  const int C = 1 << lg;
  const int c = t & (C - 1), i0 = t >> lg, di = BT >> lg;
  const int64_t rl = rows - r0;
  const int rmax = (int)(rl < R ? rl : R);
  const bool colok = c0 + c < cols;
  gcf* base = src + r0 * sp + c0;
#pragma unroll
  for (int s = 0; s < CNT; ++s) {
    const int i = i0 + s * di;
    const bool ok = colok && i < rmax;
    const float x = base[ok ? (int64_t)i * sp + c : 0];
    v[s] = ok ? x : 0.f;
  }
}
template <int CNT>
__device__ __forceinline__ void pow2_store(const float (&v)[CNT], float* dst, int dp, int R, int lg) {
  const int t = threadIdx.x;
  const int C = 1 << lg;
#pragma unroll
  for (int s = 0; s < CNT; ++s) {
    const int e = t + s * BT;
    if (e < R * C) dst[(e >> lg) * dp + (e & (C - 1))] = v[s];
  }
}
// Fetches issued one tile ahead of their use: every load reads a valid
// element (a flat index past the tile's valid count reads the last valid
// element; a pow2 row or column past the matrix reads its last row or column)
// and carries no select, so no load is waited for before the tile is stored.
// The stores then write zero where the plain fetches above would have loaded
// zero.
template <int CNT>
__device__ __forceinline__ void flat_fetch_ahead(float (&v)[CNT], gcf* base, int valid) {
  const int t = threadIdx.x;
#pragma unroll
  for (int s = 0; s < CNT; ++s) {
    const int e = t + s * BT;
    v[s] = base[e < valid ? e : valid - 1];
  }
}
template <int CNT>
__device__ __forceinline__ void flat_store_valid(float (&v)[CNT], int valid, float* dst, int dp, int C, int total) {
  const int t = threadIdx.x;
#pragma unroll
  for (int s = 0; s < CNT; ++s)
    if (t + s * BT >= valid) v[s] = 0.f;
  flat_store<CNT>(v, dst, dp, C, total);
}
template <int CNT>
__device__ __forceinline__ void pow2_fetch_ahead(float (&v)[CNT], gcf* src, int64_t sp, int64_t r0, int64_t rows,
                                                 int64_t c0, int64_t cols, int R, int lg) {
  const int t = threadIdx.x;
  const int C = 1 << lg;
  const int c = t & (C - 1), i0 = t >> lg, di = BT >> lg;
  const int64_t rl = rows - r0;
  const int rmax = (int)(rl < R ? rl : R);
  gcf* base = src + r0 * sp + (c0 + c < cols ? c0 + c : cols - 1);
#pragma unroll
  for (int s = 0; s < CNT; ++s) {
    const int i = i0 + s * di;
    v[s] = base[(int64_t)(i < rmax ? i : rmax - 1) * sp];
  }
}
// pow2_store of a pow2_fetch_ahead tile: zero in the rows past rows - r0 and
// the columns past cols - c0.
template <int CNT>
__device__ __forceinline__ void pow2_store_valid(float (&v)[CNT], int64_t r0, int64_t rows, int64_t c0, int64_t cols,
                                                 float* dst, int dp, int R, int lg) {
  const int t = threadIdx.x;
  const int C = 1 << lg;
  const int c = t & (C - 1), i0 = t >> lg, di = BT >> lg;
  const int64_t rl = rows - r0;
  const int rmax = (int)(rl < R ? rl : R);
  const bool colok = c0 + c < cols;
#pragma unroll
  for (int s = 0; s < CNT; ++s)
    if (!(colok && i0 + s * di < rmax)) v[s] = 0.f;
  pow2_store<CNT>(v, dst, dp, R, lg);
}
__device__ __forceinline__ int ilog2(int x) { return 31 - __builtin_clz(x); }

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations
// (lgkmcnt) but leaves global loads and stores in flight, which a full
// __syncthreads() would drain.  Used where only LDS data is handed between
// threads; a full barrier follows wherever global data written by one thread
// is read by another.
__device__ __forceinline__ void lds_sync() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // vmcnt = 63, expcnt = 7, lgkmcnt = 0
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// dst[0 .. count) = src[0 .. count), eight loads in flight per thread.
__device__ __forceinline__ void copy_f(float* dst_, const float* src_, int64_t count) {
  gf* dst = GW(dst_);
  gcf* src = G(src_);
  const int t = threadIdx.x;
  for (int64_t b = 0; b < count; b += 8 * BT) {
    float v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int64_t e = b + t + (int64_t)s * BT;
      v[s] = e < count ? src[e] : 0.f;
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int64_t e = b + t + (int64_t)s * BT;
      if (e < count) dst[e] = v[s];
    }
  }
}

// Y (m x l) = X (m x n) A (n x l).  Thread (ti, tj): rows ti + tr * i,
// columns 4 tj + u.  Chunks (RT rows x NCX columns of X) run as one sequence;
// the next chunk's loads are in flight while the current one is multiplied.
template <int TC>
__device__ __noinline__ void xa_pass_t(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                                       const float* __restrict__ A, int l, float* __restrict__ Y_, float* scr) {
  const int t = threadIdx.x;
  constexpr int tr = BT / TC, RT = 4 * tr, LC = 4 * TC;
  constexpr int XCNT = RT * NCX / BT, ACNT = NCX * LC / BT;
  gf* Y = GW(Y_);
  float* Xs = scr;                      // RT x (NCX + 1)
  float* As = scr + RT * (NCX + 1);     // NCX x LC
  const int ti = t % tr, tj = t / tr;
  for (int e = t; e < NCX * LC; e += BT)
    if (e % LC >= l) As[e] = 0.f;       // padding columns, never written below
  const int nr = (int)((m + RT - 1) / RT), nc = (int)((n + NCX - 1) / NCX);
  float xv[XCNT], av[ACNT];
  int64_t fr0 = 0, fc0 = 0;  // the fetched chunk
  int avalid = 0;
#define XA_FETCH(qq)                                                                     \
  do {                                                                                   \
    fr0 = (int64_t)((qq) / nc) * RT;                                                     \
    fc0 = (int64_t)((qq) % nc) * NCX;                                                    \
    const int64_t left_ = n - fc0;                                                       \
    avalid = (int)((left_ < NCX ? left_ : NCX) * l);                                     \
    pow2_fetch_ahead<XCNT>(xv, G(X), ldx, fr0, m, fc0, n, RT, 5);                        \
    flat_fetch_ahead<ACNT>(av, G(A + fc0 * l), avalid);                                  \
  } while (0)
  XA_FETCH(0);
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[i][u] = 0.0;
  for (int qq = 0; qq < nr * nc; ++qq) {
    pow2_store_valid<XCNT>(xv, fr0, m, fc0, n, Xs, NCX + 1, RT, 5);
    flat_store_valid<ACNT>(av, avalid, As, LC, l, NCX * l);
    lds_sync();
    if (qq + 1 < nr * nc) XA_FETCH(qq + 1);
    float s[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) s[i][u] = 0.f;
#pragma unroll 2
    for (int c = 0; c < NCX; ++c) {
      float xr[4], ar[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xr[i] = Xs[(ti + tr * i) * (NCX + 1) + c];
#pragma unroll
      for (int u = 0; u < 4; ++u) ar[u] = As[c * LC + tj * 4 + u];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) s[i][u] = fmaf(xr[i], ar[u], s[i][u]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[i][u] += (double)s[i][u];
    lds_sync();
    if (qq % nc == nc - 1) {
      const int64_t r0 = (int64_t)(qq / nc) * RT;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = r0 + ti + tr * i;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = tj * 4 + u;
          if (r < m && j < l) Y[r * l + j] = (float)acc[i][u];
          acc[i][u] = 0.0;
        }
      }
    }
  }
  __syncthreads();  // Y is read next by other threads of the workgroup
#undef XA_FETCH
}

__device__ __noinline__ void xa_pass(const float* X, int64_t ldx, int64_t m, int64_t n, const float* A, int l,
                                     float* Y, int tc, float* scr) {
  if (tc == 4) xa_pass_t<4>(X, ldx, m, n, A, l, Y, scr);
  else if (tc == 8) xa_pass_t<8>(X, ldx, m, n, A, l, Y, scr);
  else xa_pass_t<16>(X, ldx, m, n, A, l, Y, scr);
}

// Z (n x l) = X^T Q, and optionally B = Z^T (l x n).  Thread (ti, tj): Z rows
// (X columns) c0 + ti + tz * i, columns 4 tj + u.  Chunks (MTZ rows x NZ
// columns of X) run as one sequence, the next one's loads in flight.
template <int TC>
__device__ __noinline__ void xtq_pass_t(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                                        const float* __restrict__ Q, int l, float* __restrict__ Z_,
                                        float* __restrict__ Bout_, float* scr) {
  const int t = threadIdx.x;
  constexpr int tz = BT / TC, NZ = 4 * tz, LC = 4 * TC;
  constexpr int XCNT = MTZ * NZ / BT, QCNT = MTZ * LC / BT;
  gf* Z = GW(Z_);
  gf* Bout = Bout_ ? GW(Bout_) : nullptr;
  float* Xs = scr;                    // MTZ x (NZ + 1)
  float* Qs = scr + MTZ * (NZ + 1);   // MTZ x LC
  const int ti = t % tz, tj = t / tz;
  const int lgz = ilog2(NZ);
  for (int e = t; e < MTZ * LC; e += BT)
    if (e % LC >= l) Qs[e] = 0.f;     // padding columns, never written below
  const int ncb = (int)((n + NZ - 1) / NZ), nrb = (int)((m + MTZ - 1) / MTZ);
  float xv[XCNT], qv[QCNT];
  int64_t fr0 = 0, fc0 = 0;  // the fetched chunk
  int qvalid = 0;
#define XTQ_FETCH(qq)                                                                    \
  do {                                                                                   \
    fc0 = (int64_t)((qq) / nrb) * NZ;                                                    \
    fr0 = (int64_t)((qq) % nrb) * MTZ;                                                   \
    const int64_t left_ = m - fr0;                                                       \
    qvalid = (int)((left_ < MTZ ? left_ : MTZ) * l);                                     \
    pow2_fetch_ahead<XCNT>(xv, G(X), ldx, fr0, m, fc0, n, MTZ, lgz);                     \
    flat_fetch_ahead<QCNT>(qv, G(Q + fr0 * l), qvalid);                                  \
  } while (0)
  XTQ_FETCH(0);
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[i][u] = 0.0;
  for (int qq = 0; qq < ncb * nrb; ++qq) {
    pow2_store_valid<XCNT>(xv, fr0, m, fc0, n, Xs, NZ + 1, MTZ, lgz);
    flat_store_valid<QCNT>(qv, qvalid, Qs, LC, l, MTZ * l);
    lds_sync();
    if (qq + 1 < ncb * nrb) XTQ_FETCH(qq + 1);
    float s[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) s[i][u] = 0.f;
#pragma unroll 2
    for (int rr = 0; rr < MTZ; ++rr) {
      float xr[4], qr[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xr[i] = Xs[rr * (NZ + 1) + ti + tz * i];
#pragma unroll
      for (int u = 0; u < 4; ++u) qr[u] = Qs[rr * LC + tj * 4 + u];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) s[i][u] = fmaf(xr[i], qr[u], s[i][u]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[i][u] += (double)s[i][u];
    lds_sync();
    if (qq % nrb == nrb - 1) {
      const int64_t c0 = (int64_t)(qq / nrb) * NZ;
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
          acc[i][u] = 0.0;
        }
      }
    }
  }
  __syncthreads();  // Z is read next by other threads of the workgroup
#undef XTQ_FETCH
}

__device__ __noinline__ void xtq_pass(const float* X, int64_t ldx, int64_t m, int64_t n, const float* Q, int l,
                                      float* Z, float* Bout, int tc, float* scr) {
  if (tc == 4) xtq_pass_t<4>(X, ldx, m, n, Q, l, Z, Bout, scr);
  else if (tc == 8) xtq_pass_t<8>(X, ldx, m, n, Q, l, Z, Bout, scr);
  else xtq_pass_t<16>(X, ldx, m, n, Q, l, Z, Bout, scr);
}

// ---------------------------------------------------------------------------
// X passes on bf16 matrix cores (v_mfma_f32_16x16x32_bf16): X stays FP32 in
// memory and is rounded to bfloat16 (nearest even) as a chunk is staged in
// LDS; the small operand (A or Q) is split into hi = bf16(a) and
// lo = bf16(a - hi), two products per tile, so only X is rounded.  Lane
// (i, g) = (lane % 16, lane / 16) holds row i of the A operand at k = 8g ..
// 8g + 7 and column i of the B operand at the same k; D[4g + e][i] comes
// back in element e.  Products accumulate in FP32 over the whole reduction.
// Chunks are 128 x 64 elements of X (32 KB); the next chunk's loads are in
// flight while the current one is multiplied.  Operand tiles in LDS are
// bfloat16 rows of 64 k values at a pitch of 72 (16-byte fragments, rows
// 144 bytes apart).
// ---------------------------------------------------------------------------
typedef __bf16 bfx8 __attribute__((ext_vector_type(8)));
typedef float fx4 __attribute__((ext_vector_type(4)));
constexpr int MKC = 64;             // k per chunk (two MFMA steps)
constexpr int MKP = MKC + 8;        // LDS pitch (bfloat16 elements)
constexpr int MRB = 128;            // X rows (xa) or X columns (xtq) per block
constexpr int MXC = MRB * MKC / BT; // X values per thread per chunk
constexpr int MAC = BLM * MKC / BT; // operand values per thread per chunk
static_assert((MRB + 2 * BLM) * MKP * 2 <= SCR_FLOATS * 4, "bf16 chunk tiles fit the scratch");

__device__ __forceinline__ unsigned short bf16_rn(float f) {
  unsigned b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (unsigned short)(b >> 16);
}
__device__ __forceinline__ fx4 mfma_bf16(bfx8 a, bfx8 b, fx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Operand chunk: rows k0 .. k0 + MKC - 1 of a packed (rows x l) matrix, stored
// transposed (column j at Oh + j * MKP) as hi and lo planes; rows past the
// matrix are zero.  Element e = t + s BT of the chunk is row e / l, column e % l.
__device__ __forceinline__ void op_fetch(float (&v)[MAC], gcf* base, int64_t k0, int64_t rows, int l, int t) {
#pragma unroll
  for (int s = 0; s < MAC; ++s) {
    const int e = t + s * BT;
    const int kk = e / l, j = e - (e / l) * l;
    int64_t r = k0 + kk;
    if (r >= rows) r = rows - 1;
    v[s] = (e < MKC * l) ? base[r * l + j] : 0.f;
  }
}
__device__ __forceinline__ void op_store(const float (&v)[MAC], unsigned short* Oh, unsigned short* Ol, int64_t k0,
                                         int64_t rows, int l) {
  const int t = threadIdx.x;
#pragma unroll
  for (int s = 0; s < MAC; ++s) {
    const int e = t + s * BT;
    if (e < MKC * l) {
      const int kk = e / l, j = e - (e / l) * l;
      const bool ok = k0 + kk < rows;
      const unsigned short h = bf16_rn(v[s]);
      const unsigned short lo = bf16_rn(v[s] - __uint_as_float((unsigned)h << 16));
      Oh[j * MKP + kk] = ok ? h : (unsigned short)0;
      Ol[j * MKP + kk] = ok ? lo : (unsigned short)0;
    }
  }
}

// Y (m x l) = X (m x n) A (n x l).  Block of 128 rows: wave w owns row tiles
// w and w + 4; chunks of 64 columns of X (and 64 rows of A) run in sequence.
__device__ __noinline__ void xa_pass_bf16(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                                          const float* __restrict__ A, int l, float* __restrict__ Y_, float* scr) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, i = lane & 15, g = lane >> 4;
  gf* Y = GW(Y_);
  gcf* Xg = G(X);
  gcf* Ag = G(A);
  unsigned short* Xs = (unsigned short*)scr;  // MRB x MKP
  unsigned short* Oh = Xs + MRB * MKP;         // BLM x MKP
  unsigned short* Ol = Oh + BLM * MKP;
  const int LT = (l + 15) / 16;
  for (int e = t; e < BLM * MKP; e += BT)
    if (e / MKP >= l) { Oh[e] = 0; Ol[e] = 0; }  // operand columns past l, never written below
  const int nr = (int)((m + MRB - 1) / MRB), nc = (int)((n + MKC - 1) / MKC);
  float xv[MXC], av[MAC];
  int64_t fr0 = 0, fc0 = 0;
  auto fetch = [&](int qq) {
    fr0 = (int64_t)(qq / nc) * MRB;
    fc0 = (int64_t)(qq % nc) * MKC;
    // an opaque copy of the thread index keeps the per-element offsets out of
    // the loop-invariant set (they would be hoisted and spilled otherwise)
    int tt = t;
    __asm__ volatile("" : "+v"(tt));
#pragma unroll
    for (int s = 0; s < MXC; ++s) {
      const int e = tt + s * BT;
      int64_t r = fr0 + (e >> 6), c = fc0 + (e & 63);
      if (r >= m) r = m - 1;
      if (c >= n) c = n - 1;
      xv[s] = Xg[r * ldx + c];
    }
    op_fetch(av, Ag, fc0, n, l, tt);
  };
  fetch(0);
  fx4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = fx4{0.f, 0.f, 0.f, 0.f};
  for (int qq = 0; qq < nr * nc; ++qq) {
#pragma unroll
    for (int s = 0; s < MXC; ++s) {
      const int e = t + s * BT;
      const bool ok = fr0 + (e >> 6) < m && fc0 + (e & 63) < n;
      Xs[(e >> 6) * MKP + (e & 63)] = ok ? bf16_rn(xv[s]) : (unsigned short)0;
    }
    op_store(av, Oh, Ol, fc0, n, l);
    const int64_t r0 = fr0;
    lds_sync();
    if (qq + 1 < nr * nc) fetch(qq + 1);
#pragma unroll
    for (int kk = 0; kk < MKC; kk += 32) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const bfx8 xa = *(const bfx8*)(Xs + (16 * (wave + 4 * rt) + i) * MKP + kk + 8 * g);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
          if (ct < LT) {
            const bfx8 h = *(const bfx8*)(Oh + (16 * ct + i) * MKP + kk + 8 * g);
            const bfx8 lo = *(const bfx8*)(Ol + (16 * ct + i) * MKP + kk + 8 * g);
            acc[rt][ct] = mfma_bf16(xa, h, acc[rt][ct]);
            acc[rt][ct] = mfma_bf16(xa, lo, acc[rt][ct]);
          }
      }
    }
    lds_sync();
    if (qq % nc == nc - 1) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t r = r0 + 16 * (wave + 4 * rt) + 4 * g + e;
            const int c = 16 * ct + i;
            if (ct < LT && r < m && c < l) Y[r * l + c] = acc[rt][ct][e];
          }
          acc[rt][ct] = fx4{0.f, 0.f, 0.f, 0.f};
        }
    }
  }
  __syncthreads();  // Y is read next by other threads of the workgroup
}

// Z (n x l) = X^T Q, and optionally B = Z^T (l x n).  Block of 128 columns of
// X: wave w owns column tiles w and w + 4; chunks of 64 rows of X (and of Q)
// run in sequence.  The X chunk is stored transposed (column c of X at
// Xt + c * MKP), so both operands are read as contiguous k fragments.
__device__ __noinline__ void xtq_pass_bf16(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                                           const float* __restrict__ Q, int l, float* __restrict__ Z_,
                                           float* __restrict__ Bout_, float* scr) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, i = lane & 15, g = lane >> 4;
  gf* Z = GW(Z_);
  gf* Bout = Bout_ ? GW(Bout_) : nullptr;
  gcf* Xg = G(X);
  gcf* Qg = G(Q);
  unsigned short* Xt = (unsigned short*)scr;  // MRB x MKP
  unsigned short* Oh = Xt + MRB * MKP;         // BLM x MKP
  unsigned short* Ol = Oh + BLM * MKP;
  const int LT = (l + 15) / 16;
  for (int e = t; e < BLM * MKP; e += BT)
    if (e / MKP >= l) { Oh[e] = 0; Ol[e] = 0; }
  const int ncb = (int)((n + MRB - 1) / MRB), nrb = (int)((m + MKC - 1) / MKC);
  float xv[MXC], qv[MAC];
  int64_t fr0 = 0, fc0 = 0;
  // element e = t + s BT of an X chunk: row e / MRB, column e % MRB (along the row)
  auto fetch = [&](int qq) {
    fc0 = (int64_t)(qq / nrb) * MRB;
    fr0 = (int64_t)(qq % nrb) * MKC;
    int tt = t;
    __asm__ volatile("" : "+v"(tt));
#pragma unroll
    for (int s = 0; s < MXC; ++s) {
      const int e = tt + s * BT;
      int64_t r = fr0 + e / MRB, c = fc0 + (e % MRB);
      if (r >= m) r = m - 1;
      if (c >= n) c = n - 1;
      xv[s] = Xg[r * ldx + c];
    }
    op_fetch(qv, Qg, fr0, m, l, tt);
  };
  fetch(0);
  fx4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = fx4{0.f, 0.f, 0.f, 0.f};
  for (int qq = 0; qq < ncb * nrb; ++qq) {
#pragma unroll
    for (int s = 0; s < MXC; ++s) {
      const int e = t + s * BT;
      const int rr = e / MRB, cc = e % MRB;
      const bool ok = fr0 + rr < m && fc0 + cc < n;
      Xt[cc * MKP + rr] = ok ? bf16_rn(xv[s]) : (unsigned short)0;
    }
    op_store(qv, Oh, Ol, fr0, m, l);
    const int64_t c0 = fc0;
    lds_sync();
    if (qq + 1 < ncb * nrb) fetch(qq + 1);
#pragma unroll
    for (int kk = 0; kk < MKC; kk += 32) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const bfx8 xa = *(const bfx8*)(Xt + (16 * (wave + 4 * rt) + i) * MKP + kk + 8 * g);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
          if (ct < LT) {
            const bfx8 h = *(const bfx8*)(Oh + (16 * ct + i) * MKP + kk + 8 * g);
            const bfx8 lo = *(const bfx8*)(Ol + (16 * ct + i) * MKP + kk + 8 * g);
            acc[rt][ct] = mfma_bf16(xa, h, acc[rt][ct]);
            acc[rt][ct] = mfma_bf16(xa, lo, acc[rt][ct]);
          }
      }
    }
    lds_sync();
    if (qq % nrb == nrb - 1) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int64_t c = c0 + 16 * (wave + 4 * rt) + 4 * g + e;
            const int j = 16 * ct + i;
            if (ct < LT && c < n && j < l) {
              Z[c * l + j] = acc[rt][ct][e];
              if (Bout) Bout[(int64_t)j * n + c] = acc[rt][ct][e];
            }
          }
          acc[rt][ct] = fx4{0.f, 0.f, 0.f, 0.f};
        }
    }
  }
  __syncthreads();  // Z is read next by other threads of the workgroup
}

// Cholesky of the Gram in A (l x l, lower triangle and diagonal, in LDS,
// pitch P1; the strict upper triangle zero) in place, with the inverse fused,
// in blocks of 8 columns (the scheme of the single-problem factorisation).
// On exit A holds L in its strict lower triangle and X = L^{-1} transposed in
// its strict upper triangle; dL, dX the diagonals.  Returns false if a pivot
// is not positive and finite.
__device__ __noinline__ bool chol_lds(double* A, double* dL, double* dX, int* flag, int l) {
  constexpr int CB = 8;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  for (int i = t; i < l; i += BT) dX[i] = 1.0;
  if (t == 0) *flag = 0;
  lds_sync();
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
    lds_sync();
    if (*flag) return false;  // the same value in every thread
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
    lds_sync();
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
    lds_sync();
  }
  return true;
}

// FP64 Gram Y^T Y of Y (rows x l, global) into A (lower triangle and
// diagonal; strict upper triangle zero; pitch P1).  The row tiles are staged
// in the same LDS region, which A overwrites only after the last tile.
__device__ __noinline__ void gram_y(const float* __restrict__ Y, int64_t rows, int l, double* A, float* scr) {
  const int t = threadIdx.x;
  float* Ys = scr;  // GT x P1
  const int ga = t % 16, gb = t / 16;
  double g[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int u = 0; u < 4; ++u) g[i][u] = 0.0;
  const int ntile = (int)((rows + GT - 1) / GT);
  float yv[16];
  flat_fetch<16>(yv, G(Y), (int)((rows < GT ? rows : GT) * l));
  for (int it = 0; it < ntile; ++it) {
    const int64_t r0 = (int64_t)it * GT;
    flat_store<16>(yv, Ys, P1, l, GT * l);
    lds_sync();
    if (it + 1 < ntile) {
      const int64_t left = rows - (r0 + GT);
      flat_fetch<16>(yv, G(Y + (r0 + GT) * l), (int)((left < GT ? left : GT) * l));
    }
    for (int rr = 0; rr < GT; ++rr) {  // (padding entries feed unstored sums)
      double ya[4], yb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ya[i] = (double)Ys[rr * P1 + ga + 16 * i];
        yb[i] = (double)Ys[rr * P1 + gb + 16 * i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) g[i][u] = fma(ya[i], yb[u], g[i][u]);
    }
    lds_sync();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int a = ga + 16 * i, b = gb + 16 * u;
      if (a < l && b < l) A[a * P1 + b] = (b <= a) ? g[i][u] : 0.0;
    }
  lds_sync();
}

// One Cholesky QR pass on Y (rows x l, global, in place): FP64 Gram, Cholesky
// with the inverse fused (when it breaks down, the Gram is recomputed and the
// diagonal shifted by 11 (rows l + l (l + 1)) u tr(G), Fukaya et al.), then
// Y <- Y L^{-T}.  Returns 0 (plain), 1 (after the shift) or 2 (failed).
__device__ __noinline__ int cholqr_pass(float* __restrict__ Y_, int64_t rows, int l, int tc, float* scr, int* flag) {
  const int t = threadIdx.x;
  float* Y = Y_;
  gf* Yw = GW(Y_);
  double* A = (double*)scr;
  double* dL = (double*)(scr + SCR_CHOL_D);
  double* dX = dL + BLM;
  float* At = scr + SCR_AT;
  int code = -1;
  for (int attempt = 0; attempt < 2 && code < 0; ++attempt) {
    gram_y(Y, rows, l, A, scr);
    if (attempt == 1) {
      double trace = 0.0;
      for (int i = 0; i < l; ++i) trace += A[i * P1 + i];  // same order in every thread
      const double shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * 1.1102230246251565e-16 * trace;
      lds_sync();
      for (int i = t; i < l; i += BT) A[i * P1 + i] += shift;
      lds_sync();
    }
    if (chol_lds(A, dL, dX, flag, l)) code = attempt;
  }
  if (code < 0) return 2;
  // At(a, c) = X(c, a) = L^{-1}(c, a) for a <= c, so Q = Y At
  for (int e = t; e < l * l; e += BT) {
    const int a = e / l, c = e - (e / l) * l;
    At[a * BLM + c] = (float)((a == c) ? dX[c] : (a < c ? A[a * P1 + c] : 0.0));
  }
  lds_sync();
  // Q = Y At in place, RT rows per tile (pitch l + 1, below At)
  {
    const int tr = BT / tc, RT = 4 * tr, pa = l + 1;
    float* Ys = scr;
    const int ti = t % tr, tj = t / tr;
    const int ntile = (int)((rows + RT - 1) / RT);
    float yv[16];
    flat_fetch<16>(yv, G(Y), (int)((rows < RT ? rows : RT) * l));
    for (int it = 0; it < ntile; ++it) {
      const int64_t r0 = (int64_t)it * RT;
      flat_store<16>(yv, Ys, pa, l, RT * l);
      lds_sync();
      if (it + 1 < ntile) {  // rows of the next tile are not written before they are loaded
        const int64_t left = rows - (r0 + RT);
        flat_fetch<16>(yv, G(Y + (r0 + RT) * l), (int)((left < RT ? left : RT) * l));
      }
      float s[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 4; ++u) s[i][u] = 0.f;
      for (int a = 0; a < l; ++a) {
        float yr[4], ar[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) yr[i] = Ys[(ti + tr * i) * pa + a];
#pragma unroll
        for (int u = 0; u < 4; ++u) ar[u] = At[a * BLM + tj * 4 + u];  // (padding: unstored sums)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int u = 0; u < 4; ++u) s[i][u] = fmaf(yr[i], ar[u], s[i][u]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t r = r0 + ti + tr * i;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = tj * 4 + u;
          if (r < rows && c < l) Yw[r * l + c] = s[i][u];
        }
      }
      lds_sync();
    }
  }
  __syncthreads();  // Y is read next by other threads of the workgroup
  return code;
}

// Cholesky QR2 (a third pass after a shifted one).  Returns status bits.
__device__ __noinline__ unsigned cholqr2(float* Y, int64_t rows, int l, int tc, float* scr, int* flag) {
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

// S = W^T W (k x k, FP64 sums) into Ss (pitch BKM); W is held by columns
// (Wc: k x m, column c at Wc + c ldw).
__device__ __noinline__ void gram_w(const float* __restrict__ Wc, int64_t m, int64_t ldw, int k, float* Ss,
                                    float* scr) {
  const int t = threadIdx.x;
  float* Wsh = scr;  // GT x (BKM + 1)
  const int gi = t % 16, gj = t / 16;
  double s[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  gcf* W = G(Wc);
  // element e = t + u BT of a tile: column e / GT, row r0 + e % GT (GT
  // consecutive floats of one column per 64 lanes).  The next tile's loads
  // are in flight while the current one is used; a position past the rows or
  // columns reads a valid element instead and is zeroed when stored.
  constexpr int NU = GT * BKM / BT;
  float wv[NU];
  auto fetch = [&](int64_t r0) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = t + u * BT;
      const int c = e / GT;
      const int64_t r = r0 + (e % GT);
      wv[u] = W[(int64_t)(c < k ? c : k - 1) * ldw + (r < m ? r : m - 1)];
    }
  };
  fetch(0);
  for (int64_t r0 = 0; r0 < m; r0 += GT) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int e = t + u * BT;
      const int c = e / GT, r = e % GT;
      Wsh[r * (BKM + 1) + c] = (c < k && r0 + r < m) ? wv[u] : 0.f;
    }
    lds_sync();
    if (r0 + GT < m) fetch(r0 + GT);
    // entries past k are read from the row's padding and feed only sums
    // that are never stored: the loads carry no condition (a load under a
    // condition is waited for inside its own branch)
    for (int rr = 0; rr < GT; ++rr) {
      double a[2], b[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int i = gi + 16 * u, j = gj + 16 * u;
        a[u] = (double)Wsh[rr * (BKM + 1) + i];
        b[u] = (double)Wsh[rr * (BKM + 1) + j];
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) s[u][v] = fma(a[u], b[v], s[u][v]);
    }
    lds_sync();
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int i = gi + 16 * u, j = gj + 16 * v;
      if (i < k && j < k) Ss[i * BKM + j] = (float)s[u][v];
    }
  lds_sync();
}

// W (m x k, rows) <-> Wc (k x m, columns), in tiles of GT rows through LDS so
// that both sides are read and written along contiguous runs.
__device__ __noinline__ void w_to_columns(float* __restrict__ Wc, const float* __restrict__ W, int64_t m,
                                          int64_t ldw, int k, float* scr) {
  const int t = threadIdx.x;
  float* Wsh = scr;  // GT x (BKM + 1)
  gf* D = GW(Wc);
  for (int64_t r0 = 0; r0 < m; r0 += GT) {
    rows_load<8>(Wsh, BKM + 1, G(W), r0, m, GT, k);
    lds_sync();
    for (int e = t; e < GT * k; e += BT) {
      const int c = e / GT, r = e % GT;
      if (r0 + r < m) D[(int64_t)c * ldw + r0 + r] = Wsh[r * (BKM + 1) + c];
    }
    lds_sync();
  }
}
__device__ __noinline__ void w_from_columns(float* __restrict__ W, const float* __restrict__ Wc, int64_t m,
                                            int64_t ldw, int k, float* scr) {
  const int t = threadIdx.x;
  float* Wsh = scr;  // GT x (BKM + 1)
  gcf* S = G(Wc);
  gf* D = GW(W);
  for (int64_t r0 = 0; r0 < m; r0 += GT) {
    for (int e = t; e < GT * k; e += BT) {
      const int c = e / GT, r = e % GT;
      if (r0 + r < m) Wsh[r * (BKM + 1) + c] = S[(int64_t)c * ldw + r0 + r];
    }
    lds_sync();
    const int64_t left = m - r0;
    const int cnt = (int)((left < GT ? left : GT) * k);
    for (int e = t; e < cnt; e += BT) D[r0 * k + e] = Wsh[(e / k) * (BKM + 1) + (e % k)];
    lds_sync();
  }
}

// W~ = Q^T W (l x k, FP64 sums) into Wts (pitch BKM).
__device__ __noinline__ void init_wt(const float* __restrict__ Q, const float* __restrict__ W, int64_t m, int l, int k, float* Wts,
                        float* scr) {
  const int t = threadIdx.x;
  float* Qsh = scr;                  // GT x P1
  float* Wsh = scr + GT * P1;        // GT x (BKM + 1)
  const int ga = t % 16, gj = t / 16;
  double s[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i) s[i][0] = s[i][1] = 0.0;
  for (int64_t r0 = 0; r0 < m; r0 += GT) {
    rows_load<16>(Qsh, P1, G(Q), r0, m, GT, l);
    rows_load<8>(Wsh, BKM + 1, G(W), r0, m, GT, k);
    lds_sync();
    for (int rr = 0; rr < GT; ++rr) {  // (padding entries feed unstored sums)
      double qa[4], wj[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) qa[i] = (double)Qsh[rr * P1 + ga + 16 * i];
#pragma unroll
      for (int u = 0; u < 2; ++u) wj[u] = (double)Wsh[rr * (BKM + 1) + gj + 16 * u];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int u = 0; u < 2; ++u) s[i][u] = fma(qa[i], wj[u], s[i][u]);
    }
    lds_sync();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int a = ga + 16 * i, j = gj + 16 * u;
      if (a < l && j < k) Wts[a * BKM + j] = (float)s[i][u];
    }
  lds_sync();
}

// Rows of H (Algorithm 1, H rule with S = W^T W), one lane per column c of H:
// the lane holds H(:, c) and the gradient g = R(c, :) - H(:, c)^T S in
// registers and runs the Gauss-Seidel chain over j on its own (the columns of
// H are independent); W~, S and the reciprocal scales are LDS broadcasts.
// KB >= k: W~ and S are zero beyond k, so the extra rows have scale zero and
// are skipped like any zero-scale row.  B^T is staged through LDS in tiles of
// NCT columns (64, 128 or 256: a tuning choice per sketch-width class, with
// NCT (l + 1) <= SCR_FLOATS; one lane per column, so NCT < BT leaves lanes
// idle while a wider tile takes two rounds of loads).  FP64 gradient; H
// entries are FP32 values (every update is rounded to FP32 before it is
// used).
template <int KB>
__device__ __forceinline__ void h_phase_t(const float* __restrict__ Bt, float* __restrict__ H, int64_t n, int l, int k,
                                       const float* Wts, const float* Ss, double* rinv, float* scr, int NCT) {
  const int t = threadIdx.x;
  gcf* Hg = G(H);
  gf* Hw = GW(H);
  const int pz = l + 1;
  float* Zs = scr;  // NCT x (l + 1)
  if (t < KB) {
    const double d = (double)Ss[t * BKM + t];
    rinv[t] = (t < k && d > 0.0) ? 1.0 / d : 0.0;
  }
  for (int64_t c0 = 0; c0 < n; c0 += NCT) {
    {
      // The thread index goes through an empty asm statement once per tile,
      // so the tile's 32 element positions are recomputed here rather than
      // hoisted out of the loop, where they would stay live across the
      // column updates (and be spilled).
      int tt = t;
      asm volatile("" : "+v"(tt));
      float zv[32];
      const int64_t left = n - c0;
      const int valid = (int)((left < NCT ? left : NCT) * l);
      // rounds of 32 loads per thread (two at most: NCT l <= SCR_FLOATS)
      for (int e0 = 0; e0 < valid; e0 += 32 * BT) {
        flat_fetch<32>(zv, G(Bt + c0 * l + e0), valid - e0, tt);
        flat_store<32>(zv, Zs, pz, l, NCT * l, tt + e0);
      }
    }
    lds_sync();
    const int64_t c = c0 + t;
    if (t < NCT && c < n) {
      float h[KB];
      double g[KB];
#pragma unroll
      for (int j = 0; j < KB; ++j) {
        h[j] = j < k ? Hg[(int64_t)j * n + c] : 0.f;
        g[j] = 0.0;
      }
      for (int a = 0; a < l; ++a) {  // R(c, j) = sum_a B(a, c) W~(a, j)
        const double bz = (double)Zs[t * pz + a];
#pragma unroll
        for (int j = 0; j < KB; ++j) g[j] = fma(bz, (double)Wts[a * BKM + j], g[j]);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
      }
      // (the compiler fences keep each step's LDS broadcasts inside the step,
      // so the unrolled loops do not hoist KB x KB values into registers)
#pragma unroll
      for (int p = 0; p < KB; ++p) {  // g(j) -= sum_p S(p, j) H(p, c)
        const double hp = (double)h[p];
#pragma unroll
        for (int j = 0; j < KB; ++j) g[j] = fma(-(double)Ss[p * BKM + j], hp, g[j]);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
      }
#pragma unroll
      for (int j = 0; j < KB; ++j) {  // Gauss-Seidel over the rows
        const double rd = rinv[j];
        if (rd > 0.0) {
          const float hn = clipf((float)fma(g[j], rd, (double)h[j]));
          const double delta = (double)hn - (double)h[j];
          h[j] = hn;
#pragma unroll
          for (int p = 0; p < KB; ++p) g[p] = fma(-(double)Ss[j * BKM + p], delta, g[p]);
        }
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
      }
#pragma unroll
      for (int j = 0; j < KB; ++j)
        if (j < k) Hw[(int64_t)j * n + c] = h[j];
    }
    lds_sync();
  }
  __syncthreads();  // H is read next by other threads of the workgroup
}

__device__ __forceinline__ void h_phase(const float* Bt, float* H, int64_t n, int l, int k, const float* Wts,
                                     const float* Ss, double* rinv, float* scr, int nct) {
  if (k <= 8) h_phase_t<8>(Bt, H, n, l, k, Wts, Ss, rinv, scr, nct);
  else if (k <= 16) h_phase_t<16>(Bt, H, n, l, k, Wts, Ss, rinv, scr, nct);
  else if (k <= 24) h_phase_t<24>(Bt, H, n, l, k, Wts, Ss, rinv, scr, nct);
  else h_phase_t<32>(Bt, H, n, l, k, Wts, Ss, rinv, scr, nct);
}

// T = B H^T (l x k) and V = H H^T (k x k) over 64-column tiles: FP32 within a
// tile, FP64 across tiles.  Threads 0..127: T entries (ga + 16 i, gj + 8 u);
// threads 128..191: V entries (vi + 8 p, vj + 8 q).
__device__ __forceinline__ void tv_phase(const float* __restrict__ Bt, const float* __restrict__ H, int64_t n, int l, int k, float* Ts,
                         float* Vs, float* scr) {
  const int t = threadIdx.x;
  float* Zs = scr;                // 64 (columns) x P1
  float* Hs = scr + 64 * P1;      // BKM x 65
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[i][u] = 0.0;
  // the next tile's loads are in flight while the current one is used
  float zv[16], hv[8];
  int zvalid = 0;
  auto fetch = [&](int64_t c0) {
    const int64_t left = n - c0;
    zvalid = (int)((left < 64 ? left : 64) * l);
    flat_fetch_ahead<16>(zv, G(Bt + c0 * l), zvalid);
    pow2_fetch_ahead<8>(hv, G(H), n, 0, k, c0, n, k, 6);
  };
  fetch(0);
  for (int64_t c0 = 0; c0 < n; c0 += 64) {
    flat_store_valid<16>(zv, zvalid, Zs, P1, l, 64 * l);
    pow2_store_valid<8>(hv, 0, k, c0, n, Hs, 65, k, 6);
    lds_sync();
    if (c0 + 64 < n) fetch(c0 + 64);
    float s[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int u = 0; u < 4; ++u) s[i][u] = 0.f;
    if (t < 128) {
      const int ga = t % 16, gj = t / 16;
      for (int c = 0; c < 64; ++c) {  // (padding entries feed unstored sums)
        float za[4], hj[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) za[i] = Zs[c * P1 + ga + 16 * i];
#pragma unroll
        for (int u = 0; u < 4; ++u) hj[u] = Hs[(gj + 8 * u) * 65 + c];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int u = 0; u < 4; ++u) s[i][u] = fmaf(za[i], hj[u], s[i][u]);
      }
    } else if (t < 192) {
      const int v = t - 128, vi = v % 8, vj = v / 8;
      for (int c = 0; c < 64; ++c) {  // (padding entries feed unstored sums)
        float hi[4], hj[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          hi[i] = Hs[(vi + 8 * i) * 65 + c];
          hj[i] = Hs[(vj + 8 * i) * 65 + c];
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
    lds_sync();
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
  lds_sync();
}

// Columns of W (Algorithm 1): update vector in the compressed space, lift and
// clip on all rows, map back.  Each wavefront owns a contiguous quarter of
// the rows and walks it in chunks of 32 rows with no workgroup barrier.  A
// chunk of Q (32 l contiguous floats) arrives by coalesced 256-byte loads,
// one chunk ahead, and is laid out in the wavefront's own LDS tile at an odd
// pitch; lane i of half h then reads row i over the columns of half h, lifts
// it (the halves' partial dot products are exchanged by a lane swap), clips,
// stores W(row, j) and accumulates Q(row, c) w(row) for its columns in
// registers.  Per column the 32 rows of a half are summed by lane
// butterflies, then the four wavefronts in FP64 through LDS, in a fixed
// order.  Reads past the chunk return zero (buffer loads) or land in the
// tile's slack and are weighted by zero.  W is held by columns (Wc: k x m,
// columns ldw floats apart, a multiple of 32 from a 128-byte boundary) and the
// wavefronts' row ranges start on multiples of 32, so the 32 rows of a chunk
// store exactly one 128-byte line of column j.
template <int NL>  // coalesced loads per lane per chunk: NL >= ceil(32 l / 64)
__device__ __noinline__ void w_phase_t(const float* __restrict__ Q, float* __restrict__ Wc, int64_t m, int64_t ldw,
                                       int l, int k,
                                       float* Wts, const float* Ts, const float* Vs, float* vec, double* red,
                                       float* scr) {
  constexpr int CR = 32;             // rows per chunk
  constexpr int NH = BLM / 2;        // columns of a half, at most
  constexpr int WT = CR * (BLM + 1) + BLM;  // LDS floats per wavefront tile
  static_assert(4 * WT <= SCR_FLOATS, "four wavefront tiles fit the scratch");
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int h = lane >> 5, i = lane & 31;
  const int L2 = (l + 1) / 2;
  const int c0 = h ? L2 : 0, nh = h ? l - L2 : L2;
  const int P = l | 1;               // odd pitch: rows of a half on distinct banks
  float* Qw = scr + wave * WT;
  const int64_t rw0 = wave == 0 ? 0 : ((m * wave / 4) & ~(int64_t)(CR - 1));
  const int64_t rw1 = wave == 3 ? m : ((m * (wave + 1) / 4) & ~(int64_t)(CR - 1));
  const int nch = (int)((rw1 - rw0 + CR - 1) / CR);
  gf* Wg = GW(Wc);
  // Q through a buffer resource (m l floats): a position past the end reads 0.
  // (The arguments of a non-inlined function arrive in vector registers: the
  // base and size are made wavefront-uniform so the resource sits in scalars.)
  const uint64_t qa = (uint64_t)(uintptr_t)Q;
  const unsigned qlo = __builtin_amdgcn_readfirstlane((unsigned)qa);
  const unsigned qhi = __builtin_amdgcn_readfirstlane((unsigned)(qa >> 32));
  const int qbytes = __builtin_amdgcn_readfirstlane((int)(m * l * (int64_t)sizeof(float)));
  const __amdgpu_buffer_rsrc_t qrs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(uintptr_t)(((uint64_t)qhi << 32) | qlo), (short)0, qbytes, 0x00020000);
  // The lift reads every entry of a row's half up to NH columns, so entries
  // that no chunk writes (a row's padding, the slack) are multiplied by zero
  // weights: they must hold finite values, not what an earlier kernel left in
  // LDS.  The wavefront clears its own tile once (its LDS operations complete
  // in order, so no barrier is needed before the first chunk lands).
  for (int e = lane; e < WT; e += 64) Qw[e] = 0.f;
  // LDS position of this lane's element e = lane + 64 s of a chunk (row e / l,
  // column e % l), the same for every chunk; elements past the chunk go to
  // the tile's slack
  int pos[NL];
#pragma unroll
  for (int s2 = 0; s2 < NL; ++s2) {
    const int e = lane + 64 * s2;
    pos[s2] = e < CR * l ? (e / l) * P + (e - (e / l) * l) : CR * P + lane;
  }
  // rows past the wave's range: the chunk is read from the wave's own rows
  // only up to rw1 (the rest reads Q's next rows or zeros) and weighted 0
  auto fetch = [&](float (&v)[NL], int ch) __attribute__((always_inline)) {
    const int vo = (int)(((rw0 + (int64_t)ch * CR) * l + lane) * (int64_t)sizeof(float));
#pragma unroll
    for (int s2 = 0; s2 < NL; ++s2)
      v[s2] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(qrs, vo, 256 * s2, 0));
  };
  for (int j = 0; j < k; ++j) {
    const float d = Vs[j * BKM + j];
    if (!(d > 0.f)) continue;  // uniform: V is shared by the workgroup
    if (t < l) {
      float s0 = Ts[t * BKM + j], s1 = 0.f;
      int ii = 0;
      for (; ii + 2 <= k; ii += 2) {
        s0 = fmaf(-Wts[t * BKM + ii], Vs[ii * BKM + j], s0);
        s1 = fmaf(-Wts[t * BKM + ii + 1], Vs[(ii + 1) * BKM + j], s1);
      }
      for (; ii < k; ++ii) s0 = fmaf(-Wts[t * BKM + ii], Vs[ii * BKM + j], s0);
      vec[t] = Wts[t * BKM + j] + (s0 + s1) / d;
    }
    lds_sync();
    float vv[NH], acc[NH];
#pragma unroll
    for (int c = 0; c < NH; ++c) {
      vv[c] = c < nh ? vec[c0 + c] : 0.f;
      acc[c] = 0.f;
    }
    float qn[NL];
    if (nch > 0) fetch(qn, 0);
    for (int ch = 0; ch < nch; ++ch) {
      // lay the chunk out in the tile (the previous chunk's reads are done:
      // LDS operations of a wavefront complete in order)
#pragma unroll
      for (int s2 = 0; s2 < NL; ++s2) Qw[pos[s2]] = qn[s2];
      if (ch + 1 < nch) fetch(qn, ch + 1);
      float q[NH];
#pragma unroll
      for (int c = 0; c < NH; ++c) q[c] = Qw[i * P + c0 + c];
      float u0 = 0.f, u1 = 0.f;
#pragma unroll
      for (int c = 0; c < NH; c += 2) {
        u0 = fmaf(q[c], vv[c], u0);
        u1 = fmaf(q[c + 1], vv[c + 1], u1);
      }
      const float part = u0 + u1;
      const float other = __shfl_xor(part, 32);
      const int64_t r = rw0 + (int64_t)ch * CR + i;
      // the same sum on both halves: half 0's part first
      const float tot = h ? other + part : part + other;
      const float w = r < rw1 ? clipf(tot) : 0.f;
      if (h == 0 && r < rw1) Wg[(int64_t)j * ldw + r] = w;
#pragma unroll
      for (int c = 0; c < NH; ++c) acc[c] = fmaf(q[c], w, acc[c]);
    }
    // sums over the 32 rows of each half (every lane of the half gets them)
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
#pragma unroll
      for (int c = 0; c < NH; ++c) acc[c] += __shfl_xor(acc[c], o);
    }
    float mine = 0.f;
#pragma unroll
    for (int c = 0; c < NH; ++c) mine = (c == i) ? acc[c] : mine;
    if (i < nh) red[wave * BLM + c0 + i] = (double)mine;
    lds_sync();
    if (t < l) Wts[t * BKM + j] = (float)((red[t] + red[BLM + t]) + (red[2 * BLM + t] + red[3 * BLM + t]));
    lds_sync();
  }
  __syncthreads();  // W is read next by other threads of the workgroup
}
__device__ __forceinline__ void w_phase(const float* Q, float* Wc, int64_t m, int64_t ldw, int l, int k, float* Wts,
                                        const float* Ts, const float* Vs, float* vec, double* red, float* scr) {
  if (l <= 16) w_phase_t<8>(Q, Wc, m, ldw, l, k, Wts, Ts, Vs, vec, red, scr);
  else if (l <= 32) w_phase_t<16>(Q, Wc, m, ldw, l, k, Wts, Ts, Vs, vec, red, scr);
  else if (l <= 48) w_phase_t<24>(Q, Wc, m, ldw, l, k, Wts, Ts, Vs, vec, red, scr);
  else w_phase_t<32>(Q, Wc, m, ldw, l, k, Wts, Ts, Vs, vec, red, scr);
}

// The H rows and the T, V products in one call: the two phases are inlined
// here, so the registers they use are saved once per sweep, and their code
// is scheduled as one function (measured: 244.8 -> 238.9 ms per FP32 run of
// the 512-problem workload; merging the W phase and S = W^T W as well made it
// slower).
__device__ __noinline__ void h_tv(const float* Bt, float* H, int64_t n, int l, int k, const float* Wts,
                                  const float* Ss, double* rinv, float* scr, int nct, float* Ts, float* Vs) {
  h_phase(Bt, H, n, l, k, Wts, Ss, rinv, scr, nct);
  tv_phase(Bt, H, n, l, k, Ts, Vs, scr);
}

// ||X - W H||_F^2 and ||X||_F^2 (FP64 sums, fixed order) for thread 0.
__device__ __noinline__ void rel_err(const float* __restrict__ X, int64_t ldx, int64_t m, int64_t n, const float* __restrict__ W,
                        const float* __restrict__ H, int k, float* scr, double* red, double* out) {
  const int t = threadIdx.x;
  float* Xs = scr;                      // 64 x 65
  float* Wsh = scr + 64 * 65;           // 64 x (BKM + 1)
  float* Hs = Wsh + 64 * (BKM + 1);     // BKM x 65
  const int ti = t % 16, tj = t / 16;
  double e2 = 0.0, x2 = 0.0;
  for (int64_t r0 = 0; r0 < m; r0 += 64) {
    rows_load<8>(Wsh, BKM + 1, G(W), r0, m, 64, k);
    for (int64_t c0 = 0; c0 < n; c0 += 64) {
      {
        float xv[16], hv[8];
        pow2_fetch<16>(xv, G(X), ldx, r0, m, c0, n, 64, 6);
        pow2_fetch<8>(hv, G(H), n, 0, k, c0, n, k, 6);
        pow2_store<16>(xv, Xs, 65, 64, 6);
        pow2_store<8>(hv, Hs, 65, k, 6);
      }
      lds_sync();
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
      lds_sync();
    }
  }
  red[t] = e2;
  red[BT + t] = x2;
  lds_sync();
  for (int o = BT / 2; o > 0; o >>= 1) {
    if (t < o) {
      red[t] += red[t + o];
      red[BT + t] += red[BT + t + o];
    }
    lds_sync();
  }
  if (t == 0) {
    out[0] = red[0];
    out[1] = red[BT];
  }
  lds_sync();
}

__global__ __launch_bounds__(BT, 2) void batch_kernel(const BDesc* __restrict__ descs, int nprob, int q, int nsweeps,
                                                   unsigned* counter, double* err, unsigned* status) {
  extern __shared__ float lds[];
  __shared__ int cur, flag;
  const int t = threadIdx.x;
  float* Wts = lds + OFF_WT;
  float* Ts = lds + OFF_T;
  float* Vs = lds + OFF_V;
  float* Ss = lds + OFF_S;
  float* vec = lds + OFF_VEC;
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
    const bool bf = p.prec == RNMF_PREC_BF16;
    const int qe = q + (bf ? 1 : 0);  // the BF16 form adds one subspace iteration
    unsigned st = 0;
    // range finder (Algorithm 1, steps 3-8)
    if (bf) xa_pass_bf16(p.X, ldx, m, n, p.Omega, l, p.Q, scr);
    else xa_pass(p.X, ldx, m, n, p.Omega, l, p.Q, tc, scr);
    st |= cholqr2(p.Q, m, l, tc, scr, &flag);
    for (int it = 0; it < qe && !(st & ST_NOT_SPD); ++it) {
      if (bf) xtq_pass_bf16(p.X, ldx, m, n, p.Q, l, p.Z, nullptr, scr);
      else xtq_pass(p.X, ldx, m, n, p.Q, l, p.Z, nullptr, tc, scr);
      st |= cholqr2(p.Z, n, l, tc, scr, &flag);
      if (st & ST_NOT_SPD) break;
      if (bf) xa_pass_bf16(p.X, ldx, m, n, p.Z, l, p.Q, scr);
      else xa_pass(p.X, ldx, m, n, p.Z, l, p.Q, tc, scr);
      st |= cholqr2(p.Q, m, l, tc, scr, &flag);
    }
    if (!(st & ST_NOT_SPD)) {
      // compression (step 9): B^T into Z for the sweeps, B for the caller
      if (bf) xtq_pass_bf16(p.X, ldx, m, n, p.Q, l, p.Z, p.B, scr);
      else xtq_pass(p.X, ldx, m, n, p.Q, l, p.Z, p.B, tc, scr);
      // initialisation (step 10)
      // W is held by columns during the sweeps (Wc: k x m after B^T in Z, from
      // the next 128-byte boundary, columns ldw = m rounded up to 32 floats
      // apart), so the W phase stores each column as whole cache lines
      float* Wc = (float*)(((uintptr_t)(p.Z + n * (int64_t)l) + 127) & ~(uintptr_t)127);
      const int64_t ldw = (m + 31) & ~(int64_t)31;
      for (int e = t; e < OFF_VEC; e += BT) lds[e] = 0.f;  // W~, T, V, S zero beyond k
      w_to_columns(Wc, p.W0, m, ldw, k, scr);
      copy_f(p.H, p.H0, (int64_t)k * n);
      __syncthreads();
      init_wt(p.Q, p.W0, m, l, k, Wts, scr);
      // sweeps (steps 11-22): H rows, then W columns
      for (int s = 0; s < nsweeps; ++s) {
        gram_w(Wc, m, ldw, k, Ss, scr);
        h_tv(p.Z, p.H, n, l, k, Wts, Ss, red, scr, d.hct, Ts, Vs);
        w_phase(p.Q, Wc, m, ldw, l, k, Wts, Ts, Vs, vec, red, scr);
      }
      w_from_columns(p.W, Wc, m, ldw, k, scr);
      __syncthreads();
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
bool batch_hct_ok(int hct, int l) {
  return (hct == 64 || hct == 128 || hct == 256) && hct * (l + 1) <= SCR_FLOATS;
}

void batch_fill_desc(void* dst, const rnmf_problem& p, int idx, int tc, int hct) {
  BDesc d;
  d.p = p;
  d.idx = idx;
  d.tc = tc;
  d.hct = hct;
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

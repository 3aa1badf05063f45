// Passes over the data matrix X (m x n, row-major, leading dimension ldx):
//   NN:  Y = X A        (sketch X Omega and power half-step X Q; Sec. 2.3)
//   TN:  Z = X^T Q      (power half-step X^T Q and, transposed, B = Q^T X)
// The small operand (A or Q, at most 128 columns) is pre-packed transposed so
// that every MFMA operand fragment is a contiguous run along the reduction
// index.  Each workgroup streams a disjoint block of X exactly once; split
// reductions write partials that a second kernel adds in fixed order, so
// results are deterministic.
//
// Matrix-core forms (gfx950):
//   FP32: v_mfma_f32_16x16x4_f32, lane (i, g) = (lane % 16, lane / 16) holds
//         A[i][g] and B[g][i]; D[4g + e][i] in element e.
//   BF16: v_mfma_f32_16x16x32_bf16, lane (i, g) holds A[i][8g..8g+7] and
//         B[8g..8g+7][i]; same D layout.  X is bfloat16.  The packed small
//         operand has hi + lo bfloat16 planes: the compression B = Q^T X
//         uses both (two MFMAs per tile, so only X is rounded); the passes
//         inside the subspace iteration (Y = X Omega, Z = X^T Q, Y = X Z) use
//         the hi plane, the operand rounded to nearest even.  They only steer
//         the subspace, which the next orthonormalisation and the extra
//         iteration of the BF16 form absorb (final error unchanged to 2e-6
//         relative at 100,000 x 5,000, k = 50), with half the operand blocks
//         and products (NN 252 against 343 us, TN 232 against 247 us).
//   FP64: vector FMA, register-blocked through LDS.
#include "rnmf_common.h"

namespace rnmf {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushort4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma_bf(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ unsigned scan_f32(float v) {
  unsigned f = 0;
  if (!(v == v) || fabsf(v) == INFINITY) f |= ST_NONFINITE;
  else if (v < 0.0f) f |= ST_NEGATIVE;
  return f;
}

template <int VW> struct fvec;
template <> struct fvec<1> { typedef float t; };
template <> struct fvec<2> { typedef floatx2 t; };
template <> struct fvec<4> { typedef floatx4 t; };

template <int VW>
__device__ __forceinline__ typename fvec<VW>::t ldv(const float* p) {
  return *(const typename fvec<VW>::t*)p;
}
template <int VW>
__device__ __forceinline__ float el(const typename fvec<VW>::t& v, int s) {
  if constexpr (VW == 1) return v;
  else return v[s];
}
template <int VW>
__device__ __forceinline__ typename fvec<VW>::t ldv_guard(const float* p, int64_t idx, int64_t end) {
  typename fvec<VW>::t r;
  if constexpr (VW == 1) {
    r = idx < end ? p[0] : 0.0f;
  } else {
#pragma unroll
    for (int s = 0; s < VW; ++s) r[s] = (idx + s < end) ? p[s] : 0.0f;
  }
  return r;
}

// ---------------------------------------------------------------------------
// Packing of the small operand: dst[i][r] = src[r][i] (i < cols), 0 for
// cols <= i < lp or rows <= r < ldp.  For bf16 the hi plane is followed by the
// lo plane: hi = bf16(x), lo = bf16(x - hi).
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned short bf16_rne(float f) {
  unsigned b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (unsigned short)(b >> 16);
}

template <typename ST, typename DT>
__global__ __launch_bounds__(256) void pack_t_kernel(const ST* __restrict__ src, int64_t rows, int cols,
                                                     int lp, int64_t ldp, DT* __restrict__ dst) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  const int i0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    int64_t r = r0 + yy;
    int i = i0 + tx;
    tile[yy][tx] = (r < rows && i < cols) ? (double)src[r * cols + i] : 0.0;
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    int i = i0 + yy;
    int64_t r = r0 + tx;
    if (i < lp && r < ldp) dst[(int64_t)i * ldp + r] = (DT)tile[tx][yy];
  }
}

template <typename ST>
__global__ __launch_bounds__(256) void pack_t_bf16_kernel(const ST* __restrict__ src, int64_t rows, int cols,
                                                          int lp, int64_t ldp, unsigned short* __restrict__ dst,
                                                          int hi_only) {
  __shared__ float tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  const int i0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int yy = ty; yy < 32; yy += 8) {
    int64_t r = r0 + yy;
    int i = i0 + tx;
    tile[yy][tx] = (r < rows && i < cols) ? (float)src[r * cols + i] : 0.0f;
  }
  __syncthreads();
  unsigned short* lo = dst + (int64_t)lp * ldp;
  for (int yy = ty; yy < 32; yy += 8) {
    int i = i0 + yy;
    int64_t r = r0 + tx;
    if (i < lp && r < ldp) {
      float x = tile[tx][yy];
      unsigned short h = bf16_rne(x);
      float hf = __uint_as_float(((unsigned)h) << 16);
      dst[(int64_t)i * ldp + r] = h;
      lo[(int64_t)i * ldp + r] = hi_only ? (unsigned short)0 : bf16_rne(x - hf);
    }
  }
}

hipError_t launch_pack_t(const void* src, int dt, int64_t rows, int cols, int lp, int64_t ldp,
                         void* dst, int cdt, hipStream_t s, int hi_only) {
  dim3 grid((unsigned)ceil_div(ldp, 32), (unsigned)ceil_div(lp, 32));
  if (cdt == 2) {
    if (dt == 0)
      hipLaunchKernelGGL(pack_t_bf16_kernel<double>, grid, dim3(256), 0, s, (const double*)src, rows,
                         cols, lp, ldp, (unsigned short*)dst, hi_only);
    else
      hipLaunchKernelGGL(pack_t_bf16_kernel<float>, grid, dim3(256), 0, s, (const float*)src, rows,
                         cols, lp, ldp, (unsigned short*)dst, hi_only);
  } else if (cdt == 1) {
    if (dt == 0)
      hipLaunchKernelGGL((pack_t_kernel<double, float>), grid, dim3(256), 0, s, (const double*)src,
                         rows, cols, lp, ldp, (float*)dst);
    else
      hipLaunchKernelGGL((pack_t_kernel<float, float>), grid, dim3(256), 0, s, (const float*)src,
                         rows, cols, lp, ldp, (float*)dst);
  } else {
    if (dt == 0)
      hipLaunchKernelGGL((pack_t_kernel<double, double>), grid, dim3(256), 0, s, (const double*)src,
                         rows, cols, lp, ldp, (double*)dst);
    else
      hipLaunchKernelGGL((pack_t_kernel<float, double>), grid, dim3(256), 0, s, (const float*)src,
                         rows, cols, lp, ldp, (double*)dst);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// NN, FP32 matrix cores.  Workgroup: 4 waves x (16 * RW) rows, all lp = 16 NT
// columns; grid.y splits the reduction over n.
// ---------------------------------------------------------------------------
template <int NT, int VW, int RW>
__global__ __launch_bounds__(256) void nn_f32_kernel(const float* __restrict__ X, int64_t m, int64_t n,
                                                     int64_t ldx, const float* __restrict__ At, int64_t ldat,
                                                     int l, float* __restrict__ Y, float* __restrict__ part,
                                                     int64_t klen, unsigned* status, int check,
                                                     const unsigned* skip) {
  if (skip && *skip == 0u) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int64_t row_base = (int64_t)blockIdx.x * (64 * RW) + wave * (16 * RW);
  const int64_t kb = (int64_t)blockIdx.y * klen;
  const int64_t ke = (kb + klen < n) ? kb + klen : n;
  constexpr int KS = 4 * VW;
  floatx4 acc[RW][NT];
#pragma unroll
  for (int a = 0; a < RW; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  const float* xr[RW];
  bool rv[RW];
#pragma unroll
  for (int rt = 0; rt < RW; ++rt) {
    int64_t r = row_base + rt * 16 + i;
    rv[rt] = r < m;
    xr[rt] = X + (rv[rt] ? r : (m - 1)) * ldx + VW * g;
  }
  const float* ar[NT];
#pragma unroll
  for (int ct = 0; ct < NT; ++ct) ar[ct] = At + (int64_t)(ct * 16 + i) * ldat + VW * g;
  unsigned flag = 0;
  int64_t k0 = kb;
  for (; k0 + KS <= ke; k0 += KS) {
    typename fvec<VW>::t xa[RW], av[NT];
#pragma unroll
    for (int rt = 0; rt < RW; ++rt) xa[rt] = ldv<VW>(xr[rt] + k0);
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) av[ct] = ldv<VW>(ar[ct] + k0);
    if (check) {
#pragma unroll
      for (int rt = 0; rt < RW; ++rt)
        if (rv[rt])
#pragma unroll
          for (int s = 0; s < VW; ++s) flag |= scan_f32(el<VW>(xa[rt], s));
    }
#pragma unroll
    for (int s = 0; s < VW; ++s)
#pragma unroll
      for (int rt = 0; rt < RW; ++rt)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) acc[rt][ct] = mfma4(el<VW>(xa[rt], s), el<VW>(av[ct], s), acc[rt][ct]);
  }
  if (k0 < ke) {
    const int64_t kk = k0 + VW * g;
    typename fvec<VW>::t xa[RW], av[NT];
#pragma unroll
    for (int rt = 0; rt < RW; ++rt) xa[rt] = ldv_guard<VW>(xr[rt] + k0, kk, ke);
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) av[ct] = ldv_guard<VW>(ar[ct] + k0, kk, ke);
    if (check) {
#pragma unroll
      for (int rt = 0; rt < RW; ++rt)
        if (rv[rt])
#pragma unroll
          for (int s = 0; s < VW; ++s) flag |= scan_f32(el<VW>(xa[rt], s));
    }
#pragma unroll
    for (int s = 0; s < VW; ++s)
#pragma unroll
      for (int rt = 0; rt < RW; ++rt)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) acc[rt][ct] = mfma4(el<VW>(xa[rt], s), el<VW>(av[ct], s), acc[rt][ct]);
  }
  if (check && __ballot(flag != 0)) {
    for (int o = 32; o > 0; o >>= 1) flag |= __shfl_xor(flag, o);
    if (lane == 0 && flag) atomicOr(status, flag);
  }
  const int lp = NT * 16;
#pragma unroll
  for (int rt = 0; rt < RW; ++rt)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int64_t r = row_base + rt * 16 + 4 * g + e;
        int c = ct * 16 + i;
        if (r < m && c < l) {
          if (part) part[((int64_t)blockIdx.y * m + r) * lp + c] = acc[rt][ct][e];
          else Y[r * l + c] = acc[rt][ct][e];
        }
      }
}

// ---------------------------------------------------------------------------
// NN, BF16 matrix cores (X bfloat16 with ldx % 8 == 0; At hi and lo planes).
// ---------------------------------------------------------------------------
template <int NT, int RW>
__global__ __launch_bounds__(256) void nn_bf16_kernel(const bf16_t* __restrict__ X, int64_t m, int64_t n,
                                                      int64_t ldx, const bf16_t* __restrict__ At, int64_t ldat,
                                                      int lp_all, int l, float* __restrict__ Y,
                                                      float* __restrict__ part, int64_t klen) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int64_t row_base = (int64_t)blockIdx.x * (64 * RW) + wave * (16 * RW);
  const int64_t kb = (int64_t)blockIdx.y * klen;
  const int64_t ke = (kb + klen < n) ? kb + klen : n;
  floatx4 acc[RW][NT];
#pragma unroll
  for (int a = 0; a < RW; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  const bf16_t* xr[RW];
#pragma unroll
  for (int rt = 0; rt < RW; ++rt) {
    int64_t r = row_base + rt * 16 + i;
    xr[rt] = X + (r < m ? r : (m - 1)) * ldx + 8 * g;
  }
  // the operand's hi plane (the operand rounded to bfloat16), as in nn2_kernel
  (void)lp_all;
  const bf16_t* ah[NT];
#pragma unroll
  for (int ct = 0; ct < NT; ++ct) ah[ct] = At + (int64_t)(ct * 16 + i) * ldat + 8 * g;
  int64_t k0 = kb;
  for (; k0 + 32 <= ke; k0 += 32) {
    bf16x8 xa[RW], hv[NT];
#pragma unroll
    for (int rt = 0; rt < RW; ++rt) xa[rt] = *(const bf16x8*)(xr[rt] + k0);
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) hv[ct] = *(const bf16x8*)(ah[ct] + k0);
#pragma unroll
    for (int rt = 0; rt < RW; ++rt)
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[rt][ct] = mfma_bf(xa[rt], hv[ct], acc[rt][ct]);
  }
  if (k0 < ke) {
    const int64_t kk = k0 + 8 * g;
    bf16x8 xa[RW], hv[NT];
#pragma unroll
    for (int rt = 0; rt < RW; ++rt)
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        unsigned short v = (kk + s < ke) ? xr[rt][k0 + s] : (unsigned short)0;
        xa[rt][s] = __builtin_bit_cast(__bf16, v);
      }
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        unsigned short h = (kk + s < ke) ? ah[ct][k0 + s] : (unsigned short)0;
        hv[ct][s] = __builtin_bit_cast(__bf16, h);
      }
#pragma unroll
    for (int rt = 0; rt < RW; ++rt)
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[rt][ct] = mfma_bf(xa[rt], hv[ct], acc[rt][ct]);
  }
  const int lp = NT * 16;
#pragma unroll
  for (int rt = 0; rt < RW; ++rt)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int64_t r = row_base + rt * 16 + 4 * g + e;
        int c = ct * 16 + i;
        if (r < m && c < l) {
          if (part) part[((int64_t)blockIdx.y * m + r) * lp + c] = acc[rt][ct][e];
          else Y[r * l + c] = acc[rt][ct][e];
        }
      }
}

// ---------------------------------------------------------------------------
// NN, streamed form (FP32 or BF16 X, 16-byte aligned rows).  Total bytes that
// enter the CUs (X from HBM plus the small operand from L2) bound these
// passes, so a workgroup of 8 waves owns a contiguous range of 16-row tiles
// (about m / #CUs rows) and reads the small operand once per pass.  X and
// operand rows travel by direct global->LDS loads, double-buffered by stage.
// A stage covers one 128-byte line of every row (64 k in BF16, 32 in FP32):
// a 16-row block arrives as two 1 KB loads of 8 whole lines each (a load of
// 16 half lines streams markedly slower).  Lane L of such a load takes row
// L / 8 and 16-byte chunk (L % 8) ^ (L / 8); the second half of a block sits
// 16 bytes past a 1 KB boundary.  The MFMA fragment of lane (i, g) at k-step
// u (chunk 4u + g of row i) is then read back from a bank-conflict-free
// position.
//   BF16: fragment = 16 rows x 32 k (8 per lane); one operand plane (hi).
//   FP32: fragment = 16 rows x 16 k (4 per lane: MFMA s uses k = 4g + s).
// Wave w owns tiles w, w + 8, ... of the range.
// ---------------------------------------------------------------------------
constexpr int NN2_HALF = 1024 + 16;          // second half of a block
constexpr int NN2_BLOCK = NN2_HALF + 1024;   // bytes of one 16-row block
#define RNMF_GPTR(p) ((const __attribute__((address_space(1))) void*)(p))
#define RNMF_LPTR(p) ((__attribute__((address_space(3))) void*)(p))

__device__ __forceinline__ void lds_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0) only: outstanding global loads stay in flight
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <typename E, int NT, int KU, int RWMAX>
__global__ __launch_bounds__(512) void nn2_kernel(const E* __restrict__ X, int64_t m, int64_t n, int64_t ldx,
                                                  const E* __restrict__ At, int64_t ldat, int lp_all, int l,
                                                  float* __restrict__ Y, float* __restrict__ part, int64_t klen,
                                                  int tiles, int G, unsigned* status, int check,
                                                  const unsigned* skip) {
  extern __shared__ __attribute__((aligned(16))) unsigned char nn2_lds[];
  if (skip && *skip == 0u) return;
  constexpr bool BF = sizeof(E) == 2;
  constexpr int KS = BF ? 32 : 16;       // k per fragment
  constexpr int EPC = BF ? 8 : 4;        // elements per lane chunk (16 bytes)
  constexpr int NPL = 1;                 // operand planes read (BF16: the hi plane only)
  static_assert(KU * KS * (int)sizeof(E) == 128, "a stage covers one 128-byte line of every row");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, gq = lane >> 4;
  const int gidx = blockIdx.x;
  const int t0 = (int)((int64_t)tiles * gidx / G), t1 = (int)((int64_t)tiles * (gidx + 1) / G);
  const int nt = t1 - t0;               // tiles of this workgroup, <= 8 * RWMAX
  const int NB = nt + NPL * NT;         // 16-row blocks per stage (X tiles, then operand planes)
  const int64_t kb = (int64_t)blockIdx.y * klen;
  const int64_t ke = (kb + klen < n) ? kb + klen : n;
  const int nst = (int)((ke - kb + KS * KU - 1) / (KS * KU));
  const int64_t plane = (int64_t)lp_all * ldat;
  // swizzled placement: lane L of a half-block load takes row L / 8 and the
  // 16-byte chunk (L % 8) ^ (L / 8) of that row's 128 bytes
  const int srow = lane >> 3, schunk = (lane & 7) ^ srow;
  // the lane's MFMA fragment of k-step u inside a block (see the header)
  auto frag_ofs = [&](int u) -> int {
    return (i >> 3) * NN2_HALF + (8 * (i & 7) + ((4 * u + gq) ^ (i & 7))) * 16;
  };
  floatx4 acc[RWMAX][NT];
#pragma unroll
  for (int a = 0; a < RWMAX; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

  auto issue = [&](int st) {
    const int64_t k = kb + (int64_t)st * KS * KU;
    unsigned char* base = nn2_lds + (size_t)(st & 1) * NB * NN2_BLOCK;
    for (int f = wave; f < 2 * NB; f += 8) {
      const int b = f >> 1, j = f & 1;
      const E* src;
      if (b < nt) {
        int64_t r = (int64_t)(t0 + b) * 16 + 8 * j + srow;
        if (r >= m) r = m - 1;
        int64_t c = k + schunk * EPC;
        if (c >= ke || c + EPC > n) c = 0;  // in-bounds address; fixed up after arrival
        src = X + r * ldx + c;
      } else {
        const int a = b - nt;
        const int pl = a / NT, ct = a - (a / NT) * NT;
        src = At + pl * plane + (int64_t)(ct * 16 + 8 * j + srow) * ldat + k + schunk * EPC;
      }
      __builtin_amdgcn_global_load_lds(RNMF_GPTR(src), RNMF_LPTR(base + (size_t)b * NN2_BLOCK + j * NN2_HALF), 16,
                                       0, 0);
    }
  };
  // tail stage: in this lane's own chunks, zero the elements at or beyond ke
  // and load element by element a chunk that runs past the end of the row
  auto patch = [&](int st) {
    const int64_t k = kb + (int64_t)st * KS * KU;
    unsigned char* base = nn2_lds + (size_t)(st & 1) * NB * NN2_BLOCK;
    for (int f = wave; f < 2 * nt; f += 8) {
      const int b = f >> 1, j = f & 1;
      const int64_t c = k + schunk * EPC;
      if (c + EPC > ke) {
        int64_t r = (int64_t)(t0 + b) * 16 + 8 * j + srow;
        if (r >= m) r = m - 1;
        const bool reload = c < ke && c + EPC > n;
        E* dst = (E*)(base + (size_t)b * NN2_BLOCK + j * NN2_HALF + lane * 16);
#pragma unroll
        for (int e = 0; e < EPC; ++e)
          if (c + e >= ke) dst[e] = (E)0;
          else if (reload) dst[e] = X[r * ldx + c + e];
      }
    }
  };

  unsigned flag = 0;
  if (nst > 0) issue(0);
  for (int st = 0; st < nst; ++st) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this stage has landed (only it is in flight)
    const int64_t k = kb + (int64_t)st * KS * KU;
    if (k + KS * KU > ke) patch(st);
    lds_barrier();
    if (st + 1 < nst) issue(st + 1);
    const unsigned char* base = nn2_lds + (size_t)(st & 1) * NB * NN2_BLOCK;
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      if (k + u * KS >= ke) break;
      const int fo = frag_ofs(u);
      if constexpr (BF) {
        bf16x8 xa[RWMAX];
#pragma unroll
        for (int rt = 0; rt < RWMAX; ++rt) {
          const int tau = wave + 8 * rt;
          if (tau < nt) xa[rt] = *(const bf16x8*)(base + (size_t)tau * NN2_BLOCK + fo);
        }
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          const bf16x8 h = *(const bf16x8*)(base + (size_t)(nt + ct) * NN2_BLOCK + fo);
#pragma unroll
          for (int rt = 0; rt < RWMAX; ++rt)
            if (wave + 8 * rt < nt) acc[rt][ct] = mfma_bf(xa[rt], h, acc[rt][ct]);
        }
      } else {
        floatx4 xa[RWMAX];
#pragma unroll
        for (int rt = 0; rt < RWMAX; ++rt) {
          const int tau = wave + 8 * rt;
          if (tau < nt) {
            xa[rt] = *(const floatx4*)(base + (size_t)tau * NN2_BLOCK + fo);
            if (check)
#pragma unroll
              for (int e = 0; e < 4; ++e) flag |= scan_f32(xa[rt][e]);
          }
        }
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          const floatx4 av = *(const floatx4*)(base + (size_t)(nt + ct) * NN2_BLOCK + fo);
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int rt = 0; rt < RWMAX; ++rt)
              if (wave + 8 * rt < nt) acc[rt][ct] = mfma4(xa[rt][e], av[e], acc[rt][ct]);
        }
      }
    }
  }
  if (check && __ballot(flag != 0)) {
    for (int o = 32; o > 0; o >>= 1) flag |= __shfl_xor(flag, o);
    if (lane == 0 && flag) atomicOr(status, flag);
  }
  const int lp = NT * 16;
#pragma unroll
  for (int rt = 0; rt < RWMAX; ++rt) {
    const int tau = wave + 8 * rt;
    if (tau >= nt) continue;
#pragma unroll
    for (int ct = 0; ct < NT; ++ct)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t r = (int64_t)(t0 + tau) * 16 + 4 * gq + e;
        const int c = ct * 16 + i;
        if (r < m && c < l) {
          if (part) part[((int64_t)blockIdx.y * m + r) * lp + c] = acc[rt][ct][e];
          else Y[r * l + c] = acc[rt][ct][e];
        }
      }
  }
}

// ---------------------------------------------------------------------------
// TN, streamed form: Z = X^T Q over a row split, for a block of 512 columns
// (8 waves x 64).  Each stage is 32 rows: X arrives row-major in LDS by
// direct loads of whole 1 KB row segments, Q^T fragments (packed transposed,
// zero beyond m) arrive in fragment layout.  Lane (i, g) of a wave owns
// columns c + 4i + j (j < 4).
//   BF16: MFMA depth 32 rows; the lane reads rows 8g + e (e < 8) x 4 columns
//         with 8-byte LDS reads and regroups them into four B fragments.
//   FP32: two MFMA groups of 16 rows; the lane reads rows 4g + s (s < 4) x 4
//         columns with 16-byte LDS reads; each value is one MFMA operand.
// ---------------------------------------------------------------------------
template <typename E, int NT, int NPL>  // NPL: operand planes read (BF16: 2 = hi + lo, 1 = hi)
__global__ __launch_bounds__(512) void tn2_kernel(const E* __restrict__ X, int64_t m, int64_t n, int64_t ldx,
                                                  const E* __restrict__ Qt, int64_t ldqt, int lp_all,
                                                  float* __restrict__ part, int64_t mlen) {
  extern __shared__ __attribute__((aligned(16))) unsigned char tn2_lds[];
  constexpr bool BF = sizeof(E) == 2;
  constexpr int SR = 32;                       // rows per stage
  constexpr int EPC = BF ? 8 : 4;              // elements per 16-byte chunk
  constexpr int RB = 512 * (int)sizeof(E);     // bytes of one row of the block
  constexpr int PITCH = RB + 16;               // LDS row pitch
  constexpr int XI = SR * (RB / 1024);         // X load instructions per stage
  constexpr int QF = (BF ? NPL : 1) * NT * (BF ? 1 : 2);  // Q fragments per stage (1 KB each)
  constexpr int FI = XI + QF;
  constexpr int SLOT = SR * PITCH + QF * 1024;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, gq = lane >> 4;
  const int64_t cb = (int64_t)blockIdx.x * 512;
  const int64_t mb = (int64_t)blockIdx.y * mlen;
  const int64_t me = (mb + mlen < m) ? mb + mlen : m;
  const int nst = (int)((me - mb + SR - 1) / SR);
  const int64_t plane = (int64_t)lp_all * ldqt;
  floatx4 acc[NT][4];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};

  auto issue = [&](int st) {
    const int64_t r0 = mb + (int64_t)st * SR;
    unsigned char* base = tn2_lds + (size_t)(st & 1) * SLOT;
    for (int f = wave; f < FI; f += 8) {
      if (f < XI) {
        const int rr = f / (RB / 1024), pp = f - (f / (RB / 1024)) * (RB / 1024);
        int64_t r = r0 + rr;
        if (r >= m) r = m - 1;
        int64_t c = cb + (int64_t)pp * (1024 / (int)sizeof(E)) + lane * EPC;
        if (c + EPC > n) c = 0;  // in-bounds address; a straddling chunk is reloaded
        __builtin_amdgcn_global_load_lds(RNMF_GPTR(X + r * ldx + c),
                                         RNMF_LPTR(base + (size_t)rr * PITCH + (size_t)pp * 1024), 16, 0, 0);
      } else {
        const int a = f - XI;
        const E* src;
        if constexpr (BF) {
          const int pl = a / NT, t = a - (a / NT) * NT;   // fragment: 16 l x 32 rows
          src = Qt + pl * plane + (int64_t)(t * 16 + i) * ldqt + r0 + 8 * gq;
        } else {
          const int h = a / NT, t = a - (a / NT) * NT;    // fragment: 16 l x 16 rows
          src = Qt + (int64_t)(t * 16 + i) * ldqt + r0 + 16 * h + 4 * gq;
        }
        __builtin_amdgcn_global_load_lds(RNMF_GPTR(src), RNMF_LPTR(base + (size_t)SR * PITCH + (size_t)a * 1024),
                                         16, 0, 0);
      }
    }
  };
  // a chunk that runs past the end of the row: load its valid elements one by one
  auto patch = [&](int st) {
    const int64_t r0 = mb + (int64_t)st * SR;
    unsigned char* base = tn2_lds + (size_t)(st & 1) * SLOT;
    for (int f = wave; f < XI; f += 8) {
      const int rr = f / (RB / 1024), pp = f - (f / (RB / 1024)) * (RB / 1024);
      const int64_t c = cb + (int64_t)pp * (1024 / (int)sizeof(E)) + lane * EPC;
      if (c < n && c + EPC > n) {
        int64_t r = r0 + rr;
        if (r >= m) r = m - 1;
        E* dst = (E*)(base + (size_t)rr * PITCH + (size_t)pp * 1024 + lane * 16);
#pragma unroll
        for (int e = 0; e < EPC; ++e) dst[e] = (c + e < n) ? X[r * ldx + c + e] : (E)0;
      }
    }
  };

  const bool edge = cb + 512 > n && (n % EPC) != 0;
  if (nst > 0) issue(0);
  for (int st = 0; st < nst; ++st) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this stage has landed (only it is in flight)
    if (edge) patch(st);
    lds_barrier();
    if (st + 1 < nst) issue(st + 1);
    const unsigned char* base = tn2_lds + (size_t)(st & 1) * SLOT;
    const unsigned char* qb = base + (size_t)SR * PITCH;
    const int cofs = (wave * 64 + 4 * i) * (int)sizeof(E);
    if constexpr (BF) {
      typedef unsigned uint2v __attribute__((ext_vector_type(2)));
      uint2v xv[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) xv[e] = *(const uint2v*)(base + (size_t)(8 * gq + e) * PITCH + cofs);
      bf16x8 b[4];
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const unsigned a0 = xv[2 * d].x, a1 = xv[2 * d + 1].x, b0 = xv[2 * d].y, b1 = xv[2 * d + 1].y;
        typedef unsigned uint4v __attribute__((ext_vector_type(4)));
        // column j of rows 2d, 2d + 1 packed into one dword of fragment j
        const unsigned w0 = (a0 & 0xFFFFu) | (a1 << 16), w1 = (a0 >> 16) | (a1 & 0xFFFF0000u);
        const unsigned w2 = (b0 & 0xFFFFu) | (b1 << 16), w3 = (b0 >> 16) | (b1 & 0xFFFF0000u);
        uint4v t0 = __builtin_bit_cast(uint4v, b[0]), t1 = __builtin_bit_cast(uint4v, b[1]);
        uint4v t2 = __builtin_bit_cast(uint4v, b[2]), t3 = __builtin_bit_cast(uint4v, b[3]);
        t0[d] = w0; t1[d] = w1; t2[d] = w2; t3[d] = w3;
        b[0] = __builtin_bit_cast(bf16x8, t0); b[1] = __builtin_bit_cast(bf16x8, t1);
        b[2] = __builtin_bit_cast(bf16x8, t2); b[3] = __builtin_bit_cast(bf16x8, t3);
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const bf16x8 h = *(const bf16x8*)(qb + (size_t)t * 1024 + lane * 16);
        if constexpr (NPL == 2) {
          const bf16x8 lo = *(const bf16x8*)(qb + (size_t)(NT + t) * 1024 + lane * 16);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            acc[t][j] = mfma_bf(h, b[j], acc[t][j]);
            acc[t][j] = mfma_bf(lo, b[j], acc[t][j]);
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[t][j] = mfma_bf(h, b[j], acc[t][j]);
        }
      }
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        floatx4 xv[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) xv[s4] = *(const floatx4*)(base + (size_t)(16 * h + 4 * gq + s4) * PITCH + cofs);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const floatx4 qa = *(const floatx4*)(qb + (size_t)(h * NT + t) * 1024 + lane * 16);
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[t][j] = mfma4(qa[s4], xv[s4][j], acc[t][j]);
        }
      }
    }
  }
  const int lp = NT * 16;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = cb + wave * 64 + 4 * i + j;
      if (col < n) *(floatx4*)(part + ((int64_t)blockIdx.y * n + col) * lp + t * 16 + 4 * gq) = acc[t][j];
    }
}

// ---------------------------------------------------------------------------
// TN, FP32 matrix cores.  Each wave owns 16 * VW columns of X; lane (i, g)
// loads rows m0 + 4g + s (s < 4) x VW columns; MFMA (s, c) uses row 4g + s
// and column VW * i + c, paired with Qt rows t * 16 + i at m0 + 4g + s.
// ---------------------------------------------------------------------------
template <int NT, int VW>
__global__ __launch_bounds__(256) void tn_f32_kernel(const float* __restrict__ X, int64_t m, int64_t n,
                                                     int64_t ldx, const float* __restrict__ Qt, int64_t ldqt,
                                                     float* __restrict__ part, int64_t mlen) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int64_t col0 = (int64_t)blockIdx.x * (64 * VW) + wave * (16 * VW) + VW * i;
  const int64_t mb = (int64_t)blockIdx.y * mlen;
  const int64_t me = (mb + mlen < m) ? mb + mlen : m;
  floatx4 acc[NT][VW];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < VW; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  const bool cfull = col0 + VW <= n;
  const bool cany = col0 < n;
  const float* xc = X + (cany ? col0 : 0);
  const float* qr[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) qr[t] = Qt + (int64_t)(t * 16 + i) * ldqt + 4 * g;
  int64_t m0 = mb;
  for (; m0 + 16 <= me; m0 += 16) {
    typename fvec<VW>::t xv[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const float* p = xc + (m0 + 4 * g + s) * ldx;
      xv[s] = cfull ? ldv<VW>(p) : ldv_guard<VW>(p, col0, cany ? n : col0);
    }
    floatx4 qa[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) qa[t] = *(const floatx4*)(qr[t] + m0);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int c = 0; c < VW; ++c) acc[t][c] = mfma4(qa[t][s], el<VW>(xv[s], c), acc[t][c]);
  }
  if (m0 < me) {
    typename fvec<VW>::t xv[4];
    floatx4 qa[NT];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      int64_t r = m0 + 4 * g + s;
      if (r < me) {
        const float* p = xc + r * ldx;
        xv[s] = cfull ? ldv<VW>(p) : ldv_guard<VW>(p, col0, cany ? n : col0);
      } else {
        xv[s] = ldv_guard<VW>(xc, 0, 0);
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) qa[t][s] = (r < me) ? qr[t][m0 + s] : 0.0f;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int c = 0; c < VW; ++c) acc[t][c] = mfma4(qa[t][s], el<VW>(xv[s], c), acc[t][c]);
  }
  const int lp = NT * 16;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int c = 0; c < VW; ++c) {
      int64_t col = col0 + c;
      if (col < n) {
        float* dst = part + ((int64_t)blockIdx.y * n + col) * lp + t * 16 + 4 * g;
        *(floatx4*)dst = acc[t][c];
      }
    }
}

// ---------------------------------------------------------------------------
// TN, BF16 matrix cores (X bfloat16 with ldx % 4 == 0).  Lane (i, g) loads
// rows m0 + 8g + s (s < 8) x 4 columns (8 bytes each) and regroups them in
// registers into four B fragments (8 consecutive rows of one column each).
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(256) void tn_bf16_kernel(const bf16_t* __restrict__ X, int64_t m, int64_t n,
                                                      int64_t ldx, const bf16_t* __restrict__ Qt, int64_t ldqt,
                                                      int lp_all, float* __restrict__ part, int64_t mlen) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int64_t col0 = (int64_t)blockIdx.x * 256 + wave * 64 + 4 * i;
  const int64_t mb = (int64_t)blockIdx.y * mlen;
  const int64_t me = (mb + mlen < m) ? mb + mlen : m;
  floatx4 acc[NT][4];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  const bool cfull = col0 + 4 <= n;
  const bf16_t* xc = X + (col0 < n ? col0 : 0);
  const int64_t plane = (int64_t)lp_all * ldqt;
  const bf16_t* qr[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) qr[t] = Qt + (int64_t)(t * 16 + i) * ldqt + 8 * g;
  for (int64_t m0 = mb; m0 < me; m0 += 32) {
    const bool full = (m0 + 32 <= me) && cfull;
    ushort4_t xv[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      int64_t r = m0 + 8 * g + s;
      if (full) {
        xv[s] = *(const ushort4_t*)(xc + r * ldx);
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c)
          xv[s][c] = (r < me && col0 + c < n) ? xc[r * ldx + c] : (unsigned short)0;
      }
    }
    bf16x8 b[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int s = 0; s < 8; ++s) b[c][s] = __builtin_bit_cast(__bf16, (unsigned short)xv[s][c]);
    bf16x8 hv[NT], lv[NT];
    if (m0 + 32 <= me) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        hv[t] = *(const bf16x8*)(qr[t] + m0);
        lv[t] = *(const bf16x8*)(qr[t] + plane + m0);
      }
    } else {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          bool ok = m0 + 8 * g + s < me;
          hv[t][s] = __builtin_bit_cast(__bf16, ok ? qr[t][m0 + s] : (unsigned short)0);
          lv[t][s] = __builtin_bit_cast(__bf16, ok ? qr[t][plane + m0 + s] : (unsigned short)0);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        acc[t][c] = mfma_bf(hv[t], b[c], acc[t][c]);
        acc[t][c] = mfma_bf(lv[t], b[c], acc[t][c]);
      }
  }
  const int lp = NT * 16;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int64_t col = col0 + c;
      if (col < n) {
        float* dst = part + ((int64_t)blockIdx.y * n + col) * lp + t * 16 + 4 * g;
        *(floatx4*)dst = acc[t][c];
      }
    }
}

// ---------------------------------------------------------------------------
// Vector-FMA forms (FP64, and bfloat16 X without 16-byte row alignment).
// NN: workgroup = 64 rows x lp columns, 16-wide reduction chunks in LDS.
// ---------------------------------------------------------------------------
template <typename XT> __device__ __forceinline__ float to_f(XT v) { return (float)v; }
template <> __device__ __forceinline__ float to_f<bf16_t>(bf16_t v) { return __uint_as_float(((unsigned)v) << 16); }

template <typename XT, typename CT, typename AT, int NT>
__global__ __launch_bounds__(256) void nn_valu_kernel(const XT* __restrict__ X, int64_t m, int64_t n, int64_t ldx,
                                                      const AT* __restrict__ At, int64_t ldat, int lp_all, int l,
                                                      CT* __restrict__ Y, CT* __restrict__ part, int64_t klen,
                                                      unsigned* status, int check, const unsigned* skip) {
  if (skip && *skip == 0u) return;
  constexpr int KC = 16;
  __shared__ CT Xs[64][KC + 1];
  __shared__ CT As[KC][NT * 16 + 1];
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int64_t kb = (int64_t)blockIdx.y * klen;
  const int64_t ke = (kb + klen < n) ? kb + klen : n;
  CT acc[4][NT];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = (CT)0;
  unsigned flag = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += KC) {
    for (int e = threadIdx.x; e < 64 * KC; e += 256) {
      int rr = e / KC, kk = e % KC;
      int64_t r = r0 + rr, k = k0 + kk;
      CT v = (CT)0;
      if (r < m && k < ke) {
        if constexpr (sizeof(XT) == 2) v = (CT)to_f<XT>(X[r * ldx + k]);
        else v = (CT)X[r * ldx + k];
        if (check) {
          double d = (double)v;
          if (!(d == d) || fabs(d) == INFINITY) flag |= ST_NONFINITE;
          else if (d < 0.0) flag |= ST_NEGATIVE;
        }
      }
      Xs[rr][kk] = v;
    }
    for (int e = threadIdx.x; e < KC * NT * 16; e += 256) {
      int kk = e / (NT * 16), c = e % (NT * 16);
      int64_t k = k0 + kk;
      CT v = (CT)0;
      if (k < ke) {
        if constexpr (sizeof(AT) == 2) {
          // BF16 sketch pass: the operand's hi plane (rounded to bfloat16),
          // as in the matrix-core kernels
          const bf16_t* ah = (const bf16_t*)At;
          v = (CT)to_f<bf16_t>(ah[(int64_t)c * ldat + k]);
        } else {
          v = (CT)At[(int64_t)c * ldat + k];
        }
      }
      As[kk][c] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KC; ++kk) {
      CT xa[4], av[NT];
#pragma unroll
      for (int a = 0; a < 4; ++a) xa[a] = Xs[tr * 4 + a][kk];
#pragma unroll
      for (int b = 0; b < NT; ++b) av[b] = As[kk][tc + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = fma(xa[a], av[b], acc[a][b]);
    }
    __syncthreads();
  }
  if (check && flag) atomicOr(status, flag);
  const int lp = NT * 16;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int64_t r = r0 + tr * 4 + a;
    if (r >= m) continue;
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      int c = tc + 16 * b;
      if (c >= l) continue;
      if (part) part[((int64_t)blockIdx.y * m + r) * lp + c] = acc[a][b];
      else Y[r * l + c] = acc[a][b];
    }
  }
}

// TN: workgroup = 64 columns of X x lp, over a split of the rows.
template <typename XT, typename CT, typename AT, int NT>
__global__ __launch_bounds__(256) void tn_valu_kernel(const XT* __restrict__ X, int64_t m, int64_t n, int64_t ldx,
                                                      const AT* __restrict__ Qt, int64_t ldqt, int lp_all,
                                                      CT* __restrict__ part, int64_t mlen) {
  constexpr int KC = 16;
  __shared__ CT Xs[KC][64 + 1];
  __shared__ CT Qs[KC][NT * 16 + 1];
  const int tcol = threadIdx.x >> 4, ta = threadIdx.x & 15;
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  const int64_t mb = (int64_t)blockIdx.y * mlen;
  const int64_t me = (mb + mlen < m) ? mb + mlen : m;
  CT acc[4][NT];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = (CT)0;
  for (int64_t m0 = mb; m0 < me; m0 += KC) {
    for (int e = threadIdx.x; e < KC * 64; e += 256) {
      int rr = e / 64, cc = e % 64;
      int64_t r = m0 + rr, c = c0 + cc;
      CT v = (CT)0;
      if (r < me && c < n) {
        if constexpr (sizeof(XT) == 2) v = (CT)to_f<XT>(X[r * ldx + c]);
        else v = (CT)X[r * ldx + c];
      }
      Xs[rr][cc] = v;
    }
    for (int e = threadIdx.x; e < KC * NT * 16; e += 256) {
      int rr = e / (NT * 16), a = e % (NT * 16);
      int64_t r = m0 + rr;
      CT v = (CT)0;
      if (r < me) {
        if constexpr (sizeof(AT) == 2) {
          const bf16_t* qh = (const bf16_t*)Qt;
          v = (CT)to_f<bf16_t>(qh[(int64_t)a * ldqt + r]) +
              (CT)to_f<bf16_t>(qh[(int64_t)lp_all * ldqt + (int64_t)a * ldqt + r]);
        } else {
          v = (CT)Qt[(int64_t)a * ldqt + r];
        }
      }
      Qs[rr][a] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < KC; ++rr) {
      CT xa[4], qv[NT];
#pragma unroll
      for (int a = 0; a < 4; ++a) xa[a] = Xs[rr][tcol * 4 + a];
#pragma unroll
      for (int b = 0; b < NT; ++b) qv[b] = Qs[rr][ta + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = fma(xa[a], qv[b], acc[a][b]);
    }
    __syncthreads();
  }
  const int lp = NT * 16;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int64_t c = c0 + tcol * 4 + a;
    if (c >= n) continue;
#pragma unroll
    for (int b = 0; b < NT; ++b) part[((int64_t)blockIdx.y * n + c) * lp + ta + 16 * b] = acc[a][b];
  }
}

// Fixed-order sum of split partials: out = sum_s part[s] (rows x l), written
// row-major (rows x l) or transposed (l x rows).
template <typename CT, typename OT>
__global__ __launch_bounds__(256) void reduce_parts_kernel(const CT* __restrict__ part, int splits, int64_t rows,
                                                           int l, int lp, OT* __restrict__ out, int transposed) {
  const int64_t total = rows * l;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t r, c;
    if (transposed) { c = e / rows; r = e - c * rows; }   // coalesced stores along rows
    else { r = e / l; c = e - r * l; }
    CT s = (CT)0;
    for (int p = 0; p < splits; ++p) s += part[((int64_t)p * rows + r) * lp + c];
    if (transposed) out[c * rows + r] = (OT)s;
    else out[r * l + c] = (OT)s;
  }
}

// FP32 partials: a block sums a 16-row tile of every split with 16-byte reads
// along the row (the same split order as above), then writes the tile through
// LDS, so that the transposed output is stored along its rows too.
__global__ __launch_bounds__(256) void reduce_tile_kernel(const float* __restrict__ part, int splits, int64_t rows,
                                                          int l, int lp, float* __restrict__ out, int transposed) {
  constexpr int RT = 16;
  __shared__ float tile[RT][LMAX + 1];
  const int64_t r0 = (int64_t)blockIdx.x * RT;
  const int nq = lp / 4;
  for (int q = threadIdx.x; q < RT * nq; q += 256) {
    const int rr = q / nq, cq = q - (q / nq) * nq;
    const int64_t r = r0 + rr;
    floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
    if (r < rows) {
      const float* src = part + r * lp + 4 * cq;
#pragma unroll 8
      for (int p = 0; p < splits; ++p) acc += *(const floatx4*)(src + (int64_t)p * rows * lp);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) tile[rr][4 * cq + e] = acc[e];
  }
  __syncthreads();
  if (transposed) {
    for (int e = threadIdx.x; e < l * RT; e += 256) {
      const int c = e / RT, rr = e - (e / RT) * RT;
      const int64_t r = r0 + rr;
      if (r < rows) out[(int64_t)c * rows + r] = tile[rr][c];
    }
  } else {
    for (int e = threadIdx.x; e < RT * l; e += 256) {
      const int rr = e / l, c = e - (e / l) * l;
      const int64_t r = r0 + rr;
      if (r < rows) out[r * l + c] = tile[rr][c];
    }
  }
}

template <typename CT, typename OT>
static hipError_t launch_reduce(const CT* part, int splits, int64_t rows, int l, int lp, OT* out, int tr,
                                hipStream_t s) {
  int64_t total = rows * l;
  if (total == 0) return hipSuccess;
  if constexpr (sizeof(CT) == 4 && sizeof(OT) == 4) {
    if (lp % 4 == 0 && lp <= LMAX && ((uintptr_t)part % 16) == 0) {
      hipLaunchKernelGGL(reduce_tile_kernel, dim3((unsigned)ceil_div(rows, 16)), dim3(256), 0, s,
                         (const float*)part, splits, rows, l, lp, (float*)out, tr);
      return hipGetLastError();
    }
  }
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((reduce_parts_kernel<CT, OT>), dim3((unsigned)blocks), dim3(256), 0, s, part, splits,
                     rows, l, lp, out, tr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Planning and dispatch
// ---------------------------------------------------------------------------
static int vec_width(const void* X, int64_t ldx, int esize) {
  uintptr_t a = (uintptr_t)X;
  if (ldx % 4 == 0 && a % (4 * esize) == 0) return 4;
  if (ldx % 2 == 0 && a % (2 * esize) == 0) return 2;
  return 1;
}

// Streamed NN (nn2_kernel) plan: G row groups x S reduction splits.  The
// bytes entering the CUs are X once, the small operand once per row group,
// and the split partials written and read back; a plan that leaves CUs idle
// or needs a second round of workgroups is charged for it.
static constexpr int NN2_KU = 2, NN2_RWMAX = 4, NN2_LDS_KB = 160;

static void plan_nn2(XPlan& p, int64_t m, int64_t n, int l, int cdt, int cus) {
  p.use2 = 0;
  const int nt = ceil_div(l, 16);
  if (!(cdt == 1 || cdt == 2) || nt > 8 || m < 16) return;
  const int lp = nt * 16;
  const int ks = (cdt == 2) ? 32 : 16, stage = ks * NN2_KU;
  const int af = nt;  // operand blocks per stage
  int ntmax = NN2_LDS_KB * 1024 / 2 / NN2_BLOCK - af;
  if (ntmax > 8 * NN2_RWMAX) ntmax = 8 * NN2_RWMAX;
  if (ntmax < 1) return;
  const int64_t tiles = ceil_div(m, 16);
  const int64_t gmin = ceil_div(tiles, ntmax);
  const double xbytes = (double)m * n * (cdt == 2 ? 2 : 4);
  const double abytes = (double)n * lp * 4.0;
  double best = 0.0;
  for (int sp = 1; sp <= 16; ++sp) {
    if (sp > 1 && n < (int64_t)sp * stage * 2) break;
    int64_t g = cus / sp;
    if (g < gmin) g = gmin;
    if (g > tiles) g = tiles;
    if (g < 1) g = 1;
    const int64_t klen = round_up((size_t)ceil_div(n, sp), (size_t)stage);
    const int se = (int)ceil_div(n, klen);
    const int64_t wgs = g * se;
    const int64_t rounds = ceil_div(wgs, cus);
    const double util = (double)wgs / (double)(rounds * cus);
    const double bytes = xbytes + (double)g * abytes + (se > 1 ? 2.0 * se * m * lp * 4.0 : 0.0);
    const double cost = bytes / util;
    if (!p.use2 || cost < best) {
      best = cost;
      p.use2 = 1;
      p.g2 = (int)g;
      p.s2 = se;
      p.klen2 = klen;
      p.lds2 = (size_t)2 * ((size_t)ceil_div(tiles, g) + af) * NN2_BLOCK;
    }
  }
}

XPlan plan_nn(int64_t m, int64_t n, int l, int cdt, int cus) {
  XPlan p;
  const int lp = ceil_div(l, 16) * 16;
  const int rows_wg = (cdt == 0) ? 64 : 128;
  const int wg_m = ceil_div(m, rows_wg);
  int target = 2 * cus;
  int splits = wg_m >= target ? 1 : ceil_div(target, wg_m);
  int maxs = (int)(n / 256);
  if (maxs < 1) maxs = 1;
  if (splits > maxs) splits = maxs;
  if (splits > 64) splits = 64;
  p.splits = splits;
  p.part_elems = splits > 1 ? (size_t)splits * (size_t)m * (size_t)lp : 0;
  plan_nn2(p, m, n, l, cdt, cus);
  if (p.use2 && p.s2 > 1) {
    size_t e2 = (size_t)p.s2 * (size_t)m * (size_t)lp;
    if (e2 > p.part_elems) p.part_elems = e2;
  }
  return p;
}

// Streamed TN (tn2_kernel) plan: 512-column blocks x S row splits.  Bytes:
// X once, Q^T once per column block, split partials written and read back.
static void plan_tn2(XPlan& p, int64_t m, int64_t n, int l, int cdt, int cus) {
  p.use2 = 0;
  const int nt = ceil_div(l, 16);
  if (!(cdt == 1 || cdt == 2) || nt > 8 || m < 32) return;
  const int lp = nt * 16;
  const int64_t nb = ceil_div(n, 512);
  const double xbytes = (double)m * n * (cdt == 2 ? 2 : 4);
  const double qbytes = (double)m * lp * 4.0;
  double best = 0.0;
  for (int64_t sp = 1; sp <= 1024; sp = (sp < 8) ? sp + 1 : sp * 2) {
    int64_t spl = sp;
    if (spl * 64 > m) break;
    const int64_t mlen = round_up((size_t)ceil_div(m, spl), 32);
    const int64_t se = ceil_div(m, mlen);
    const int64_t wgs = nb * se;
    const int64_t rounds = ceil_div(wgs, cus);
    const double util = (double)wgs / (double)(rounds * cus);
    const double bytes = xbytes + (double)nb * qbytes + 2.0 * se * n * lp * 4.0;
    const double cost = bytes / util;
    if (!p.use2 || cost < best) {
      best = cost;
      p.use2 = 1;
      p.g2 = (int)nb;
      p.s2 = (int)se;
      p.klen2 = mlen;
    }
  }
  {  // the split count that exactly fills the CUs
    int64_t spl = cus / nb;
    if (spl >= 1 && spl * 64 <= m) {
      const int64_t mlen = round_up((size_t)ceil_div(m, spl), 32);
      const int64_t se = ceil_div(m, mlen);
      const int64_t wgs = nb * se;
      const int64_t rounds = ceil_div(wgs, cus);
      const double util = (double)wgs / (double)(rounds * cus);
      const double cost = (xbytes + (double)nb * qbytes + 2.0 * se * n * lp * 4.0) / util;
      if (!p.use2 || cost < best) {
        p.use2 = 1;
        p.g2 = (int)nb;
        p.s2 = (int)se;
        p.klen2 = mlen;
      }
    }
  }
  const int es = (cdt == 2) ? 2 : 4;
  p.lds2 = (size_t)2 * (32 * (512 * es + 16) + (size_t)2 * nt * 1024);  // two stages: X rows + Q^T fragments
}

XPlan plan_tn(int64_t m, int64_t n, int l, int cdt, int cus) {
  XPlan p;
  const int lp = ceil_div(l, 16) * 16;
  const int wg_n = ceil_div(n, 256);
  int target = 2 * cus;
  int splits = ceil_div(target, wg_n);
  int maxs = (int)(m / 64);
  if (maxs < 1) maxs = 1;
  if (splits > maxs) splits = maxs;
  if (splits > 512) splits = 512;
  if (splits < 1) splits = 1;
  p.splits = splits;
  p.part_elems = (size_t)splits * (size_t)n * (size_t)lp;
  plan_tn2(p, m, n, l, cdt, cus);
  if (p.use2) {
    size_t e2 = (size_t)p.s2 * (size_t)n * (size_t)lp;
    if (e2 > p.part_elems) p.part_elems = e2;
  }
  return p;
}

#define NT_SWITCH(NTV, CALL)        \
  switch (NTV) {                    \
    case 1: { constexpr int NT = 1; CALL; } break; \
    case 2: { constexpr int NT = 2; CALL; } break; \
    case 3: { constexpr int NT = 3; CALL; } break; \
    case 4: { constexpr int NT = 4; CALL; } break; \
    case 5: { constexpr int NT = 5; CALL; } break; \
    case 6: { constexpr int NT = 6; CALL; } break; \
    case 7: { constexpr int NT = 7; CALL; } break; \
    default: { constexpr int NT = 8; CALL; } break; \
  }

template <typename E, int NT>
static hipError_t launch_nn2_t(dim3 grid, const XPlan& pl, hipStream_t s, const E* X, int64_t m, int64_t n,
                               int64_t ldx, const E* At, int64_t ldat, int lp, int l, float* Y, float* part,
                               int tiles, unsigned* status, int check, const unsigned* skip) {
  auto fn = nn2_kernel<E, NT, NN2_KU, NN2_RWMAX>;
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds2);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, grid, dim3(512), pl.lds2, s, X, m, n, ldx, At, ldat, lp, l, Y, part, pl.klen2, tiles,
                     pl.g2, status, check, skip);
  return hipGetLastError();
}

hipError_t launch_nn(const void* X, int cdt, int64_t m, int64_t n, int64_t ldx, const void* At, int64_t ldat,
                     int l, void* Y, void* part, const XPlan& pl, unsigned* status, int check, hipStream_t s,
                     const unsigned* skip) {
  const int ntile = ceil_div(l, 16);
  const int lp = ntile * 16;
  const int splits = pl.splits;
  if (pl.use2 && (cdt == 1 || cdt == 2) && ldat % 64 == 0 &&
      ((cdt == 1 && vec_width(X, ldx, 4) == 4) || (cdt == 2 && ldx % 8 == 0 && ((uintptr_t)X % 16) == 0))) {
    const int rs = pl.s2;
    dim3 grid((unsigned)pl.g2, (unsigned)rs);
    float* pp = rs > 1 ? (float*)part : nullptr;
    const int tiles = (int)ceil_div(m, 16);
    hipError_t e0;
    if (cdt == 1) {
      NT_SWITCH(ntile, e0 = (launch_nn2_t<float, NT>)(grid, pl, s, (const float*)X, m, n, ldx, (const float*)At, ldat,
                                                    lp, l, (float*)Y, pp, tiles, status, check, skip));
    } else {
      NT_SWITCH(ntile, e0 = (launch_nn2_t<bf16_t, NT>)(grid, pl, s, (const bf16_t*)X, m, n, ldx, (const bf16_t*)At,
                                                     ldat, lp, l, (float*)Y, pp, tiles, status, 0, skip));
    }
    if (e0 != hipSuccess) return e0;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || rs == 1) return e;
    return launch_reduce<float, float>((const float*)part, rs, m, l, lp, (float*)Y, 0, s);
  }
  if (cdt == 1) {
    const int64_t klen = round_up((size_t)ceil_div(n, splits), 16);
    const int rs = ceil_div(n, klen);
    dim3 grid((unsigned)ceil_div(m, 128), (unsigned)rs);
    float* pp = rs > 1 ? (float*)part : nullptr;
    int vw = vec_width(X, ldx, 4);
    if (vw == 4) {
      NT_SWITCH(ntile, hipLaunchKernelGGL((nn_f32_kernel<NT, 4, 2>), grid, dim3(256), 0, s, (const float*)X, m, n,
                                          ldx, (const float*)At, ldat, l, (float*)Y, pp, klen, status, check, skip));
    } else if (vw == 2) {
      NT_SWITCH(ntile, hipLaunchKernelGGL((nn_f32_kernel<NT, 2, 2>), grid, dim3(256), 0, s, (const float*)X, m, n,
                                          ldx, (const float*)At, ldat, l, (float*)Y, pp, klen, status, check, skip));
    } else {
      NT_SWITCH(ntile, hipLaunchKernelGGL((nn_f32_kernel<NT, 1, 2>), grid, dim3(256), 0, s, (const float*)X, m, n,
                                          ldx, (const float*)At, ldat, l, (float*)Y, pp, klen, status, check, skip));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || rs == 1) return e;
    return launch_reduce<float, float>((const float*)part, rs, m, l, lp, (float*)Y, 0, s);
  }
  if (cdt == 2) {
    const int64_t klen = round_up((size_t)ceil_div(n, splits), 32);
    const int rs = ceil_div(n, klen);
    dim3 grid((unsigned)ceil_div(m, 128), (unsigned)rs);
    float* pp = rs > 1 ? (float*)part : nullptr;
    if (ldx % 8 == 0 && ((uintptr_t)X % 16) == 0) {
      NT_SWITCH(ntile, hipLaunchKernelGGL((nn_bf16_kernel<NT, 2>), grid, dim3(256), 0, s, (const bf16_t*)X, m, n,
                                          ldx, (const bf16_t*)At, ldat, lp, l, (float*)Y, pp, klen));
    } else {
      dim3 g2((unsigned)ceil_div(m, 64), (unsigned)rs);
      NT_SWITCH(ntile, hipLaunchKernelGGL((nn_valu_kernel<bf16_t, float, bf16_t, NT>), g2, dim3(256), 0, s,
                                          (const bf16_t*)X, m, n, ldx, (const bf16_t*)At, ldat, lp, l, (float*)Y,
                                          pp, klen, status, 0, skip));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || rs == 1) return e;
    return launch_reduce<float, float>((const float*)part, rs, m, l, lp, (float*)Y, 0, s);
  }
  // FP64
  const int64_t klen = round_up((size_t)ceil_div(n, splits), 16);
  const int rs = ceil_div(n, klen);
  dim3 grid((unsigned)ceil_div(m, 64), (unsigned)rs);
  double* pp = rs > 1 ? (double*)part : nullptr;
  NT_SWITCH(ntile, hipLaunchKernelGGL((nn_valu_kernel<double, double, double, NT>), grid, dim3(256), 0, s,
                                      (const double*)X, m, n, ldx, (const double*)At, ldat, lp, l, (double*)Y,
                                      pp, klen, status, check, skip));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || rs == 1) return e;
  return launch_reduce<double, double>((const double*)part, rs, m, l, lp, (double*)Y, 0, s);
}

template <typename E, int NT>
static hipError_t launch_tn2_t(dim3 grid, const XPlan& pl, hipStream_t s, const E* X, int64_t m, int64_t n,
                               int64_t ldx, const E* Qt, int64_t ldqt, int lp, float* part, int one_plane) {
  auto fn = (sizeof(E) == 2 && one_plane) ? tn2_kernel<E, NT, 1> : tn2_kernel<E, NT, 2>;
  hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds2);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, grid, dim3(512), pl.lds2, s, X, m, n, ldx, Qt, ldqt, lp, part, pl.klen2);
  return hipGetLastError();
}

hipError_t launch_tn(const void* X, int cdt, int64_t m, int64_t n, int64_t ldx, const void* Qt, int64_t ldqt,
                     int l, void* Z, int transposed, void* part, const XPlan& pl, hipStream_t s, int one_plane) {
  const int ntile = ceil_div(l, 16);
  const int lp = ntile * 16;
  const int splits = pl.splits;
  if (pl.use2 && (cdt == 1 || cdt == 2) && ldqt % 64 == 0 &&
      ((cdt == 1 && vec_width(X, ldx, 4) == 4) || (cdt == 2 && ldx % 8 == 0 && ((uintptr_t)X % 16) == 0))) {
    dim3 grid((unsigned)pl.g2, (unsigned)pl.s2);
    hipError_t e0;
    if (cdt == 1) {
      NT_SWITCH(ntile, e0 = (launch_tn2_t<float, NT>)(grid, pl, s, (const float*)X, m, n, ldx, (const float*)Qt,
                                                    ldqt, lp, (float*)part, 0));
    } else {
      NT_SWITCH(ntile, e0 = (launch_tn2_t<bf16_t, NT>)(grid, pl, s, (const bf16_t*)X, m, n, ldx, (const bf16_t*)Qt,
                                                     ldqt, lp, (float*)part, one_plane));
    }
    if (e0 != hipSuccess) return e0;
    return launch_reduce<float, float>((const float*)part, pl.s2, n, l, lp, (float*)Z, transposed, s);
  }
  if (cdt == 1) {
    const int64_t mlen = round_up((size_t)ceil_div(m, splits), 16);
    const int rs = ceil_div(m, mlen);
    int vw = vec_width(X, ldx, 4);
    dim3 grid((unsigned)ceil_div(n, 64 * vw), (unsigned)rs);
    if (vw == 4) {
      NT_SWITCH(ntile, hipLaunchKernelGGL((tn_f32_kernel<NT, 4>), grid, dim3(256), 0, s, (const float*)X, m, n, ldx,
                                          (const float*)Qt, ldqt, (float*)part, mlen));
    } else if (vw == 2) {
      NT_SWITCH(ntile, hipLaunchKernelGGL((tn_f32_kernel<NT, 2>), grid, dim3(256), 0, s, (const float*)X, m, n, ldx,
                                          (const float*)Qt, ldqt, (float*)part, mlen));
    } else {
      NT_SWITCH(ntile, hipLaunchKernelGGL((tn_f32_kernel<NT, 1>), grid, dim3(256), 0, s, (const float*)X, m, n, ldx,
                                          (const float*)Qt, ldqt, (float*)part, mlen));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce<float, float>((const float*)part, rs, n, l, lp, (float*)Z, transposed, s);
  }
  if (cdt == 2) {
    const int64_t mlen = round_up((size_t)ceil_div(m, splits), 32);
    const int rs = ceil_div(m, mlen);
    if (ldx % 4 == 0 && ((uintptr_t)X % 8) == 0) {
      dim3 grid((unsigned)ceil_div(n, 256), (unsigned)rs);
      NT_SWITCH(ntile, hipLaunchKernelGGL((tn_bf16_kernel<NT>), grid, dim3(256), 0, s, (const bf16_t*)X, m, n, ldx,
                                          (const bf16_t*)Qt, ldqt, lp, (float*)part, mlen));
    } else {
      dim3 grid((unsigned)ceil_div(n, 64), (unsigned)rs);
      NT_SWITCH(ntile, hipLaunchKernelGGL((tn_valu_kernel<bf16_t, float, bf16_t, NT>), grid, dim3(256), 0, s,
                                          (const bf16_t*)X, m, n, ldx, (const bf16_t*)Qt, ldqt, lp, (float*)part,
                                          mlen));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce<float, float>((const float*)part, rs, n, l, lp, (float*)Z, transposed, s);
  }
  const int64_t mlen = round_up((size_t)ceil_div(m, splits), 16);
  const int rs = ceil_div(m, mlen);
  dim3 grid((unsigned)ceil_div(n, 64), (unsigned)rs);
  NT_SWITCH(ntile, hipLaunchKernelGGL((tn_valu_kernel<double, double, double, NT>), grid, dim3(256), 0, s,
                                      (const double*)X, m, n, ldx, (const double*)Qt, ldqt, lp, (double*)part, mlen));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce<double, double>((const double*)part, rs, n, l, lp, (double*)Z, transposed, s);
}

}  // namespace rnmf

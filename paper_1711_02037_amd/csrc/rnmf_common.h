// Internal declarations shared by the HIP translation units of librnmf.
// Every kernel is launched through a host wrapper defined in the same file as
// the kernel, so the library needs no relocatable device code.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <cstddef>
#include <cstdint>

struct rnmf_problem;

namespace rnmf {

typedef unsigned long long u64;
typedef uint16_t bf16_t;  // raw bfloat16 bits

// Device status word bits (first 4 bytes of every workspace).
enum : unsigned {
  ST_NONFINITE = 1u << 0,
  ST_NEGATIVE = 1u << 1,
  ST_NOT_SPD = 1u << 2,
  ST_SHIFTED = 1u << 3,      // informational: a shifted Cholesky QR pass ran
  ST_TIMEOUT = 1u << 4,
  ST_NONFINITE_SWEEP = 1u << 5,
};

constexpr int LMAX = 128;  // largest sketch width the kernels support
constexpr int KMAX = 64;   // largest rank the sweep kernel supports
constexpr int GRAM_ROWS_MAX = 96;  // most rows of a short-wide FP64 Gram (hgram_kernel)
constexpr int LSVD = 96;           // largest sketch width of the SVD-based initialization

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

// Bump allocator over the caller's workspace.  With base == nullptr it only
// counts bytes, so the same planning code sizes and carves the workspace.
struct Arena {
  char* base;
  size_t used;
  explicit Arena(void* b) : base((char*)b), used(0) {}
  template <typename T>
  T* take(size_t count) {
    size_t off = round_up(used, 256);
    used = off + round_up(count * sizeof(T), 256);
    return base ? (T*)(base + off) : (T*)nullptr;
  }
};

struct Dev {
  hipStream_t stream;
  int cus;        // compute units
  int max_lds;    // bytes of LDS per workgroup
};

// ---------------------------------------------------------------------------
// Host launch wrappers (each returns hipSuccess or the launch error)
// ---------------------------------------------------------------------------

// misc.hip
hipError_t launch_fill_u32(unsigned* p, size_t count, unsigned v, hipStream_t s);
// dist: 0 standard normal, 1 uniform [0, 1), 2 standard normal with the
// negative entries set to zero
hipError_t launch_philox_raw(const unsigned* ctr, const unsigned* key, unsigned* out, int64_t count,
                             hipStream_t s);
hipError_t launch_philox(void* out, int dt, int64_t rows, int64_t cols, uint64_t seed,
                         unsigned stream_id, int dist, hipStream_t s);
hipError_t launch_cast_bf16(const float* X, int64_t m, int64_t n, int64_t ldx, bf16_t* Xb,
                            int64_t ldb, unsigned* status, int check, hipStream_t s);
hipError_t launch_check_input(const void* X, int dt, int64_t m, int64_t n, int64_t ldx,
                              unsigned* status, hipStream_t s);
// relerr partial sums; `part` holds 2 doubles per workgroup; `out` 2 doubles
hipError_t launch_relerr(const void* X, int xt, int dt, int64_t m, int64_t n, int64_t ldx,
                         const void* W, const void* H, int k, double* part, int nparts_max,
                         double* out, hipStream_t s);
int relerr_parts(int64_t m, int64_t n);

// xpass.hip: passes over X.
// Small operand packing: src (rows x cols, ld = cols, dtype dt) -> dst, the
// transpose (lp x ldp, ldp >= rows) in the compute dtype; rows i >= cols are
// zero.  For bf16 the destination holds hi then lo planes (lo zero when
// hi_only: the operand rounded to bfloat16).
hipError_t launch_pack_t(const void* src, int dt, int64_t rows, int cols, int lp, int64_t ldp,
                         void* dst, int cdt, hipStream_t s, int hi_only = 0);
// Y (m x l) = X (m x n) * A, with At = A^T packed (lp x ldat).  Output in dt
// (float or double).  Split-K partials in `part` (float or double) if needed.
struct XPlan {
  int splits;           // reduction splits of the register-blocked kernels
  size_t part_elems;    // partial-sum elements the workspace must hold
  int use2 = 0;         // streamed NN kernel applicable (FP32/BF16, l <= 128)
  int g2 = 0, s2 = 0;   // its row groups and reduction splits
  int64_t klen2 = 0;    // reduction length per split
  size_t lds2 = 0;      // its LDS bytes
};
XPlan plan_nn(int64_t m, int64_t n, int l, int cdt, int cus);
XPlan plan_tn(int64_t m, int64_t n, int l, int cdt, int cus);
hipError_t launch_nn(const void* X, int cdt, int64_t m, int64_t n, int64_t ldx, const void* At,
                     int64_t ldat, int l, void* Y, void* part, const XPlan& pl,
                     unsigned* status, int check, hipStream_t s,
                     const unsigned* skip = nullptr);
// Z = X^T Q: writes Z (n x l) if !transposed, else Z^T (l x n).  bf16 with
// one_plane: the streamed kernel reads only the hi plane of Qt (whose lo
// plane the other kernels then read as zeros, see launch_pack_t's hi_only).
hipError_t launch_tn(const void* X, int cdt, int64_t m, int64_t n, int64_t ldx, const void* Qt,
                     int64_t ldqt, int l, void* Z, int transposed, void* part,
                     const XPlan& pl, hipStream_t s, int one_plane = 0);

// qr.hip: Cholesky QR pass pieces.
int gram_splits(int64_t rows, int cus);
hipError_t launch_gram(const void* Y, int dt, int64_t rows, int l, double* gpart, int splits,
                       double* G, hipStream_t s, const unsigned* skip = nullptr);
// Fixed-order sum of Gram partials (entry (a, b), a <= b, at a * LMAX + b).
hipError_t launch_gram_sum(const double* gpart, int splits, int l, double* G, hipStream_t s);

// hals.hip: deterministic HALS pieces (dt: 0 FP64, 1 FP32).
// Regularization weights of the HALS rules (ridge alpha, LASSO beta; Sec. 3.4).
struct Reg {
  double aw, ah, bw, bh;
};

hipError_t launch_hrow(const void* R, const double* S, void* H, int64_t n, int k, double ah, double bh, int dt,
                       hipStream_t s);
hipError_t launch_wrow(const void* Tm, const double* V, void* W, int64_t m, int k, double aw, double bw, int dt,
                       hipStream_t s);
hipError_t launch_pad(const void* H, int k, int64_t n, int lp, int64_t ldp, void* Hp, int dt, hipStream_t s);
int hgram_splits(int64_t n);
hipError_t launch_hgram(const void* H, int k, int64_t n, double* part, int dt, hipStream_t s);

// Reverse mode through unrolled sweeps (adjoint.hip).  dt: 0 = double
// states, 1 = float states; adjoints are FP64.
hipError_t ad_gemm_sd(int64_t M, int64_t N, int64_t K, const void* A, int adt, int64_t lda, int ta, const void* B,
                      int bdt, int64_t ldb, int tb, double* C, int64_t ldc, double alpha, int acc, hipStream_t s);
struct WrevShape {
  int G, GR, GC;
  int64_t rows_per;
  bool res;  // the Q slab stays in LDS
  size_t lds_bytes;
};
WrevShape plan_wrev(int64_t m, int l, int k, int dt, int cus, int max_lds);
size_t wrev_ws_words(const WrevShape& sh);
hipError_t ad_wrev(const WrevShape& sh, const void* Q, const void* Wn, const double* V, int64_t m, int l, int k,
                   double* gW, double* gWt, double* GU, u64* xbuf, unsigned* status, int dt, hipStream_t s);
hipError_t ad_wpost_run(const void* Wto, const void* Wtn, const double* Tm, const double* V, const double* GU,
                        int l, int k, double* gT, double* gV, int dt, hipStream_t s);
hipError_t ad_hrows_run(const void* Hn, const double* S, int64_t n, int k, double* gH, double* gA, int dt,
                        hipStream_t s);
int ad_wgram_splits(int64_t m, int cus);
hipError_t ad_wgram_run(const void* W, int64_t m, int k, double* part, int splits, double* S, int dt, hipStream_t s);
hipError_t ad_symm_pad_run(const double* G, int k, double* Mp, hipStream_t s);
// C (M x K) += A Mp with Mp the K x K factor zero-padded to 64 x 64
hipError_t ad_rowmat_run(const void* A, const double* Mm, int64_t M, int K, double* C, int dt, hipStream_t s);
hipError_t ad_gs_run(const void* Hn, const void* Ho, const double* gA, const double* S, int64_t n, int k,
                     double* gS, int dt, hipStream_t s);
hipError_t ad_scale_rows_run(double* gA, const double* S, int64_t n, int k, hipStream_t s);
hipError_t ad_symm_run(const double* G, int k, double* M, hipStream_t s);
hipError_t ad_fill_run(double* p, int64_t count, double v, hipStream_t s);

// Sweeps with an explicit order of block updates (ordered.hip).  Entry e < k
// updates column e of W, entry e >= k row e - k of H.  part holds
// ord_part_elems doubles, vec l + k doubles.
int ord_part_elems(int64_t m, int64_t n, int l, int k);
hipError_t launch_ordered_update(const void* Q, const void* B, void* W, void* Wt, void* H, int64_t m, int64_t n,
                                 int l, int k, int e, double* part, double* vec, int dt, hipStream_t s);

// SVD-based initialization (svdinit.hip).  Workspace pieces, all FP64:
// gpart (hgram_splits(n) x LMAX x LMAX), C (l x l), Ub (l x k), sv (k),
// upart (svd_row_blocks(m) x k x 2), vpart (svd_col_blocks(n) x k x 2),
// coef (k x 3).
struct SvdBufs {
  double *gpart, *C, *Ub, *sv, *upart, *vpart, *coef;
};
// Batched randomized HALS (batch.hip).
size_t batch_desc_bytes();
size_t batch_lds_bytes();
void batch_fill_desc(void* dst, const ::rnmf_problem& p, int idx, int tc, int hct);
bool batch_hct_ok(int hct, int l);  // H-phase tile width valid for sketch width l
hipError_t launch_batch(const void* descs, int nprob, int q, int nsweeps, unsigned* counter, double* err,
                        unsigned* status, int grid, hipStream_t s);

int svd_row_blocks(int64_t m);
int svd_col_blocks(int64_t n);
hipError_t launch_svd_init(const void* Q, const void* B, int64_t m, int64_t n, int l, int k, void* W, void* H,
                           int dt, const SvdBufs& b, hipStream_t s);

// One workgroup: Cholesky of G (l x l, FP64) with optional shift; writes the
// transposed inverse factor packed for the GEMM (lp x lp, dtype cdt) and
// updates flags.  `pass_ctl`: 0 first pass of a pair, 1 second pass, 2 extra.
hipError_t launch_chol(double* G, int l, int64_t rows, void* RinvT, int lp, int cdt,
                       unsigned* ctl, int pass, int allow_shift, unsigned* status,
                       hipStream_t s);

// sweep.hip
struct SweepShape {
  int G, GR, GC, rows_per, cols_per, rows_lds, cb, nt, red2_elems, alias_sv, regq;
  int xown;  // dedicated exchange-owner workgroups (the last xown of G; no rows or columns)
  int wglobal;  // register-Q path with the W rows in global memory instead of LDS
  size_t lds_bytes;
};
SweepShape plan_sweep(int64_t m, int64_t n, int l, int k, int dt, const Dev& d, bool need_pg);
size_t sweep_ws_words(const SweepShape& sh, int l);
hipError_t launch_sweep(const SweepShape& sh, int dt, const void* Q, const void* B, void* W,
                        void* Wt, void* H, int64_t m, int64_t n, int l, int k, int nsweeps,
                        double tol, int gram_mode, int order, const Reg& reg, u64* xbuf, double* stats,
                        unsigned* status, u64* trace, hipStream_t s);

}  // namespace rnmf

// Host side of librnmf: argument checks, workspace planning and the order of
// kernel launches for each entry point of include/rnmf.h.
//
// The workspace is carved by one bump allocator (Arena); the size query runs
// the same planning code with a null base, so the two always agree.
#include "rnmf.h"
#include "rnmf_common.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>
#include <algorithm>

using namespace rnmf;

namespace {

thread_local std::string g_err;

rnmf_status fail(rnmf_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(RNMF_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t HDR_BYTES = 4096;
constexpr size_t TRACE_OFFSET = 1024;  // phase timestamps of a traced sweep
// header layout (bytes): 0 status u32, 4 QR control u32, 64 stats (8 doubles),
// 128 relative-error sums (2 doubles)
struct Hdr {
  unsigned* status;
  unsigned* ctl;
  double* stats;
  double* rel;
};
Hdr header(void* ws) {
  char* b = (char*)ws;
  return Hdr{(unsigned*)b, (unsigned*)(b + 4), (double*)(b + 64), (double*)(b + 128)};
}

bool get_dev(Dev& d, hipStream_t s) {
  int id = 0;
  if (hipGetDevice(&id) != hipSuccess) return false;
  static std::mutex mu;
  static int cache_cus[64] = {0}, cache_lds[64] = {0};
  std::lock_guard<std::mutex> lk(mu);
  if (id < 0 || id >= 64) return false;
  if (cache_cus[id] == 0) {
    int cus = 0, lds = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, id) != hipSuccess) return false;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, id) != hipSuccess) return false;
    cache_cus[id] = cus;
    cache_lds[id] = lds;
  }
  d.stream = s;
  d.cus = cache_cus[id];
  d.max_lds = cache_lds[id];
  return true;
}

// Device properties for sizing when no device is usable (size queries on a
// host without a GPU): MI355X values.
Dev default_dev() { return Dev{nullptr, 256, 160 * 1024}; }

struct Mode {
  int dt;    // factor dtype: 0 f64, 1 f32
  int cdt;   // X-pass compute: 0 f64, 1 f32, 2 bf16
  int gdt;   // GEMM dtype of the orthonormalisation: 0 f64, 1 f32
  size_t es; // bytes per factor element
};

Mode mode_of(const rnmf_opts* o) {
  Mode md;
  if (o->prec == RNMF_PREC_F64) { md.dt = 0; md.cdt = 0; md.gdt = 0; md.es = 8; }
  else if (o->prec == RNMF_PREC_F32) { md.dt = 1; md.cdt = 1; md.gdt = 1; md.es = 4; }
  else { md.dt = 1; md.cdt = 2; md.gdt = 1; md.es = 4; }
  return md;
}

int q_effective(const rnmf_opts* o) {
  int q = o->q;
  if (o->prec == RNMF_PREC_BF16 && !(o->flags & RNMF_FLAG_EXACT_Q)) q += 1;
  return q;
}

int lwidth(const rnmf_opts* o, int64_t m, int64_t n) {
  int64_t l = (int64_t)o->k + o->p;
  if (l > m) l = m;
  if (l > n) l = n;
  return (int)l;
}

rnmf_status check_reg(const rnmf_opts* o) {
  const double w[4] = {o->alpha_w, o->alpha_h, o->beta_w, o->beta_h};
  for (double v : w)
    if (!(v >= 0.0) || !(v < INFINITY))
      return fail(RNMF_ERR_ARG, "regularization weights must be finite and >= 0");
  return RNMF_OK;
}

Reg reg_of(const rnmf_opts* o) { return Reg{o->alpha_w, o->alpha_h, o->beta_w, o->beta_h}; }

rnmf_status check_opts(const rnmf_opts* o, int64_t m, int64_t n, bool need_kmax) {
  if (!o) return fail(RNMF_ERR_ARG, "opts is NULL");
  if (o->reserved != 0) return fail(RNMF_ERR_ARG, "opts.reserved must be 0");
  if (m < 1 || n < 1) return fail(RNMF_ERR_SHAPE, "empty matrix (m=%lld, n=%lld)", (long long)m, (long long)n);
  if (m > 0x7fffffffLL || n > 0x7fffffffLL) return fail(RNMF_ERR_SHAPE, "m and n must be below 2^31");
  if (o->k < 1 || (int64_t)o->k >= (m < n ? m : n))
    return fail(RNMF_ERR_ARG, "need 1 <= k < min(m, n) (k=%d, m=%lld, n=%lld)", o->k, (long long)m, (long long)n);
  if (o->p < 0) return fail(RNMF_ERR_ARG, "p must be >= 0");
  if (o->q < 0 || o->q > 32) return fail(RNMF_ERR_ARG, "q must be in [0, 32]");
  if (o->max_iter < 0) return fail(RNMF_ERR_ARG, "max_iter must be >= 0");
  if (o->prec < 0 || o->prec > 2) return fail(RNMF_ERR_ARG, "unknown precision mode %d", o->prec);
  if (o->omega_dist < 0 || o->omega_dist > 1) return fail(RNMF_ERR_ARG, "unknown omega_dist %d", o->omega_dist);
  if (o->gram_mode < 0 || o->gram_mode > 2) return fail(RNMF_ERR_ARG, "unknown gram_mode %d", o->gram_mode);
  if (o->order < 0 || o->order > 1) return fail(RNMF_ERR_ARG, "unknown order %d", o->order);
  if (o->flags & ~(RNMF_FLAG_CHECK_INPUT | RNMF_FLAG_NO_SHIFT | RNMF_FLAG_EXACT_Q | RNMF_FLAG_TRACE |
                   RNMF_FLAG_SHIFTED_QR3 | RNMF_FLAG_SVD_INIT | RNMF_FLAG_GAUSS_INIT))
    return fail(RNMF_ERR_ARG, "unknown flag bits 0x%x", o->flags);
  if (!(o->tol == o->tol)) return fail(RNMF_ERR_ARG, "tol is NaN");
  if (check_reg(o) != RNMF_OK) return RNMF_ERR_ARG;
  int l = lwidth(o, m, n);
  if (l > LMAX) return fail(RNMF_ERR_ARG, "sketch width l = min(k + p, m, n) = %d exceeds %d", l, LMAX);
  if (need_kmax && o->k > KMAX) return fail(RNMF_ERR_ARG, "k = %d exceeds the supported %d", o->k, KMAX);
  if ((o->flags & RNMF_FLAG_SVD_INIT) && l > LSVD)
    return fail(RNMF_ERR_ARG, "the SVD-based initialization needs l <= %d (l = %d)", LSVD, l);
  return RNMF_OK;
}

rnmf_status check_xt(const rnmf_opts* o, int xt) {
  if (o->prec == RNMF_PREC_F64 && xt != RNMF_F64) return fail(RNMF_ERR_DTYPE, "RNMF_PREC_F64 needs X in RNMF_F64");
  if (o->prec == RNMF_PREC_F32 && xt != RNMF_F32) return fail(RNMF_ERR_DTYPE, "RNMF_PREC_F32 needs X in RNMF_F32");
  if (o->prec == RNMF_PREC_BF16 && xt != RNMF_F32 && xt != RNMF_BF16)
    return fail(RNMF_ERR_DTYPE, "RNMF_PREC_BF16 needs X in RNMF_F32 or RNMF_BF16");
  return RNMF_OK;
}

rnmf_status check_ws(void* ws, size_t have, size_t need) {
  if (!ws) return fail(RNMF_ERR_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256) return fail(RNMF_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (have < need) return fail(RNMF_ERR_WORKSPACE, "workspace too small: %zu bytes given, %zu needed", have, need);
  return RNMF_OK;
}

int64_t bf16_ld(int64_t n) { return (int64_t)round_up((size_t)n, 8); }

// ---------------------------------------------------------------------------
// Plans: pointer sets carved from an arena
// ---------------------------------------------------------------------------
struct QrBufs {
  double* gpart;
  double* G;
  void* rinv;
  int gsplits;
};
QrBufs plan_qr(Arena& a, int64_t rows, int l, const Mode& md, const Dev& d) {
  QrBufs b;
  b.gsplits = gram_splits(rows, d.cus);
  b.gpart = a.take<double>((size_t)b.gsplits * LMAX * LMAX);
  b.G = a.take<double>((size_t)l * l);
  int lp = ceil_div(l, 16) * 16;
  b.rinv = a.take<char>((size_t)lp * lp * (md.gdt == 0 ? 8 : 4));
  return b;
}

struct SketchBufs {
  void* om;
  void* at;
  int64_t ldp;
  void* y;
  void* y2;
  void* z;
  void* z2;
  void* z3;
  void* part;
  QrBufs qy, qz;
  XPlan nn, tn, nnq;
};
SketchBufs plan_sketch(Arena& a, int64_t m, int64_t n, int l, const Mode& md, const Dev& d) {
  SketchBufs b;
  const int lp = ceil_div(l, 16) * 16;
  b.ldp = (int64_t)round_up((size_t)(m > n ? m : n), 64);  // streamed NN reads whole 64-wide stages
  b.om = a.take<char>((size_t)n * l * md.es);
  b.at = a.take<char>((size_t)lp * b.ldp * (md.cdt == 0 ? 8 : 4));  // bf16: two planes of 2 bytes
  b.y = a.take<char>((size_t)m * l * md.es);
  b.y2 = a.take<char>((size_t)m * l * md.es);
  b.z = a.take<char>((size_t)n * l * md.es);
  b.z2 = a.take<char>((size_t)n * l * md.es);
  b.z3 = a.take<char>((size_t)n * l * md.es);
  b.nn = plan_nn(m, n, l, md.cdt, d.cus);
  b.tn = plan_tn(m, n, l, md.cdt, d.cus);
  size_t pe = b.nn.part_elems > b.tn.part_elems ? b.nn.part_elems : b.tn.part_elems;
  b.part = a.take<char>(pe * (md.cdt == 0 ? 8 : 4));
  b.qy = plan_qr(a, m, l, md, d);
  b.qz = plan_qr(a, n, l, md, d);
  return b;
}

struct CompressBufs {
  void* at;
  int64_t ldp;
  void* part;
  XPlan tn;
};
CompressBufs plan_compress(Arena& a, int64_t m, int64_t n, int l, const Mode& md, const Dev& d) {
  CompressBufs b;
  const int lp = ceil_div(l, 16) * 16;
  b.ldp = (int64_t)round_up((size_t)m, 64);  // streamed TN reads whole 32-row stages
  b.at = a.take<char>((size_t)lp * b.ldp * (md.cdt == 0 ? 8 : 4));
  b.tn = plan_tn(m, n, l, md.cdt, d.cus);
  b.part = a.take<char>(b.tn.part_elems * (md.cdt == 0 ? 8 : 4));
  return b;
}

struct InitBufs {
  void* at;
  int64_t ldp;
  void* part;
  XPlan tn;
};
InitBufs plan_init(Arena& a, int64_t m, int k, int l, const Mode& md, const Dev& d) {
  InitBufs b;
  const int lp = ceil_div(l, 16) * 16;
  b.ldp = (int64_t)round_up((size_t)m, 64);
  b.at = a.take<char>((size_t)lp * b.ldp * md.es);
  b.tn = plan_tn(m, k, l, md.dt, d.cus);
  b.part = a.take<char>(b.tn.part_elems * md.es);
  return b;
}

SvdBufs plan_svd(Arena& a, int64_t m, int64_t n, int l, int k) {
  SvdBufs b;
  b.gpart = a.take<double>((size_t)hgram_splits(n) * LMAX * LMAX);
  b.C = a.take<double>((size_t)l * l);
  b.Ub = a.take<double>((size_t)l * k);
  b.sv = a.take<double>((size_t)k);
  b.upart = a.take<double>((size_t)svd_row_blocks(m) * k * 2);
  b.vpart = a.take<double>((size_t)svd_col_blocks(n) * k * 2);
  b.coef = a.take<double>((size_t)k * 3);
  return b;
}

struct SweepBufs {
  SweepShape sh;
  u64* xbuf;
};
SweepBufs plan_hals(Arena& a, int64_t m, int64_t n, int l, int k, const Mode& md, const Dev& d, bool need_pg) {
  SweepBufs b;
  b.sh = plan_sweep(m, n, l, k, md.dt, d, need_pg);
  b.xbuf = a.take<u64>(sweep_ws_words(b.sh, l));
  return b;
}

struct DHalsBufs {
  void* wp;         // W packed transposed, lp x ldpm (the TN pass operand)
  int64_t ldpm;
  void* hp;         // H zero-padded, lp x ldpn (the NN pass operand)
  int64_t ldpn;
  void* R;          // X^T W, n x k
  void* T;          // X H^T, m x k
  double* S;        // W^T W, k x k
  double* V;        // H H^T, k x k
  double* gpart;    // Gram partials of W^T W
  int gsplits;
  double* hpart;    // Gram partials of H H^T
  void* part;       // split partials of the X passes
  XPlan nn, tn;
};
DHalsBufs plan_dhals(Arena& a, int64_t m, int64_t n, int k, const Mode& md, const Dev& d) {
  DHalsBufs b;
  const int lp = ceil_div(k, 16) * 16;
  const size_t es = md.es;
  b.ldpm = (int64_t)round_up((size_t)m, 64);
  b.ldpn = (int64_t)round_up((size_t)n, 64);
  b.wp = a.take<char>((size_t)lp * b.ldpm * es);
  b.hp = a.take<char>((size_t)lp * b.ldpn * es);
  b.R = a.take<char>((size_t)n * k * es);
  b.T = a.take<char>((size_t)m * k * es);
  b.S = a.take<double>((size_t)k * k);
  b.V = a.take<double>((size_t)k * k);
  b.gsplits = gram_splits(m, d.cus);
  b.gpart = a.take<double>((size_t)b.gsplits * LMAX * LMAX);
  b.hpart = a.take<double>((size_t)hgram_splits(n) * LMAX * LMAX);
  b.nn = plan_nn(m, n, k, md.cdt, d.cus);
  b.tn = plan_tn(m, n, k, md.cdt, d.cus);
  const size_t pe = b.nn.part_elems > b.tn.part_elems ? b.nn.part_elems : b.tn.part_elems;
  b.part = a.take<char>(pe * es);
  return b;
}

struct RelBufs {
  double* part;
  int np;
};
RelBufs plan_rel(Arena& a, int64_t m, int64_t n) {
  RelBufs b;
  b.np = relerr_parts(m, n);
  b.part = a.take<double>((size_t)2 * b.np);
  return b;
}

// ---------------------------------------------------------------------------
// Orchestration
// ---------------------------------------------------------------------------

// One Cholesky QR pass: out = in * L^{-T} where L = chol(in^T in).  With
// `skip` (the control word), the whole pass is skipped on the device when the
// word is zero; `out` may then equal `in` (the product is row-local).
rnmf_status qr_pass(const void* in, int64_t rows, int l, void* out, const QrBufs& qb, const Mode& md, int extra,
                    unsigned* ctl, int allow_shift, unsigned* status, const Dev& d, const unsigned* skip) {
  hipStream_t s = d.stream;
  const int lp = ceil_div(l, 16) * 16;
  HIPCHK(launch_gram(in, md.dt, rows, l, qb.gpart, qb.gsplits, qb.G, s, skip));
  HIPCHK(launch_chol(qb.G, l, rows, qb.rinv, lp, md.gdt, ctl, extra ? 2 : 0, allow_shift, status, s));
  XPlan pl = plan_nn(rows, l, l, md.gdt, d.cus);
  pl.splits = 1;
  HIPCHK(launch_nn(in, md.gdt, rows, l, l, qb.rinv, lp, l, out, nullptr, pl, status, 0, s, skip));
  return RNMF_OK;
}

// Thin QR by Cholesky QR2 (plus a third pass when the first needed a shift).
// `in` is overwritten.  Result in `out`.  With passes = 1 (the iterates inside
// the subspace iteration, whose span is all the next product uses) one pass,
// plus a second only when the first needed a shift: a Cholesky QR pass
// spans exactly the span of its input, and the final basis still gets two.
rnmf_status cholqr(void* in, int64_t rows, int l, void* out, void* tmp, const QrBufs& qb, const Mode& md,
                   unsigned* ctl, int allow_shift, unsigned* status, const Dev& d, int passes = 2) {
  HIPCHK(launch_fill_u32(ctl, 1, 0u, d.stream));
  rnmf_status r;
  // allow_shift: 0 never shift, 1 shift a pass whose Gram is not numerically
  // positive definite, 2 also shift the first pass unconditionally
  const int later = allow_shift ? 1 : 0;
  if (passes == 1) {
    if ((r = qr_pass(in, rows, l, out, qb, md, 0, ctl, allow_shift, status, d, nullptr)) != RNMF_OK) return r;
    return qr_pass(out, rows, l, out, qb, md, 1, ctl, later, status, d, ctl);
  }
  if ((r = qr_pass(in, rows, l, tmp, qb, md, 0, ctl, allow_shift, status, d, nullptr)) != RNMF_OK) return r;
  if ((r = qr_pass(tmp, rows, l, out, qb, md, 0, ctl, later, status, d, nullptr)) != RNMF_OK) return r;
  // third pass, in place, only after a shifted pass (decided on the device)
  return qr_pass(out, rows, l, out, qb, md, 1, ctl, later, status, d, ctl);
}

rnmf_status run_sketch(const void* Xc, int64_t m, int64_t n, int64_t ldx, const void* Omega, const rnmf_opts* o,
                       void* Q, const SketchBufs& b, const Mode& md, const Hdr& h, int check, const Dev& d) {
  hipStream_t s = d.stream;
  const int l = lwidth(o, m, n);
  const int lp = ceil_div(l, 16) * 16;
  const int allow_shift = (o->flags & RNMF_FLAG_NO_SHIFT) ? 0 : (o->flags & RNMF_FLAG_SHIFTED_QR3) ? 2 : 1;
  const void* om = Omega;
  if (!om) {
    HIPCHK(launch_philox(b.om, md.dt, n, l, o->seed, 3u, o->omega_dist, s));
    om = b.om;
  }
  rnmf_status r;
  // Y = X Omega
  HIPCHK(launch_pack_t(om, md.dt, n, l, lp, b.ldp, b.at, md.cdt, s));
  HIPCHK(launch_nn(Xc, md.cdt, m, n, ldx, b.at, b.ldp, l, b.y, b.part, b.nn, h.status, check, s));
  const int q = q_effective(o);
  for (int it = 0; it < q; ++it) {
    // Q = qr(Y); Z = X^T Q; Q = qr(Z); Y = X Q
    if ((r = cholqr(b.y, m, l, b.y2, Q, b.qy, md, h.ctl, allow_shift, h.status, d, 1)) != RNMF_OK) return r;
    // the half-step Z = X^T Q only steers the subspace: in the BF16 form its
    // operand is Q rounded to bfloat16 (one plane), as in the sketch passes
    HIPCHK(launch_pack_t(b.y2, md.dt, m, l, lp, b.ldp, b.at, md.cdt, s, 1));
    HIPCHK(launch_tn(Xc, md.cdt, m, n, ldx, b.at, b.ldp, l, b.z, 0, b.part, b.tn, s, 1));
    if ((r = cholqr(b.z, n, l, b.z2, b.z3, b.qz, md, h.ctl, allow_shift, h.status, d, 1)) != RNMF_OK) return r;
    HIPCHK(launch_pack_t(b.z2, md.dt, n, l, lp, b.ldp, b.at, md.cdt, s));
    HIPCHK(launch_nn(Xc, md.cdt, m, n, ldx, b.at, b.ldp, l, b.y, b.part, b.nn, h.status, 0, s));
  }
  return cholqr(b.y, m, l, Q, b.y2, b.qy, md, h.ctl, allow_shift, h.status, d);
}

rnmf_status run_compress(const void* Xc, int64_t m, int64_t n, int64_t ldx, const void* Q, int l, void* B,
                         const CompressBufs& b, const Mode& md, const Dev& d) {
  const int lp = ceil_div(l, 16) * 16;
  HIPCHK(launch_pack_t(Q, md.dt, m, l, lp, b.ldp, b.at, md.cdt, d.stream));
  HIPCHK(launch_tn(Xc, md.cdt, m, n, ldx, b.at, b.ldp, l, B, 1, b.part, b.tn, d.stream));
  return RNMF_OK;
}

// W~ = Q^T W
rnmf_status run_init_wt(const void* Q, const void* W, int64_t m, int k, int l, void* Wt, const InitBufs& b,
                        const Mode& md, const Dev& d) {
  const int lp = ceil_div(l, 16) * 16;
  HIPCHK(launch_pack_t(Q, md.dt, m, l, lp, b.ldp, b.at, md.dt, d.stream));
  HIPCHK(launch_tn(W, md.dt, m, k, k, b.at, b.ldp, l, Wt, 1, b.part, b.tn, d.stream));
  return RNMF_OK;
}

rnmf_status status_from_bits(unsigned bits) {
  if (bits & ST_TIMEOUT) return fail(RNMF_ERR_DEVICE_TIMEOUT, "a device-wide wait hit its spin limit");
  if (bits & ST_NONFINITE) return fail(RNMF_ERR_NONFINITE, "X contains NaN or Inf");
  if (bits & ST_NEGATIVE) return fail(RNMF_ERR_NEGATIVE_INPUT, "X contains a negative entry");
  if (bits & ST_NOT_SPD) return fail(RNMF_ERR_NOT_SPD, "Cholesky QR broke down");
  if (bits & ST_NONFINITE_SWEEP) return fail(RNMF_ERR_NONFINITE, "a sweep produced NaN or Inf");
  return RNMF_OK;
}

size_t factorize_bytes(int64_t m, int64_t n, const rnmf_opts* o, int xt, const Dev& d, void* base,
                       void** pQ, void** pB, void** pWt, void** pXb, SketchBufs* sb, CompressBufs* cb, InitBufs* ib,
                       SweepBufs* wb, RelBufs* rb, SvdBufs* vb = nullptr) {
  const Mode md = mode_of(o);
  const int l = lwidth(o, m, n);
  Arena a(base);
  a.take<char>(HDR_BYTES);
  void* Q = a.take<char>((size_t)m * l * md.es);
  void* B = a.take<char>((size_t)l * n * md.es);
  void* Wt = a.take<char>((size_t)l * o->k * md.es);
  // the stage buffers (a union) start at the same offset in every precision
  // form; the BF16 copy of X goes after them, so that the sweep's exchange
  // words sit at the same addresses in both forms of one workspace (the
  // sweep's speed depends a few percent on where they sit)
  const size_t start = round_up(a.used, 256);
  size_t mx = 0;
  char* sub = base ? (char*)base + start : nullptr;
  { Arena s(sub); SketchBufs t = plan_sketch(s, m, n, l, md, d); if (sb) *sb = t; mx = s.used > mx ? s.used : mx; }
  { Arena s(sub); CompressBufs t = plan_compress(s, m, n, l, md, d); if (cb) *cb = t; mx = s.used > mx ? s.used : mx; }
  { Arena s(sub); InitBufs t = plan_init(s, m, o->k, l, md, d); if (ib) *ib = t; mx = s.used > mx ? s.used : mx; }
  { Arena s(sub); SweepBufs t = plan_hals(s, m, n, l, o->k, md, d, o->tol > 0.0); if (wb) *wb = t; mx = s.used > mx ? s.used : mx; }
  { Arena s(sub); RelBufs t = plan_rel(s, m, n); if (rb) *rb = t; mx = s.used > mx ? s.used : mx; }
  if (o->flags & RNMF_FLAG_SVD_INIT) {
    Arena s(sub);
    SvdBufs t = plan_svd(s, m, n, l, o->k);
    if (vb) *vb = t;
    mx = s.used > mx ? s.used : mx;
  }
  void* Xb = nullptr;
  size_t end = start + mx;
  if (md.cdt == 2 && xt == RNMF_F32) {
    end = round_up(end, 256);
    Xb = base ? (void*)((char*)base + end) : nullptr;
    end += round_up((size_t)m * bf16_ld(n) * sizeof(bf16_t), 256);
  }
  if (pQ) *pQ = Q;
  if (pB) *pB = B;
  if (pWt) *pWt = Wt;
  if (pXb) *pXb = Xb;
  return end;
}

size_t op_bytes(int op, int64_t m, int64_t n, const rnmf_opts* o, int xt, const Dev& d) {
  const Mode md = mode_of(o);
  const int l = lwidth(o, m, n);
  Arena a(nullptr);
  a.take<char>(HDR_BYTES);
  switch (op) {
    case RNMF_OP_SKETCH:
      if (md.cdt == 2 && xt == RNMF_F32) a.take<bf16_t>((size_t)m * bf16_ld(n));
      plan_sketch(a, m, n, l, md, d);
      return a.used;
    case RNMF_OP_COMPRESS: {
      int64_t lc = (int64_t)o->k + o->p;
      if (lc > m) lc = m;
      if (md.cdt == 2 && xt == RNMF_F32) a.take<bf16_t>((size_t)m * bf16_ld(n));
      plan_compress(a, m, n, (int)lc, md, d);
      return a.used;
    }
    case RNMF_OP_HALS_STEP:
      plan_hals(a, m, n, l, o->k, md, d, o->tol > 0.0);
      return a.used;
    case RNMF_OP_REL_ERROR:
      plan_rel(a, m, n);
      return a.used;
    case RNMF_OP_HALS:
      plan_dhals(a, m, n, o->k, md, d);
      return a.used;
    case RNMF_OP_FACTORIZE:
      return factorize_bytes(m, n, o, xt, d, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                             nullptr, nullptr, nullptr);
    case RNMF_OP_SVD_INIT:
      plan_svd(a, m, n, l, o->k);
      return a.used;
    default:
      return 0;
  }
}

// Resolves the X operand actually streamed (casting to BF16 into ws if needed).
// ---- batched runs ----------------------------------------------------------
struct BatchLayout {
  unsigned* counter;
  void* descs;
  double* err;
  unsigned* status;
  size_t bytes;
};
BatchLayout batch_layout(void* ws, int nprob) {
  Arena a(ws);
  BatchLayout L;
  L.counter = a.take<unsigned>(64);
  L.descs = a.take<char>((size_t)nprob * batch_desc_bytes());
  L.err = a.take<double>(2 * (size_t)nprob);
  L.status = a.take<unsigned>((size_t)nprob);
  L.bytes = a.used;
  return L;
}

// Per sketch-width class (l <= 16, 32, 48, 64): X-pass column groups
// (entries 0-3) and H-phase tile widths (entries 4-7).  The autotune table,
// the library's only global state.
std::mutex g_batch_mu;
int g_batch_tc[8] = {4, 8, 16, 16, 256, 256, 128, 128};

int l_class(int l) { return l <= 16 ? 0 : (l <= 32 ? 1 : (l <= 48 ? 2 : 3)); }

rnmf_status check_problem(const rnmf_problem& p, int i) {
  if (!p.X || !p.Omega || !p.W0 || !p.H0 || !p.W || !p.H || !p.Q || !p.B || !p.Z)
    return fail(RNMF_ERR_ARG, "problem %d: every pointer must be non-NULL", i);
  if (p.m < 1 || p.n < 1 || p.m > 0x7fffffffLL || p.n > 0x7fffffffLL)
    return fail(RNMF_ERR_SHAPE, "problem %d: bad m or n", i);
  if (p.ldx < p.n) return fail(RNMF_ERR_SHAPE, "problem %d: ldx < n", i);
  if (p.l < 1 || p.l > 64 || p.l > p.m || p.l > p.n)
    return fail(RNMF_ERR_SHAPE, "problem %d: need 1 <= l <= min(64, m, n) (l = %d)", i, p.l);
  if (p.k < 1 || p.k > 32 || p.k > p.l) return fail(RNMF_ERR_ARG, "problem %d: need 1 <= k <= min(32, l)", i);
  if (p.prec != RNMF_PREC_F32 && p.prec != RNMF_PREC_BF16)
    return fail(RNMF_ERR_ARG, "problem %d: prec must be RNMF_PREC_F32 or RNMF_PREC_BF16", i);
  if (p.reserved != 0) return fail(RNMF_ERR_ARG, "problem %d: reserved must be 0", i);
  return RNMF_OK;
}

// Descriptors in cost order (largest first; ties by index), tiling per class.
rnmf_status upload_plan(const rnmf_problem* probs, int nprob, const BatchLayout& L, const int* table,
                        std::vector<int>* order_out, hipStream_t s) {
  std::vector<int> order((size_t)nprob);
  std::vector<double> cost((size_t)nprob);
  for (int i = 0; i < nprob; ++i) {
    const rnmf_problem& p = probs[i];
    order[i] = i;
    // X passes plus 100 sweeps of lift and map-back, in multiply-adds
    cost[i] = 8.0 * p.m * p.n * p.l + 400.0 * p.m * p.l * p.k;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  const size_t db = batch_desc_bytes();
  std::vector<char> host((size_t)nprob * db);
  for (int j = 0; j < nprob; ++j) {
    const rnmf_problem& p = probs[order[j]];
    int tc = table[l_class(p.l)];
    while (4 * tc < p.l) tc *= 2;
    int hct = table[4 + l_class(p.l)];
    while (!batch_hct_ok(hct, p.l) && hct > 64) hct /= 2;
    batch_fill_desc(host.data() + (size_t)j * db, p, order[j], tc, hct);
  }
  HIPCHK(hipMemcpyAsync(L.descs, host.data(), host.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  if (order_out) *order_out = order;
  return RNMF_OK;
}

rnmf_status prepare_x(const void* X, int xt, int64_t m, int64_t n, int64_t ldx, const rnmf_opts* o, const Mode& md,
                      void* xb_slot, const Hdr& h, const Dev& d, const void** Xc, int64_t* ldc, int* check_in_pass) {
  const int check = (o->flags & RNMF_FLAG_CHECK_INPUT) ? 1 : 0;
  *check_in_pass = 0;
  if (md.cdt == 2 && xt == RNMF_F32) {
    int64_t ldb = bf16_ld(n);
    HIPCHK(launch_cast_bf16((const float*)X, m, n, ldx, (bf16_t*)xb_slot, ldb, h.status, check, d.stream));
    *Xc = xb_slot;
    *ldc = ldb;
  } else {
    *Xc = X;
    *ldc = ldx;
    *check_in_pass = (md.cdt != 2) ? check : 0;
  }
  return RNMF_OK;
}


// ---------------------------------------------------------------------------
// Reverse mode through unrolled sweeps
// ---------------------------------------------------------------------------
struct State {
  void* W;   // m x k
  void* Wt;  // l x k
  void* H;   // k x n
};
State take_state(Arena& a, int64_t m, int64_t n, int l, int k, size_t es) {
  State st;
  st.W = a.take<char>((size_t)m * k * es);
  st.Wt = a.take<char>((size_t)l * k * es);
  st.H = a.take<char>((size_t)k * n * es);
  return st;
}

struct BackBufs {
  SweepBufs sw;
  std::vector<State> ckpt;  // states at the start of segments 1..nseg-1
  std::vector<State> seg;   // the states of one segment, len + 1 of them
  double *gWt, *gA, *gT, *gV, *gS, *Msym, *Mpad, *S, *Tm, *V, *GU;
  double *gpart, *hpart;  // Gram partials of W^T W and of H H^T
  WrevShape wsh;          // the persistent reverse W phase
  u64* wx;                // its exchange slots
  int gsplits, hsplits;
  int nseg, len;
};
BackBufs plan_backward(Arena& a, int64_t m, int64_t n, int l, int k, int T, int ckpt, const Mode& md,
                       const Dev& d) {
  BackBufs b;
  b.sw = plan_hals(a, m, n, l, k, md, d, false);
  // ckpt == 0: the caller recorded every state; nothing is recomputed
  b.len = ckpt == 0 ? 0 : (T < ckpt ? T : ckpt);
  b.nseg = (T == 0 || ckpt == 0) ? 0 : (T + ckpt - 1) / ckpt;
  for (int c = 1; c < b.nseg; ++c) b.ckpt.push_back(take_state(a, m, n, l, k, md.es));
  for (int i = 0; i <= b.len && T > 0; ++i) b.seg.push_back(take_state(a, m, n, l, k, md.es));
  b.gWt = a.take<double>((size_t)l * k);
  b.gA = a.take<double>((size_t)k * n);
  b.gT = a.take<double>((size_t)l * k);
  b.gV = a.take<double>((size_t)k * k);
  b.gS = a.take<double>((size_t)k * k);
  b.Msym = a.take<double>((size_t)k * k);
  b.Mpad = a.take<double>((size_t)KMAX * KMAX);
  b.S = a.take<double>((size_t)k * k);
  b.Tm = a.take<double>((size_t)l * k);
  b.V = a.take<double>((size_t)k * k);
  b.GU = a.take<double>((size_t)l * k);
  b.wsh = plan_wrev(m, l, k, md.dt, d.cus, d.max_lds);
  b.wx = a.take<u64>(wrev_ws_words(b.wsh));
  b.gsplits = ad_wgram_splits(m, d.cus);
  b.gpart = a.take<double>((size_t)b.gsplits * LMAX * LMAX);
  b.hsplits = hgram_splits(n);
  b.hpart = a.take<double>((size_t)b.hsplits * LMAX * LMAX);
  return b;
}

rnmf_status check_backward(int64_t m, int64_t n, int l, int k, int T, int ckpt, const rnmf_opts* o) {
  if (!o) return fail(RNMF_ERR_ARG, "opts is NULL");
  if (m < 1 || n < 1 || m > 0x7fffffffLL || n > 0x7fffffffLL) return fail(RNMF_ERR_SHAPE, "bad m or n");
  if (k < 1 || k > KMAX) return fail(RNMF_ERR_ARG, "need 1 <= k <= %d", KMAX);
  if (l < k || l > LMAX || l > m) return fail(RNMF_ERR_SHAPE, "need k <= l <= min(m, %d)", LMAX);
  if (T < 0) return fail(RNMF_ERR_ARG, "T < 0");
  if (ckpt < 0) return fail(RNMF_ERR_ARG, "ckpt_every must be >= 0");
  if (o->prec < 0 || o->prec > 2) return fail(RNMF_ERR_ARG, "unknown precision mode");
  if (o->gram_mode != RNMF_GRAM_FULL) return fail(RNMF_ERR_ARG, "the reverse pass needs gram_mode RNMF_GRAM_FULL");
  if (o->order != RNMF_ORDER_H_FIRST) return fail(RNMF_ERR_ARG, "the reverse pass needs order RNMF_ORDER_H_FIRST");
  if (o->alpha_w != 0.0 || o->alpha_h != 0.0 || o->beta_w != 0.0 || o->beta_h != 0.0)
    return fail(RNMF_ERR_ARG, "the reverse pass covers the plain rules (zero regularization weights)");
  return RNMF_OK;
}

hipError_t copy_state(const State& dst, const void* W, const void* Wt, const void* H, int64_t m, int64_t n, int l,
                      int k, size_t es, hipStream_t s) {
  hipError_t e;
  if ((e = hipMemcpyAsync(dst.W, W, (size_t)m * k * es, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(dst.Wt, Wt, (size_t)l * k * es, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
  return hipMemcpyAsync(dst.H, H, (size_t)k * n * es, hipMemcpyDeviceToDevice, s);
}

// The reverse of one sweep from (Wo, Wto, Ho) to (Wn, Wtn, Hn).  On entry gW,
// gWt, gH hold the adjoints of the sweep's outputs; on return those of its
// inputs, and gB has been accumulated.
rnmf_status reverse_sweep(const void* Q, const void* B, const State& o_, const State& n_, int64_t m, int64_t n,
                          int l, int k, double* gB, double* gW, double* gH, const BackBufs& b, unsigned* status,
                          int dt, hipStream_t s) {
  const int sd = dt;  // dtype code of the states, Q and B
  // T = B H'^T (l x k), V = H' H'^T (k x k)
  HIPCHK(ad_gemm_sd(l, k, n, B, sd, n, 0, n_.H, sd, n, 1, b.Tm, k, 1.0, 0, s));
  HIPCHK(launch_hgram(n_.H, k, n, b.hpart, dt, s));
  HIPCHK(launch_gram_sum(b.hpart, b.hsplits, k, b.V, s));
  // W columns in reverse (one persistent launch), then the T and V adjoints
  HIPCHK(ad_wrev(b.wsh, Q, n_.W, b.V, m, l, k, gW, b.gWt, b.GU, b.wx, status, dt, s));
  HIPCHK(ad_wpost_run(o_.Wt, n_.Wt, b.Tm, b.V, b.GU, l, k, b.gT, b.gV, dt, s));
  // T and V to H' and B: gB += gT H', gH += gT^T B + (gV + gV^T) H'
  HIPCHK(ad_gemm_sd(l, n, k, b.gT, 0, k, 0, n_.H, sd, n, 0, gB, n, 1.0, 1, s));
  HIPCHK(ad_gemm_sd(k, n, l, b.gT, 0, k, 1, B, sd, n, 0, gH, n, 1.0, 1, s));
  HIPCHK(ad_symm_run(b.gV, k, b.Msym, s));
  HIPCHK(ad_gemm_sd(k, n, k, b.Msym, 0, k, 0, n_.H, sd, n, 0, gH, n, 1.0, 1, s));
  // H rows in reverse with S = W^T W of the sweep's input
  HIPCHK(ad_wgram_run(o_.W, m, k, b.gpart, b.gsplits, b.S, dt, s));
  HIPCHK(ad_hrows_run(n_.H, b.S, n, k, gH, b.gA, dt, s));
  HIPCHK(ad_gs_run(n_.H, o_.H, b.gA, b.S, n, k, b.gS, dt, s));
  HIPCHK(ad_scale_rows_run(b.gA, b.S, n, k, s));
  // R = B^T W~: gB += W~ gA, gW~ += B gA^T; S: gW += W (gS + gS^T)
  HIPCHK(ad_gemm_sd(l, n, k, o_.Wt, sd, k, 0, b.gA, 0, n, 0, gB, n, 1.0, 1, s));
  HIPCHK(ad_gemm_sd(l, k, n, B, sd, n, 0, b.gA, 0, n, 1, b.gWt, k, 1.0, 1, s));
  HIPCHK(ad_symm_pad_run(b.gS, k, b.Mpad, s));
  HIPCHK(ad_rowmat_run(o_.W, b.Mpad, m, k, gW, dt, s));
  return RNMF_OK;
}

// Scratch of rnmf_hals_step_noalloc: one copy per GPU in the library's device
// code.  In host code `noalloc_scratch` names a host-side stand-in, never the
// device memory: the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char noalloc_scratch[RNMF_NOALLOC_SCRATCH_BYTES];

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[64] = {nullptr};

rnmf_status noalloc_scratch_ptr(void** out) {
  int id = 0;
  HIPCHK(hipGetDevice(&id));
  if (id < 0 || id >= 64) return fail(RNMF_ERR_HIP, "device id %d out of range", id);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[id]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)));
    if (!p || (uintptr_t)p % 256) return fail(RNMF_ERR_HIP, "scratch symbol address unusable");
    g_noalloc_ptr[id] = p;
  }
  *out = g_noalloc_ptr[id];
  return RNMF_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void rnmf_default_opts(rnmf_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->k = 0;
  o->p = 20;
  o->q = 2;
  o->max_iter = 200;
  o->tol = 0.0;
  o->seed = 0;
  o->prec = RNMF_PREC_F32;
  o->omega_dist = RNMF_OMEGA_GAUSSIAN;
  o->gram_mode = RNMF_GRAM_FULL;
  o->order = RNMF_ORDER_H_FIRST;
  o->flags = RNMF_FLAG_CHECK_INPUT;
}

const char* rnmf_status_string(int s) {
  switch (s) {
    case RNMF_OK: return "ok";
    case RNMF_ERR_ARG: return "invalid argument";
    case RNMF_ERR_SHAPE: return "invalid or unsupported shape";
    case RNMF_ERR_DTYPE: return "dtype not valid for the precision mode";
    case RNMF_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case RNMF_ERR_NONFINITE: return "non-finite value";
    case RNMF_ERR_NEGATIVE_INPUT: return "negative entry in X";
    case RNMF_ERR_NOT_SPD: return "Cholesky QR breakdown";
    case RNMF_ERR_HIP: return "HIP runtime error";
    case RNMF_ERR_DEVICE_TIMEOUT: return "device-wide wait timed out";
    case RNMF_NOT_CONVERGED: return "iteration cap reached before the tolerance";
    default: return "unknown status";
  }
}

const char* rnmf_last_error(void) { return g_err.c_str(); }

int32_t rnmf_sketch_width(int32_t k, int32_t p, int64_t m, int64_t n) {
  int64_t l = (int64_t)k + p;
  if (l > m) l = m;
  if (l > n) l = n;
  return (int32_t)l;
}

size_t rnmf_workspace_bytes(int op, int64_t m, int64_t n, const rnmf_opts* o) {
  g_err.clear();
  if (op == RNMF_OP_HALS_STEP) {
    if (!o) { fail(RNMF_ERR_ARG, "opts is NULL"); return 0; }
    if (m < 1 || n < 1 || o->k < 1 || o->k > KMAX) { fail(RNMF_ERR_ARG, "bad shape or k for the sweep"); return 0; }
  } else if (op == RNMF_OP_REL_ERROR) {
    if (m < 1 || n < 1) { fail(RNMF_ERR_SHAPE, "empty matrix"); return 0; }
  } else if (op == RNMF_OP_HALS) {
    if (!o) { fail(RNMF_ERR_ARG, "opts is NULL"); return 0; }
    if (m < 1 || n < 1 || o->k < 1 || o->k > KMAX || o->k > m || o->k > n) {
      fail(RNMF_ERR_ARG, "need 1 <= k <= min(%d, m, n)", KMAX);
      return 0;
    }
    if (o->prec != RNMF_PREC_F32 && o->prec != RNMF_PREC_F64) {
      fail(RNMF_ERR_ARG, "deterministic HALS runs in RNMF_PREC_F32 or RNMF_PREC_F64");
      return 0;
    }
  } else if (op == RNMF_OP_SVD_INIT) {
    if (!o) { fail(RNMF_ERR_ARG, "opts is NULL"); return 0; }
    const int l = lwidth(o, m, n);
    if (m < 1 || n < 1 || o->k < 1 || o->k > KMAX || o->k > l || l > LSVD) {
      fail(RNMF_ERR_ARG, "the SVD-based initialization needs 1 <= k <= min(l, %d) and l <= %d", KMAX, LSVD);
      return 0;
    }
  } else {
    if (check_opts(o, m, n, op == RNMF_OP_FACTORIZE) != RNMF_OK) return 0;
  }
  if (op < RNMF_OP_SKETCH || op > RNMF_OP_SVD_INIT) { fail(RNMF_ERR_ARG, "unknown op %d", op); return 0; }
  Dev d = default_dev();
  Dev q;
  if (get_dev(q, nullptr)) d = q;
  rnmf_opts tmp;
  if (!o) { rnmf_default_opts(&tmp); tmp.k = 1; o = &tmp; }
  // the F32 cast slot is sized whenever the BF16 mode might receive FP32 X
  return op_bytes(op, m, n, o, RNMF_F32, d);
}

rnmf_status rnmf_sketch(const void* X, int xt, int64_t m, int64_t n, int64_t ldx, const void* Omega,
                        const rnmf_opts* o, void* Q, int32_t* l_out, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  rnmf_status r;
  if ((r = check_opts(o, m, n, false)) != RNMF_OK) return r;
  if ((r = check_xt(o, xt)) != RNMF_OK) return r;
  if (!X || !Q) return fail(RNMF_ERR_ARG, "X and Q must be non-NULL");
  if (ldx < n) return fail(RNMF_ERR_SHAPE, "ldx < n");
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  const Mode md = mode_of(o);
  if ((r = check_ws(ws, ws_bytes, op_bytes(RNMF_OP_SKETCH, m, n, o, xt, d))) != RNMF_OK) return r;
  Hdr h = header(ws);
  Arena a(ws);
  a.take<char>(HDR_BYTES);
  void* xb = (md.cdt == 2 && xt == RNMF_F32) ? (void*)a.take<bf16_t>((size_t)m * bf16_ld(n)) : nullptr;
  SketchBufs b = plan_sketch(a, m, n, lwidth(o, m, n), md, d);
  HIPCHK(launch_fill_u32(h.status, 1, 0u, d.stream));
  const void* Xc;
  int64_t ldc;
  int check;
  if ((r = prepare_x(X, xt, m, n, ldx, o, md, xb, h, d, &Xc, &ldc, &check)) != RNMF_OK) return r;
  if ((r = run_sketch(Xc, m, n, ldc, Omega, o, Q, b, md, h, check, d)) != RNMF_OK) return r;
  if (l_out) *l_out = lwidth(o, m, n);
  return RNMF_OK;
}

rnmf_status rnmf_compress(const void* X, int xt, int64_t m, int64_t n, int64_t ldx, const void* Q, int32_t l,
                          const rnmf_opts* o, void* B, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  rnmf_status r;
  if (!o) return fail(RNMF_ERR_ARG, "opts is NULL");
  // only the precision of opts matters here (B = Q^T X for any m x n X,
  // including n < l); the plan is sized with l itself
  if (l < 1 || l > LMAX || l > m) return fail(RNMF_ERR_SHAPE, "need 1 <= l <= min(m, %d)", LMAX);
  if (m < 1 || n < 1 || m > 0x7fffffffLL || n > 0x7fffffffLL) return fail(RNMF_ERR_SHAPE, "bad m or n");
  if (o->prec < 0 || o->prec > 2) return fail(RNMF_ERR_ARG, "unknown precision mode %d", o->prec);
  if ((r = check_xt(o, xt)) != RNMF_OK) return r;
  if (!X || !Q || !B) return fail(RNMF_ERR_ARG, "X, Q and B must be non-NULL");
  if (ldx < n) return fail(RNMF_ERR_SHAPE, "ldx < n");
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  const Mode md = mode_of(o);
  Arena a(ws);
  a.take<char>(HDR_BYTES);
  void* xb = (md.cdt == 2 && xt == RNMF_F32) ? (void*)a.take<bf16_t>((size_t)m * bf16_ld(n)) : nullptr;
  CompressBufs b = plan_compress(a, m, n, l, md, d);
  if ((r = check_ws(ws, ws_bytes, a.used)) != RNMF_OK) return r;
  Hdr h = header(ws);
  HIPCHK(launch_fill_u32(h.status, 1, 0u, d.stream));
  const void* Xc;
  int64_t ldc;
  int check;
  if ((r = prepare_x(X, xt, m, n, ldx, o, md, xb, h, d, &Xc, &ldc, &check)) != RNMF_OK) return r;
  (void)check;  // the input scan belongs to the first pass over X (sketch)
  return run_compress(Xc, m, n, ldc, Q, l, B, b, md, d);
}

rnmf_status rnmf_sweep_plan(int64_t m, int64_t n, int32_t l, int32_t k, const rnmf_opts* o, int32_t* out) {
  g_err.clear();
  if (!o || !out) return fail(RNMF_ERR_ARG, "opts and out must be non-NULL");
  if (m < 1 || n < 1 || m > 0x7fffffffLL || n > 0x7fffffffLL) return fail(RNMF_ERR_SHAPE, "bad m or n");
  if (k < 1 || k > KMAX) return fail(RNMF_ERR_ARG, "need 1 <= k <= %d", KMAX);
  if (l < k || l > LMAX || l > m) return fail(RNMF_ERR_SHAPE, "need k <= l <= min(m, %d)", LMAX);
  if (o->prec < 0 || o->prec > 2) return fail(RNMF_ERR_ARG, "unknown precision mode");
  Dev d;
  if (!get_dev(d, nullptr)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  const SweepShape sh = plan_sweep(m, n, l, k, mode_of(o).dt, d, o->tol > 0.0);
  out[0] = sh.G;
  out[1] = sh.rows_per;
  out[2] = sh.cols_per;
  out[3] = sh.regq;
  out[4] = sh.wglobal;
  out[5] = sh.xown;
  out[6] = (int32_t)sh.lds_bytes;
  out[7] = sh.regq ? 0 : sh.rows_lds;
  return RNMF_OK;
}

rnmf_status rnmf_hals_step(const void* Q, const void* B, int64_t m, int64_t n, int32_t l, int32_t k, void* W,
                           void* Wt, void* H, int32_t nsweeps, const rnmf_opts* o, double* dev_stats, void* ws,
                           size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!o) return fail(RNMF_ERR_ARG, "opts is NULL");
  if (!Q || !B || !W || !Wt || !H) return fail(RNMF_ERR_ARG, "Q, B, W, Wt and H must be non-NULL");
  if (m < 1 || n < 1 || m > 0x7fffffffLL || n > 0x7fffffffLL) return fail(RNMF_ERR_SHAPE, "bad m or n");
  if (k < 1 || k > KMAX) return fail(RNMF_ERR_ARG, "need 1 <= k <= %d", KMAX);
  if (l < k || l > LMAX || l > m) return fail(RNMF_ERR_SHAPE, "need k <= l <= min(m, %d)", LMAX);
  if (nsweeps < 0) return fail(RNMF_ERR_ARG, "nsweeps < 0");
  if (o->prec < 0 || o->prec > 2) return fail(RNMF_ERR_ARG, "unknown precision mode");
  if (o->gram_mode < 0 || o->gram_mode > 2) return fail(RNMF_ERR_ARG, "unknown gram_mode");
  if (o->order < 0 || o->order > 1) return fail(RNMF_ERR_ARG, "unknown order");
  if (check_reg(o) != RNMF_OK) return RNMF_ERR_ARG;
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  const Mode md = mode_of(o);
  rnmf_opts o2 = *o;
  o2.k = k;
  rnmf_status r;
  Arena a(ws);
  a.take<char>(HDR_BYTES);
  SweepBufs b = plan_hals(a, m, n, l, k, md, d, o->tol > 0.0);
  if ((r = check_ws(ws, ws_bytes, a.used)) != RNMF_OK) return r;
  Hdr h = header(ws);
  HIPCHK(launch_fill_u32(h.status, 1, 0u, d.stream));
  double* stats = dev_stats ? dev_stats : h.stats;
  u64* trace = nullptr;
  if (o->flags & RNMF_FLAG_TRACE) {
    trace = (u64*)((char*)ws + TRACE_OFFSET);
    HIPCHK(launch_fill_u32((unsigned*)trace, (HDR_BYTES - TRACE_OFFSET) / 4, 0u, d.stream));
  }
  HIPCHK(launch_sweep(b.sh, md.dt, Q, B, W, Wt, H, m, n, l, k, nsweeps, o->tol, o->gram_mode, o->order, reg_of(o), b.xbuf,
                      stats, h.status, trace, d.stream));
  return RNMF_OK;
}

rnmf_status rnmf_hals_step_noalloc(const void* Q, const void* B, int64_t m, int64_t n, int32_t l, int32_t k, void* W,
                                   void* Wt, void* H, int32_t nsweeps, const rnmf_opts* o, double* dev_stats,
                                   uint32_t* dev_status, void* stream) {
  g_err.clear();
  if (!o) return fail(RNMF_ERR_ARG, "opts is NULL");
  if (!Q || !B || !W || !Wt || !H) return fail(RNMF_ERR_ARG, "Q, B, W, Wt and H must be non-NULL");
  if (m < 1 || n < 1 || m > 0x7fffffffLL || n > 0x7fffffffLL) return fail(RNMF_ERR_SHAPE, "bad m or n");
  if (k < 1 || k > KMAX) return fail(RNMF_ERR_ARG, "need 1 <= k <= %d", KMAX);
  if (l < k || l > LMAX || l > m) return fail(RNMF_ERR_SHAPE, "need k <= l <= min(m, %d)", LMAX);
  if (nsweeps < 0) return fail(RNMF_ERR_ARG, "nsweeps < 0");
  if (o->prec < 0 || o->prec > 2) return fail(RNMF_ERR_ARG, "unknown precision mode");
  if (o->gram_mode < 0 || o->gram_mode > 2) return fail(RNMF_ERR_ARG, "unknown gram_mode");
  if (o->order < 0 || o->order > 1) return fail(RNMF_ERR_ARG, "unknown order");
  if (o->flags & RNMF_FLAG_TRACE) return fail(RNMF_ERR_ARG, "RNMF_FLAG_TRACE needs a workspace (rnmf_hals_step)");
  if (check_reg(o) != RNMF_OK) return RNMF_ERR_ARG;
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  const Mode md = mode_of(o);
  // size first (null base), then carve the scratch the same way
  Arena sz(nullptr);
  sz.take<char>(HDR_BYTES);
  plan_hals(sz, m, n, l, k, md, d, o->tol > 0.0);
  if (sz.used > (size_t)RNMF_NOALLOC_SCRATCH_BYTES)
    return fail(RNMF_ERR_WORKSPACE, "this problem needs %zu bytes of scratch; rnmf_hals_step_noalloc holds %zu "
                "(use rnmf_hals_step with a workspace)", sz.used, (size_t)RNMF_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  rnmf_status r;
  if ((r = noalloc_scratch_ptr(&ws)) != RNMF_OK) return r;
  Arena a(ws);
  a.take<char>(HDR_BYTES);
  SweepBufs b = plan_hals(a, m, n, l, k, md, d, o->tol > 0.0);
  Hdr h = header(ws);
  unsigned* status = dev_status ? (unsigned*)dev_status : h.status;
  HIPCHK(launch_fill_u32(status, 1, 0u, d.stream));
  double* stats = dev_stats ? dev_stats : h.stats;
  HIPCHK(launch_sweep(b.sh, md.dt, Q, B, W, Wt, H, m, n, l, k, nsweeps, o->tol, o->gram_mode, o->order, reg_of(o),
                      b.xbuf, stats, status, nullptr, d.stream));
  return RNMF_OK;
}

rnmf_status rnmf_unroll(const void* Q, const void* B, int64_t m, int64_t n, int32_t l, int32_t k, void* W, void* Wt,
                        void* H, int32_t T, void* states, const rnmf_opts* o, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!o) return fail(RNMF_ERR_ARG, "opts is NULL");
  if (!Q || !B || !W || !Wt || !H) return fail(RNMF_ERR_ARG, "Q, B, W, Wt and H must be non-NULL");
  if (m < 1 || n < 1 || m > 0x7fffffffLL || n > 0x7fffffffLL) return fail(RNMF_ERR_SHAPE, "bad m or n");
  if (k < 1 || k > KMAX) return fail(RNMF_ERR_ARG, "need 1 <= k <= %d", KMAX);
  if (l < k || l > LMAX || l > m) return fail(RNMF_ERR_SHAPE, "need k <= l <= min(m, %d)", LMAX);
  if (T < 0) return fail(RNMF_ERR_ARG, "T < 0");
  if (o->prec < 0 || o->prec > 2) return fail(RNMF_ERR_ARG, "unknown precision mode");
  if (o->gram_mode < 0 || o->gram_mode > 2) return fail(RNMF_ERR_ARG, "unknown gram_mode");
  if (o->order < 0 || o->order > 1) return fail(RNMF_ERR_ARG, "unknown order");
  if (check_reg(o) != RNMF_OK) return RNMF_ERR_ARG;
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  const Mode md = mode_of(o);
  rnmf_status r;
  Arena a(ws);
  a.take<char>(HDR_BYTES);
  SweepBufs b = plan_hals(a, m, n, l, k, md, d, false);
  if ((r = check_ws(ws, ws_bytes, a.used)) != RNMF_OK) return r;
  Hdr h = header(ws);
  HIPCHK(launch_fill_u32(h.status, 1, 0u, d.stream));
  const size_t wsz = (size_t)m * k * md.es, wtsz = (size_t)l * k * md.es, hsz = (size_t)k * n * md.es;
  for (int i = 0; i < T; ++i) {
    HIPCHK(launch_sweep(b.sh, md.dt, Q, B, W, Wt, H, m, n, l, k, 1, 0.0, o->gram_mode, o->order, reg_of(o), b.xbuf,
                        h.stats, h.status, nullptr, d.stream));
    if (states) {
      char* p = (char*)states + (size_t)i * (wsz + wtsz + hsz);
      HIPCHK(hipMemcpyAsync(p, W, wsz, hipMemcpyDeviceToDevice, d.stream));
      HIPCHK(hipMemcpyAsync(p + wsz, Wt, wtsz, hipMemcpyDeviceToDevice, d.stream));
      HIPCHK(hipMemcpyAsync(p + wsz + wtsz, H, hsz, hipMemcpyDeviceToDevice, d.stream));
    }
  }
  return RNMF_OK;
}

size_t rnmf_hals_ordered_workspace_bytes(int64_t m, int64_t n, int32_t l, int32_t k) {
  g_err.clear();
  if (m < 1 || n < 1 || k < 1 || k > KMAX || l < k || l > LMAX || l > m) {
    fail(RNMF_ERR_ARG, "need 1 <= k <= l <= min(m, %d), k <= %d", LMAX, KMAX);
    return 0;
  }
  Arena a(nullptr);
  a.take<char>(HDR_BYTES);
  a.take<double>((size_t)ord_part_elems(m, n, l, k));
  a.take<double>((size_t)l + k);
  return a.used;
}

rnmf_status rnmf_hals_ordered(const void* Q, const void* B, int64_t m, int64_t n, int32_t l, int32_t k, void* W,
                              void* Wt, void* H, int32_t nsweeps, const int32_t* order, const rnmf_opts* o, void* ws,
                              size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!o) return fail(RNMF_ERR_ARG, "opts is NULL");
  if (!Q || !B || !W || !Wt || !H) return fail(RNMF_ERR_ARG, "Q, B, W, Wt and H must be non-NULL");
  if (m < 1 || n < 1 || m > 0x7fffffffLL || n > 0x7fffffffLL) return fail(RNMF_ERR_SHAPE, "bad m or n");
  if (k < 1 || k > KMAX) return fail(RNMF_ERR_ARG, "need 1 <= k <= %d", KMAX);
  if (l < k || l > LMAX || l > m) return fail(RNMF_ERR_SHAPE, "need k <= l <= min(m, %d)", LMAX);
  if (nsweeps < 0) return fail(RNMF_ERR_ARG, "nsweeps < 0");
  if (nsweeps > 0 && !order) return fail(RNMF_ERR_ARG, "order is NULL");
  if (o->prec < 0 || o->prec > 2) return fail(RNMF_ERR_ARG, "unknown precision mode");
  if (o->gram_mode != RNMF_GRAM_FULL) return fail(RNMF_ERR_ARG, "ordered sweeps use gram_mode RNMF_GRAM_FULL");
  if (o->alpha_w != 0.0 || o->alpha_h != 0.0 || o->beta_w != 0.0 || o->beta_h != 0.0)
    return fail(RNMF_ERR_ARG, "ordered sweeps use the plain rules (zero regularization weights)");
  // every sweep's list must update each of the 2k blocks exactly once
  std::vector<char> seen((size_t)2 * k);
  for (int s = 0; s < nsweeps; ++s) {
    std::fill(seen.begin(), seen.end(), 0);
    for (int i = 0; i < 2 * k; ++i) {
      const int32_t e = order[(size_t)s * 2 * k + i];
      if (e < 0 || e >= 2 * k || seen[e]) return fail(RNMF_ERR_ARG, "sweep %d: order is not a permutation of 0..2k-1", s);
      seen[e] = 1;
    }
  }
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  const Mode md = mode_of(o);
  Arena a(ws);
  a.take<char>(HDR_BYTES);
  double* part = a.take<double>((size_t)ord_part_elems(m, n, l, k));
  double* vec = a.take<double>((size_t)l + k);
  rnmf_status r;
  if ((r = check_ws(ws, ws_bytes, a.used)) != RNMF_OK) return r;
  Hdr h = header(ws);
  HIPCHK(launch_fill_u32(h.status, 1, 0u, d.stream));
  for (int s = 0; s < nsweeps; ++s)
    for (int i = 0; i < 2 * k; ++i)
      HIPCHK(launch_ordered_update(Q, B, W, Wt, H, m, n, l, k, order[(size_t)s * 2 * k + i], part, vec, md.dt,
                                   d.stream));
  return RNMF_OK;
}

rnmf_status rnmf_svd_init(const void* Q, const void* B, int64_t m, int64_t n, int32_t l, int32_t k, void* W,
                          void* H, const rnmf_opts* o, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!o) return fail(RNMF_ERR_ARG, "opts is NULL");
  if (!Q || !B || !W || !H) return fail(RNMF_ERR_ARG, "Q, B, W and H must be non-NULL");
  if (m < 1 || n < 1 || m > 0x7fffffffLL || n > 0x7fffffffLL) return fail(RNMF_ERR_SHAPE, "bad m or n");
  if (l < 1 || l > LSVD || l > m) return fail(RNMF_ERR_SHAPE, "need 1 <= l <= min(m, %d)", LSVD);
  if (k < 1 || k > l || k > KMAX) return fail(RNMF_ERR_ARG, "need 1 <= k <= min(l, %d)", KMAX);
  if (o->prec < 0 || o->prec > 2) return fail(RNMF_ERR_ARG, "unknown precision mode");
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  const Mode md = mode_of(o);
  Arena a(ws);
  a.take<char>(HDR_BYTES);
  SvdBufs b = plan_svd(a, m, n, l, k);
  rnmf_status r;
  if ((r = check_ws(ws, ws_bytes, a.used)) != RNMF_OK) return r;
  HIPCHK(launch_svd_init(Q, B, m, n, l, k, W, H, md.dt, b, d.stream));
  return RNMF_OK;
}

size_t rnmf_backward_workspace_bytes(int64_t m, int64_t n, int32_t l, int32_t k, int32_t T, int32_t ckpt_every,
                                     const rnmf_opts* o) {
  g_err.clear();
  if (check_backward(m, n, l, k, T, ckpt_every, o) != RNMF_OK) return 0;
  Dev d = default_dev();
  Dev q;
  if (get_dev(q, nullptr)) d = q;
  Arena a(nullptr);
  a.take<char>(HDR_BYTES);
  plan_backward(a, m, n, l, k, T, ckpt_every, mode_of(o), d);
  return a.used;
}

rnmf_status rnmf_backward(const void* Q, const void* B, int64_t m, int64_t n, int32_t l, int32_t k, const void* W0,
                          const void* Wt0, const void* H0, int32_t T, int32_t ckpt_every, const void* states,
                          const double* gW_T, const double* gH_T, double* gB, double* gW0, double* gH0, double* gX,
                          const rnmf_opts* o, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  rnmf_status r;
  if ((r = check_backward(m, n, l, k, T, ckpt_every, o)) != RNMF_OK) return r;
  if (!Q || !B || !W0 || !Wt0 || !H0 || !gW_T || !gH_T || !gB || !gW0 || !gH0)
    return fail(RNMF_ERR_ARG, "only gX (and states, with ckpt_every >= 1) may be NULL");
  if ((ckpt_every == 0) != (states != nullptr))
    return fail(RNMF_ERR_ARG, "recorded states go with ckpt_every = 0, and ckpt_every = 0 needs them");
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  const Mode md = mode_of(o);
  hipStream_t s = d.stream;
  Arena a(ws);
  a.take<char>(HDR_BYTES);
  BackBufs b = plan_backward(a, m, n, l, k, T, ckpt_every, md, d);
  if ((r = check_ws(ws, ws_bytes, a.used)) != RNMF_OK) return r;
  Hdr h = header(ws);
  HIPCHK(launch_fill_u32(h.status, 1, 0u, s));
  const Reg none{0.0, 0.0, 0.0, 0.0};
  auto sweep = [&](const State& st) {
    return launch_sweep(b.sw.sh, md.dt, Q, B, st.W, st.Wt, st.H, m, n, l, k, 1, 0.0, RNMF_GRAM_FULL,
                        RNMF_ORDER_H_FIRST, none, b.sw.xbuf, h.stats, h.status, nullptr, s);
  };
  // adjoint accumulators: gW0 and gH0 carry gW and gH through the sweeps
  if (gW0 != gW_T) HIPCHK(hipMemcpyAsync(gW0, gW_T, (size_t)m * k * 8, hipMemcpyDeviceToDevice, s));
  if (gH0 != gH_T) HIPCHK(hipMemcpyAsync(gH0, gH_T, (size_t)k * n * 8, hipMemcpyDeviceToDevice, s));
  HIPCHK(ad_fill_run(b.gWt, (int64_t)l * k, 0.0, s));
  HIPCHK(ad_fill_run(gB, (int64_t)l * n, 0.0, s));
  // forward: the state at the start of every segment after the first, each
  // from the one before by one-sweep launches
  for (int c = 1; c < b.nseg; ++c) {
    const State& dst = b.ckpt[c - 1];
    if (c == 1) HIPCHK(copy_state(dst, W0, Wt0, H0, m, n, l, k, md.es, s));
    else HIPCHK(copy_state(dst, b.ckpt[c - 2].W, b.ckpt[c - 2].Wt, b.ckpt[c - 2].H, m, n, l, k, md.es, s));
    for (int i = 0; i < ckpt_every; ++i) HIPCHK(sweep(dst));
  }
  // recorded states: sweep i maps state i - 1 (the inputs for i = 0) to state i
  if (states) {
    const size_t wsz = (size_t)m * k * md.es, wtsz = (size_t)l * k * md.es, hsz = (size_t)k * n * md.es;
    char* base = (char*)states;
    auto rec = [&](int i) {
      char* p = base + (size_t)i * (wsz + wtsz + hsz);
      return State{p, p + wsz, p + wsz + wtsz};
    };
    const State in{(void*)W0, (void*)Wt0, (void*)H0};
    for (int i = T - 1; i >= 0; --i)
      if ((r = reverse_sweep(Q, B, i == 0 ? in : rec(i - 1), rec(i), m, n, l, k, gB, gW0, gH0, b, h.status, md.dt,
                             s)) != RNMF_OK)
        return r;
  }
  // reverse, segment by segment: recompute the segment's states, then undo
  // its sweeps last to first
  for (int c = b.nseg - 1; c >= 0; --c) {
    const int t0 = c * ckpt_every;
    const int len = (T - t0) < ckpt_every ? (T - t0) : ckpt_every;
    if (c == 0) HIPCHK(copy_state(b.seg[0], W0, Wt0, H0, m, n, l, k, md.es, s));
    else HIPCHK(copy_state(b.seg[0], b.ckpt[c - 1].W, b.ckpt[c - 1].Wt, b.ckpt[c - 1].H, m, n, l, k, md.es, s));
    for (int i = 1; i <= len; ++i) {
      HIPCHK(copy_state(b.seg[i], b.seg[i - 1].W, b.seg[i - 1].Wt, b.seg[i - 1].H, m, n, l, k, md.es, s));
      HIPCHK(sweep(b.seg[i]));
    }
    for (int i = len - 1; i >= 0; --i)
      if ((r = reverse_sweep(Q, B, b.seg[i], b.seg[i + 1], m, n, l, k, gB, gW0, gH0, b, h.status, md.dt, s)) !=
          RNMF_OK)
        return r;
  }
  // W~0 = Q^T W0: gW0 += Q gW~0; X enters through B = Q^T X: gX = Q gB
  HIPCHK(ad_gemm_sd(m, k, l, Q, md.dt, l, 0, b.gWt, 0, k, 0, gW0, k, 1.0, 1, s));
  if (gX) HIPCHK(ad_gemm_sd(m, n, l, Q, md.dt, l, 0, gB, 0, n, 0, gX, n, 1.0, 0, s));
  return RNMF_OK;
}


size_t rnmf_batch_workspace_bytes(int32_t nprob) {
  g_err.clear();
  if (nprob < 1) { fail(RNMF_ERR_ARG, "nprob must be >= 1"); return 0; }
  return batch_layout(nullptr, nprob).bytes;
}

rnmf_status rnmf_batch_plan(const rnmf_problem* probs, int32_t nprob, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!probs || nprob < 1) return fail(RNMF_ERR_ARG, "need a host array of nprob >= 1 problems");
  for (int i = 0; i < nprob; ++i) {
    rnmf_status r = check_problem(probs[i], i);
    if (r != RNMF_OK) return r;
  }
  const BatchLayout L = batch_layout(ws, nprob);
  rnmf_status r;
  if ((r = check_ws(ws, ws_bytes, L.bytes)) != RNMF_OK) return r;
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  int table[8];
  {
    std::lock_guard<std::mutex> g(g_batch_mu);
    std::memcpy(table, g_batch_tc, sizeof(table));
  }
  if ((r = upload_plan(probs, nprob, L, table, nullptr, d.stream)) != RNMF_OK) return r;
  return RNMF_OK;
}

rnmf_status rnmf_batch_run(int32_t nprob, int32_t q, int32_t nsweeps, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (nprob < 1) return fail(RNMF_ERR_ARG, "nprob must be >= 1");
  if (q < 0 || q > 32) return fail(RNMF_ERR_ARG, "q must be in [0, 32]");
  if (nsweeps < 0) return fail(RNMF_ERR_ARG, "nsweeps < 0");
  const BatchLayout L = batch_layout(ws, nprob);
  rnmf_status r;
  if ((r = check_ws(ws, ws_bytes, L.bytes)) != RNMF_OK) return r;
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  // two workgroups per compute unit (the kernel's LDS and registers allow it)
  const int grid = nprob < 2 * d.cus ? nprob : 2 * d.cus;
  HIPCHK(launch_batch(L.descs, nprob, q, nsweeps, L.counter, L.err, L.status, grid, d.stream));
  return RNMF_OK;
}

rnmf_status rnmf_batch_results(int32_t nprob, void* ws, size_t ws_bytes, double* rel_err, int32_t* status,
                               void* stream) {
  g_err.clear();
  if (nprob < 1) return fail(RNMF_ERR_ARG, "nprob must be >= 1");
  const BatchLayout L = batch_layout(ws, nprob);
  rnmf_status r;
  if ((r = check_ws(ws, ws_bytes, L.bytes)) != RNMF_OK) return r;
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  std::vector<double> e(2 * (size_t)nprob);
  std::vector<unsigned> st((size_t)nprob);
  HIPCHK(hipMemcpyAsync(e.data(), L.err, e.size() * sizeof(double), hipMemcpyDeviceToHost, d.stream));
  HIPCHK(hipMemcpyAsync(st.data(), L.status, st.size() * sizeof(unsigned), hipMemcpyDeviceToHost, d.stream));
  HIPCHK(hipStreamSynchronize(d.stream));
  for (int i = 0; i < nprob; ++i) {
    if (rel_err) rel_err[i] = (e[2 * i + 1] > 0.0 && !(st[i] & ST_NOT_SPD)) ? std::sqrt(e[2 * i] / e[2 * i + 1]) : NAN;
    if (status) status[i] = (st[i] & ST_NOT_SPD) ? RNMF_ERR_NOT_SPD : RNMF_OK;
  }
  return RNMF_OK;
}

rnmf_status rnmf_batch_set_tuning(const int32_t* table) {
  g_err.clear();
  if (!table) return fail(RNMF_ERR_ARG, "table is NULL");
  for (int c = 0; c < 4; ++c) {
    if (table[c] != 4 && table[c] != 8 && table[c] != 16)
      return fail(RNMF_ERR_ARG, "entry %d: column groups must be 4, 8 or 16", c);
    if (table[4 + c] != 64 && table[4 + c] != 128 && table[4 + c] != 256)
      return fail(RNMF_ERR_ARG, "entry %d: H-phase tile width must be 64, 128 or 256", 4 + c);
  }
  std::lock_guard<std::mutex> g(g_batch_mu);
  std::memcpy(g_batch_tc, table, sizeof(g_batch_tc));
  return RNMF_OK;
}

rnmf_status rnmf_batch_get_tuning(int32_t* table) {
  g_err.clear();
  if (!table) return fail(RNMF_ERR_ARG, "table is NULL");
  std::lock_guard<std::mutex> g(g_batch_mu);
  std::memcpy(table, g_batch_tc, sizeof(g_batch_tc));
  return RNMF_OK;
}

rnmf_status rnmf_batch_autotune(const rnmf_problem* probs, int32_t nprob, int32_t q, void* ws, size_t ws_bytes,
                                int32_t* tiling_out, void* stream) {
  g_err.clear();
  if (!probs || nprob < 1) return fail(RNMF_ERR_ARG, "need a host array of nprob >= 1 problems");
  if (q < 0 || q > 32) return fail(RNMF_ERR_ARG, "q must be in [0, 32]");
  for (int i = 0; i < nprob; ++i) {
    rnmf_status r = check_problem(probs[i], i);
    if (r != RNMF_OK) return r;
  }
  const BatchLayout L = batch_layout(ws, nprob);
  rnmf_status r;
  if ((r = check_ws(ws, ws_bytes, L.bytes)) != RNMF_OK) return r;
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  int table[8];
  {
    std::lock_guard<std::mutex> g(g_batch_mu);
    std::memcpy(table, g_batch_tc, sizeof(table));
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  struct EvGuard {
    hipEvent_t* a;
    hipEvent_t* b;
    ~EvGuard() {
      if (*a) (void)hipEventDestroy(*a);
      if (*b) (void)hipEventDestroy(*b);
    }
  } guard{&e0, &e1};
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // one timed launch (after a warm-up) of a sub-batch with a forced table
  auto time_run = [&](const std::vector<rnmf_problem>& sub, const int* forced, int nsw, float* ms) -> rnmf_status {
    const int ns = (int)sub.size();
    const BatchLayout S = batch_layout(ws, ns);
    rnmf_status rr;
    if ((rr = upload_plan(sub.data(), ns, S, forced, nullptr, d.stream)) != RNMF_OK) return rr;
    const int grid = ns < 2 * d.cus ? ns : 2 * d.cus;
    HIPCHK(launch_batch(S.descs, ns, q, nsw, S.counter, S.err, S.status, grid, d.stream));  // warm-up
    HIPCHK(hipEventRecord(e0, d.stream));
    HIPCHK(launch_batch(S.descs, ns, q, nsw, S.counter, S.err, S.status, grid, d.stream));
    HIPCHK(hipEventRecord(e1, d.stream));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(ms, e0, e1));
    return RNMF_OK;
  };
  // each sketch-width class separately, on its own problems: first every
  // X-pass tiling that covers the class's widest sketch (range finder and
  // compression only), then every H-phase tile width that fits it (with
  // TUNE_SWEEPS sweeps, the X-pass tiling just chosen)
  constexpr int TUNE_SWEEPS = 8;
  for (int cls = 0; cls < 4; ++cls) {
    std::vector<rnmf_problem> sub;
    int lmax = 0;
    for (int i = 0; i < nprob; ++i)
      if (l_class(probs[i].l) == cls) {
        sub.push_back(probs[i]);
        lmax = probs[i].l > lmax ? probs[i].l : lmax;
      }
    if (sub.empty()) continue;
    float best_ms = 0.f;
    int best = table[cls];
    for (int tc : {4, 8, 16}) {
      if (4 * tc < lmax) continue;
      int forced[8];
      for (int c = 0; c < 4; ++c) { forced[c] = tc; forced[4 + c] = table[4 + c]; }
      float ms = 0.f;
      if ((r = time_run(sub, forced, 0, &ms)) != RNMF_OK) return r;
      if (best_ms == 0.f || ms < best_ms) {
        best_ms = ms;
        best = tc;
      }
    }
    table[cls] = best;
    best_ms = 0.f;
    int best_h = table[4 + cls];
    for (int hct : {64, 128, 256}) {
      if (!batch_hct_ok(hct, lmax)) continue;
      int forced[8];
      for (int c = 0; c < 4; ++c) { forced[c] = table[c]; forced[4 + c] = hct; }
      float ms = 0.f;
      if ((r = time_run(sub, forced, TUNE_SWEEPS, &ms)) != RNMF_OK) return r;
      if (best_ms == 0.f || ms < best_ms) {
        best_ms = ms;
        best_h = hct;
      }
    }
    table[4 + cls] = best_h;
  }
  {
    std::lock_guard<std::mutex> g(g_batch_mu);
    std::memcpy(g_batch_tc, table, sizeof(table));
  }
  if (tiling_out) std::memcpy(tiling_out, table, sizeof(table));
  return upload_plan(probs, nprob, L, table, nullptr, d.stream);
}

rnmf_status rnmf_hals(const void* X, int xt, int64_t m, int64_t n, int64_t ldx, void* W, void* H, int32_t nsweeps,
                      const rnmf_opts* o, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!o) return fail(RNMF_ERR_ARG, "opts is NULL");
  if (!X || !W || !H) return fail(RNMF_ERR_ARG, "X, W and H must be non-NULL");
  if (m < 1 || n < 1 || m > 0x7fffffffLL || n > 0x7fffffffLL) return fail(RNMF_ERR_SHAPE, "bad m or n");
  if (ldx < n) return fail(RNMF_ERR_SHAPE, "ldx < n");
  const int k = o->k;
  if (k < 1 || k > KMAX || k > m || k > n) return fail(RNMF_ERR_ARG, "need 1 <= k <= min(%d, m, n)", KMAX);
  if (nsweeps < 0) return fail(RNMF_ERR_ARG, "nsweeps < 0");
  if (o->prec != RNMF_PREC_F32 && o->prec != RNMF_PREC_F64)
    return fail(RNMF_ERR_ARG, "deterministic HALS runs in RNMF_PREC_F32 or RNMF_PREC_F64");
  if (o->order < 0 || o->order > 1) return fail(RNMF_ERR_ARG, "unknown order");
  if (o->tol > 0.0) return fail(RNMF_ERR_ARG, "deterministic HALS runs a fixed number of sweeps (tol must be <= 0)");
  if (check_reg(o) != RNMF_OK) return RNMF_ERR_ARG;
  rnmf_status r;
  if ((r = check_xt(o, xt)) != RNMF_OK) return r;
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  const Mode md = mode_of(o);
  Arena a(ws);
  a.take<char>(HDR_BYTES);
  DHalsBufs b = plan_dhals(a, m, n, k, md, d);
  if ((r = check_ws(ws, ws_bytes, a.used)) != RNMF_OK) return r;
  Hdr h = header(ws);
  hipStream_t s = d.stream;
  HIPCHK(launch_fill_u32(h.status, 1, 0u, s));
  const int lp = ceil_div(k, 16) * 16;
  const int hs = hgram_splits(n);
  auto h_phase = [&]() -> rnmf_status {
    // R = X^T W, S = W^T W, then the rows of H
    HIPCHK(launch_pack_t(W, md.dt, m, k, lp, b.ldpm, b.wp, md.cdt, s));
    HIPCHK(launch_tn(X, md.cdt, m, n, ldx, b.wp, b.ldpm, k, b.R, 0, b.part, b.tn, s));
    HIPCHK(launch_gram(W, md.dt, m, k, b.gpart, b.gsplits, b.S, s));
    HIPCHK(launch_hrow(b.R, b.S, H, n, k, o->alpha_h, o->beta_h, md.dt, s));
    return RNMF_OK;
  };
  auto w_phase = [&]() -> rnmf_status {
    // T = X H^T, V = H H^T, then the columns of W (row by row)
    HIPCHK(launch_pad(H, k, n, lp, b.ldpn, b.hp, md.dt, s));
    HIPCHK(launch_hgram(H, k, n, b.hpart, md.dt, s));
    HIPCHK(launch_gram_sum(b.hpart, hs, k, b.V, s));
    HIPCHK(launch_nn(X, md.cdt, m, n, ldx, b.hp, b.ldpn, k, b.T, b.part, b.nn, h.status, 0, s));
    HIPCHK(launch_wrow(b.T, b.V, W, m, k, o->alpha_w, o->beta_w, md.dt, s));
    return RNMF_OK;
  };
  for (int it = 0; it < nsweeps; ++it) {
    if (o->order == RNMF_ORDER_W_FIRST) {
      if ((r = w_phase()) != RNMF_OK) return r;
      if ((r = h_phase()) != RNMF_OK) return r;
    } else {
      if ((r = h_phase()) != RNMF_OK) return r;
      if ((r = w_phase()) != RNMF_OK) return r;
    }
  }
  return RNMF_OK;
}

rnmf_status rnmf_rel_error(const void* X, int xt, int64_t m, int64_t n, int64_t ldx, const void* W, const void* H,
                           int32_t k, const rnmf_opts* o, double* out, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!o) return fail(RNMF_ERR_ARG, "opts is NULL");
  if (!X || !W || !H || !out) return fail(RNMF_ERR_ARG, "X, W, H and out must be non-NULL");
  if (m < 1 || n < 1) return fail(RNMF_ERR_SHAPE, "empty matrix");
  if (ldx < n) return fail(RNMF_ERR_SHAPE, "ldx < n");
  if (k < 1) return fail(RNMF_ERR_ARG, "k < 1");
  rnmf_status r;
  if ((r = check_xt(o, xt)) != RNMF_OK) return r;
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  const Mode md = mode_of(o);
  Arena a(ws);
  a.take<char>(HDR_BYTES);
  RelBufs b = plan_rel(a, m, n);
  if ((r = check_ws(ws, ws_bytes, a.used)) != RNMF_OK) return r;
  HIPCHK(launch_relerr(X, xt, md.dt, m, n, ldx, W, H, k, b.part, b.np, out, d.stream));
  return RNMF_OK;
}

rnmf_status rnmf_factorize(const void* X, int xt, int64_t m, int64_t n, int64_t ldx, const rnmf_opts* o,
                           const void* Omega, const void* W0, const void* H0, void* W, void* H, rnmf_report* rep,
                           void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  rnmf_status r;
  if ((r = check_opts(o, m, n, true)) != RNMF_OK) return r;
  if ((r = check_xt(o, xt)) != RNMF_OK) return r;
  if (!X || !W || !H) return fail(RNMF_ERR_ARG, "X, W and H must be non-NULL");
  if (ldx < n) return fail(RNMF_ERR_SHAPE, "ldx < n");
  const bool svd = (o->flags & RNMF_FLAG_SVD_INIT) != 0;
  if (svd && (W0 || H0)) return fail(RNMF_ERR_ARG, "RNMF_FLAG_SVD_INIT needs W0 and H0 to be NULL");
  if (svd && (o->flags & RNMF_FLAG_GAUSS_INIT))
    return fail(RNMF_ERR_ARG, "RNMF_FLAG_SVD_INIT and RNMF_FLAG_GAUSS_INIT exclude each other");
  Dev d;
  if (!get_dev(d, (hipStream_t)stream)) return fail(RNMF_ERR_HIP, "no usable HIP device");
  const Mode md = mode_of(o);
  const int l = lwidth(o, m, n);
  const int k = o->k;
  void *Q, *B, *Wt, *Xb;
  SketchBufs sb;
  CompressBufs cb;
  InitBufs ib;
  SweepBufs wb;
  RelBufs rb;
  SvdBufs vb;
  size_t need = factorize_bytes(m, n, o, xt, d, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                nullptr, nullptr, nullptr);
  if ((r = check_ws(ws, ws_bytes, need)) != RNMF_OK) return r;
  factorize_bytes(m, n, o, xt, d, ws, &Q, &B, &Wt, &Xb, &sb, &cb, &ib, &wb, &rb, &vb);
  Hdr h = header(ws);
  hipStream_t s = d.stream;
  HIPCHK(launch_fill_u32((unsigned*)ws, HDR_BYTES / 4, 0u, s));
  const void* Xc;
  int64_t ldc;
  int check;
  // stage timing with events on the caller's stream
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { for (int i = 0; i < 4; ++i) if (e[i]) (void)hipEventDestroy(e[i]); }
  } guard{ev};
  for (int i = 0; i < 4; ++i) HIPCHK(hipEventCreate(&ev[i]));
  HIPCHK(hipEventRecord(ev[0], s));
  if ((r = prepare_x(X, xt, m, n, ldx, o, md, Xb, h, d, &Xc, &ldc, &check)) != RNMF_OK) return r;
  if ((r = run_sketch(Xc, m, n, ldc, Omega, o, Q, sb, md, h, check, d)) != RNMF_OK) return r;
  if ((r = run_compress(Xc, m, n, ldc, Q, l, B, cb, md, d)) != RNMF_OK) return r;
  if (svd) {
    HIPCHK(launch_svd_init(Q, B, m, n, l, k, W, H, md.dt, vb, s));
  } else {
    const int idist = (o->flags & RNMF_FLAG_GAUSS_INIT) ? 2 : 1;
    if (W0) HIPCHK(hipMemcpyAsync(W, W0, (size_t)m * k * md.es, hipMemcpyDeviceToDevice, s));
    else HIPCHK(launch_philox(W, md.dt, m, k, o->seed, 4u, idist, s));
    if (H0) HIPCHK(hipMemcpyAsync(H, H0, (size_t)k * n * md.es, hipMemcpyDeviceToDevice, s));
    else HIPCHK(launch_philox(H, md.dt, k, n, o->seed, 5u, idist, s));
  }
  if ((r = run_init_wt(Q, W, m, k, l, Wt, ib, md, d)) != RNMF_OK) return r;
  HIPCHK(hipEventRecord(ev[1], s));
  HIPCHK(launch_sweep(wb.sh, md.dt, Q, B, W, Wt, H, m, n, l, k, o->max_iter, o->tol, o->gram_mode, o->order, reg_of(o),
                      wb.xbuf, h.stats, h.status, nullptr, s));
  HIPCHK(hipEventRecord(ev[2], s));
  HIPCHK(launch_relerr(X, xt, md.dt, m, n, ldx, W, H, k, rb.part, rb.np, h.rel, s));
  HIPCHK(hipEventRecord(ev[3], s));
  // compressed error ||B - W~ H|| / ||B|| (into rel[2], rel[3]); rb.part is free again
  HIPCHK(launch_relerr(B, md.dt == 0 ? RNMF_F64 : RNMF_F32, md.dt, l, n, n, Wt, H, k, rb.part, rb.np, h.rel + 2, s));
  unsigned char host[256];
  HIPCHK(hipMemcpyAsync(host, ws, sizeof(host), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  unsigned bits;
  double stats[3], rel[4];
  std::memcpy(&bits, host, 4);
  std::memcpy(stats, host + 64, sizeof(stats));
  std::memcpy(rel, host + 128, sizeof(rel));
  rnmf_status st = status_from_bits(bits);
  const int iters = (int)stats[0];
  const double ratio = stats[1] > 0 ? stats[2] / stats[1] : 0.0;
  if (st == RNMF_OK && o->tol > 0.0 && iters >= o->max_iter && !(ratio < o->tol)) st = RNMF_NOT_CONVERGED;
  if (rep) {
    rep->iters = iters;
    rep->l_eff = l;
    rep->q_eff = q_effective(o);
    rep->qr_path = (bits & ST_SHIFTED) ? 1 : 0;
    rep->status = st;
    rep->reserved = 0;
    rep->rel_err = rel[1] > 0 ? std::sqrt(rel[0] / rel[1]) : 0.0;
    rep->comp_err = rel[3] > 0 ? std::sqrt(rel[2] / rel[3]) : 0.0;
    rep->pg_ratio = ratio;
    float ms[3] = {0.f, 0.f, 0.f};
    for (int i = 0; i < 3; ++i)
      if (hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]) != hipSuccess) ms[i] = -1.f;
    rep->ms_qb = ms[0];
    rep->ms_sweeps = ms[1];
    rep->ms_error = ms[2];
  }
  return st;
}

rnmf_status rnmf_cast_bf16(const float* X, int64_t m, int64_t n, int64_t ldx, void* Xb, void* stream) {
  g_err.clear();
  if (!X || !Xb) return fail(RNMF_ERR_ARG, "X and Xb must be non-NULL");
  if (m < 1 || n < 1 || ldx < n) return fail(RNMF_ERR_SHAPE, "bad shape");
  if ((uintptr_t)Xb % 8) return fail(RNMF_ERR_ARG, "Xb must be 8-byte aligned");
  // packed output (ld = n); the kernel writes 4-element groups, so an odd
  // tail is handled element by element
  HIPCHK(launch_cast_bf16(X, m, n, ldx, (bf16_t*)Xb, n, nullptr, 0, (hipStream_t)stream));
  return RNMF_OK;
}

rnmf_status rnmf_random(void* out, int dt, int64_t rows, int64_t cols, uint64_t seed, uint32_t stream_id,
                        int32_t dist, void* stream) {
  g_err.clear();
  if (!out) return fail(RNMF_ERR_ARG, "out must be non-NULL");
  if (rows < 0 || cols < 0) return fail(RNMF_ERR_SHAPE, "bad shape");
  if (dt != RNMF_F64 && dt != RNMF_F32) return fail(RNMF_ERR_DTYPE, "out must be RNMF_F64 or RNMF_F32");
  if (dist < RNMF_OMEGA_GAUSSIAN || dist > RNMF_DIST_GAUSS_CLIPPED)
    return fail(RNMF_ERR_ARG, "dist must be RNMF_OMEGA_GAUSSIAN, RNMF_OMEGA_UNIFORM or RNMF_DIST_GAUSS_CLIPPED");
  HIPCHK(launch_philox(out, dt == RNMF_F64 ? 0 : 1, rows, cols, seed, stream_id, dist, (hipStream_t)stream));
  return RNMF_OK;
}

rnmf_status rnmf_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count,
                               void* stream) {
  g_err.clear();
  if (count < 0) return fail(RNMF_ERR_SHAPE, "count must be >= 0");
  if (count > 0 && (!ctr || !key || !out)) return fail(RNMF_ERR_ARG, "ctr, key and out must be non-NULL");
  HIPCHK(launch_philox_raw(ctr, key, out, count, (hipStream_t)stream));
  return RNMF_OK;
}

rnmf_status rnmf_read_status(void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!ws || ws_bytes < HDR_BYTES) return fail(RNMF_ERR_WORKSPACE, "workspace missing or too small");
  unsigned bits = 0;
  hipStream_t s = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(&bits, ws, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(launch_fill_u32((unsigned*)ws, 1, 0u, s));
  HIPCHK(hipStreamSynchronize(s));
  return status_from_bits(bits);
}

}  // extern "C"

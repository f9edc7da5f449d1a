// Public launchers of the axis-pass kernels: argument and footprint checks,
// then dispatch on the grid size to the per-size launchers, which are
// instantiated in the fft_sizes_*.hip translation units.
#include "fft_passes.hpp"

namespace lpt2 {

// dispatch on the grid size (the sizes of LPT2_GRID_SIZES)
#define LPT2_CASE_(NN) \
  case NN:             \
    CALL(NN);          \
    break;
#define LPT2_SWITCH_N(n, CALL)            \
  switch (n) {                            \
    LPT2_GRID_SIZES(LPT2_CASE_)           \
    default: return hipErrorInvalidValue; \
  }

LPT2_GRID_SIZES(LPT2_DECLARE_SIZE)

int col_width(int prec, int n, int kind, int i) {
  if (kind < KIND_COL || kind > KIND_X) return 0;
#define W_(NN) return prec == PREC_F32 ? col_w<float>(NN, i, kind) : col_w<double>(NN, i, kind)
#define LPT2_WCASE_(NN) \
  case NN:              \
    W_(NN);
  switch (n) { LPT2_GRID_SIZES(LPT2_WCASE_) }
#undef LPT2_WCASE_
#undef W_
  return 0;
}

// 128-byte row runs where offered (measured on MI355X: narrower tiles lose
// more to the access granularity than they gain from extra blocks per CU)
int default_width(int prec, int n, int kind) { return col_width(prec, n, kind, 1); }

static inline size_t esize(int prec) { return prec == PREC_F32 ? 4 : 8; }

static inline bool supported_n(int n) {  // a supported grid size (LPT2_GRID_SIZES)
#define LPT2_IS_(NN) || n == NN
  return false LPT2_GRID_SIZES(LPT2_IS_);
#undef LPT2_IS_
}

Batch batch_one(const void* ext, int nf, long ext_fstride, long ws_fstride) {
  Batch b;
  std::memset(&b, 0, sizeof(b));
  b.nf = nf;
  b.nr = 1;
  b.ext_fstride = ext_fstride;
  b.ws_fstride = ws_fstride;
  b.ws_rstride = 0;
  b.ext[0] = ext;
  return b;
}

// Checks a Batch against its buffers: every caller buffer holds its nf
// fields of n^3 reals at ext_fstride, the workspace every (f, r) field.
static bool batch_ok(int prec, int n, const Batch& b, size_t ext_cap, const void* ws, size_t ws_cap) {
  if (b.nf < 1 || b.nf > 16 || b.nr < 1 || b.nr > BATCH_MAX || !ws) return false;
  if (b.ext_fstride < 0 || b.ws_fstride < 0 || b.ws_rstride < 0) return false;
  const size_t es = esize(prec), n3 = (size_t)n * n * n, nnm = (size_t)n * n * (n / 2);
  if (((size_t)(b.nf - 1) * b.ext_fstride + n3) * es > ext_cap) return false;
  const size_t end = (size_t)(b.nf - 1) * b.ws_fstride + (size_t)(b.nr - 1) * b.ws_rstride + nnm;
  if (end * 2 * es > ws_cap) return false;
  for (int r = 0; r < b.nr; ++r)
    if (!b.ext[r]) return false;
  return true;
}

hipError_t launch_zr2c(int prec, int n, const Batch& b, size_t ext_cap, void* ws, size_t ws_cap, const void* tw,
                       hipStream_t s) {
  if (!supported_n(n) || !tw || !batch_ok(prec, n, b, ext_cap, ws, ws_cap)) return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? zr2c_t<float, NN>(b, ws, tw, s) : zr2c_t<double, NN>(b, ws, tw, s)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

ZPow zpow_none() {
  ZPow z;
  for (int i = 0; i < ZPOW_MAX; ++i) {
    z.r[i] = 0;
    z.fmap[i] = i;
  }
  return z;
}

static bool zpow_ok(const ZPow& zp) {
  for (int i = 0; i < ZPOW_MAX; ++i)
    if (zp.r[i] < 0 || zp.r[i] > 2) return false;
  for (int i = 0; i < 6; ++i)
    if (zp.fmap[i] < 0 || zp.fmap[i] > 5) return false;
  return true;
}

hipError_t launch_zc2r(int prec, int n, const void* ws, size_t ws_cap, const Batch& b, size_t ext_cap, const ZPow& zp,
                       const void* tw, hipStream_t s) {
  if (!supported_n(n) || !tw || !zpow_ok(zp) || !batch_ok(prec, n, b, ext_cap, ws, ws_cap)) return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? zc2r_t<float, NN>(ws, b, zp, tw, s) : zc2r_t<double, NN>(ws, b, zp, tw, s)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_zsource(int prec, int n, const void* phi, size_t phi_cap, long fstride, const ZPow& zp, void* sk,
                          size_t sk_cap, long nlines, const void* tw, hipStream_t s) {
  if (nlines <= 0) return hipSuccess;
  if (!supported_n(n) || !phi || !sk || !tw || fstride < 0 || !zpow_ok(zp)) return hipErrorInvalidValue;
  const size_t cb = 2 * esize(prec), lc = (size_t)n / 2;
  if ((5 * (size_t)fstride + (size_t)nlines * lc) * cb > phi_cap || (size_t)nlines * lc * cb > sk_cap)
    return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? zsource_t<float, NN>(phi, fstride, zp, sk, nlines, tw, s) : zsource_t<double, NN>(phi, fstride, zp, sk, nlines, tw, s)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_zmg(int prec, int n, int kind, int nt, const void* in, size_t in_cap, long fstride, void* acc,
                      size_t acc_cap, long acc_fstride, long nlines, const void* tw, hipStream_t s) {
  if (nlines <= 0) return hipSuccess;
  if (!supported_n(n) || !in || !acc || !tw || fstride < 0 || acc_fstride < 0 || kind < 0 || kind > 2 ||
      (nt != 2 && nt != 3) || (kind == 2 && nt != 3))
    return hipErrorInvalidValue;
  const int nf = kind == 2 ? 7 : 3 * nt, nacc = kind == 2 ? 4 : nt;
  const size_t es = esize(prec), lc = (size_t)n / 2;
  if (((size_t)(nf - 1) * fstride + (size_t)nlines * lc) * 2 * es > in_cap ||
      ((size_t)(nacc - 1) * acc_fstride + (size_t)nlines * n) * es > acc_cap)
    return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? zmg_k<float, NN>(kind, nt, in, fstride, acc, acc_fstride, nlines, tw, s) : zmg_k<double, NN>(kind, nt, in, fstride, acc, acc_fstride, nlines, tw, s)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_zprodrule(int prec, int n, const void* phi, size_t phi_cap, long fstride, const void* sbar,
                            size_t sbar_cap, void* out, size_t out_cap, long out_fstride, long nlines, const ZPow& zp,
                            const void* tw, hipStream_t s) {
  if (nlines <= 0) return hipSuccess;
  if (!supported_n(n) || !phi || !sbar || !out || !tw || fstride < 0 || out_fstride < 0 || !zpow_ok(zp))
    return hipErrorInvalidValue;
  // every line is read before it is written only if the six fields are distinct
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < i; ++j)
      if (zp.fmap[i] == zp.fmap[j]) return hipErrorInvalidValue;
  const size_t cb = 2 * esize(prec), lc = (size_t)n / 2;
  if ((5 * (size_t)fstride + (size_t)nlines * lc) * cb > phi_cap ||
      (size_t)nlines * n * esize(prec) > sbar_cap ||
      (5 * (size_t)out_fstride + (size_t)nlines * lc) * cb > out_cap)
    return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? zprod_t<float, NN>(phi, fstride, sbar, out, out_fstride, nlines, zp, tw, s) : zprod_t<double, NN>(phi, fstride, sbar, out, out_fstride, nlines, zp, tw, s)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_colfft(int prec, int n, int dir, void* data, size_t cap, long nplanes, long plane_stride,
                         int ncols, long rowstride, const void* tw, hipStream_t s, int w) {
  if (w == 0) w = default_width(prec, n, KIND_COL);
  if (nplanes <= 0 || ncols <= 0) return hipSuccess;
  if (!supported_n(n) || !data || !tw || plane_stride < 0 || rowstride < ncols) return hipErrorInvalidValue;
  // one past the last element touched
  const size_t end = (size_t)(nplanes - 1) * plane_stride + (size_t)(n - 1) * rowstride + (size_t)ncols;
  if (end * 2 * esize(prec) > cap) return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? colfft_t<float, NN>(w, dir, data, nplanes, plane_stride, ncols, rowstride, tw, s) : colfft_t<double, NN>(w, dir, data, nplanes, plane_stride, ncols, rowstride, tw, s)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_ycombo(int prec, int n, int nr, const void* in, size_t in_cap, long in_fstride, void* out,
                         size_t out_cap, long out_fstride, const YOp& op, const void* tw, hipStream_t s, int w,
                         unsigned* tq) {
  if (w == 0) w = default_width(prec, n, KIND_MULTI);
  if (op.nin < 1 || op.nout < 1 || op.nin > YOP_MAX || op.nout > YOP_MAX || nr < 1) return hipErrorInvalidValue;
  if (!supported_n(n) || !in || !out || !tw || in_fstride < 0 || out_fstride < 0) return hipErrorInvalidValue;
  for (int o = 0; o < op.nout; ++o)
    if (op.src[o] < 0 || op.src[o] >= op.nin || op.pw[o] < 0 || op.pw[o] > 2) return hipErrorInvalidValue;
  const size_t cb = 2 * esize(prec), field = (size_t)nr * n * n * (n / 2);
  if (((size_t)(op.nin - 1) * in_fstride + field) * cb > in_cap) return hipErrorInvalidValue;
  if (((size_t)(op.nout - 1) * out_fstride + field) * cb > out_cap) return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? ycombo_t<float, NN>(w, nr, in, in_fstride, out, out_fstride, op, tw, s, tq) : ycombo_t<double, NN>(w, nr, in, in_fstride, out, out_fstride, op, tw, s, tq)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

static bool yfan_ok(const YFan& op) {
  if (op.nin < 1 || op.nout < 1 || op.nin > YFAN_MAX || op.nout > YFAN_MAX || op.nterm < op.nout ||
      op.nterm > YFAN_MAX || op.first[0] != 0 || op.first[op.nout] != op.nterm)
    return false;
  for (int o = 0; o < op.nout; ++o)
    if (op.first[o + 1] <= op.first[o]) return false;
  for (int k = 0; k < op.nterm; ++k)
    if (op.src[k] < 0 || op.src[k] >= op.nin || op.py[k] < 0 || op.py[k] > 2 || op.pz[k] < 0 || op.pz[k] > 2)
      return false;
  return true;
}

hipError_t launch_yfanin(int prec, int n, int nr, const void* in, size_t in_cap, long in_fstride, void* out,
                         size_t out_cap, long out_fstride, const YFan& op, const void* tw, hipStream_t s, int w,
                         unsigned* tq) {
  if (w == 0) w = default_width(prec, n, KIND_MULTI);
  if (!yfan_ok(op) || nr < 1) return hipErrorInvalidValue;
  if (!supported_n(n) || !in || !out || !tw || in_fstride < 0 || out_fstride < 0) return hipErrorInvalidValue;
  const size_t cb = 2 * esize(prec), field = (size_t)nr * n * n * (n / 2);
  if (((size_t)(op.nin - 1) * in_fstride + field) * cb > in_cap) return hipErrorInvalidValue;
  if (((size_t)(op.nout - 1) * out_fstride + field) * cb > out_cap) return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? yfanin_t<float, NN>(w, nr, in, in_fstride, out, out_fstride, op, tw, s, tq) : yfanin_t<double, NN>(w, nr, in, in_fstride, out, out_fstride, op, tw, s, tq)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_xdisp(int prec, int n, int nr, int mode, const void* in, size_t in_cap, void* out, size_t out_cap,
                        long out_fstride, const void* tab, size_t tab_cap, const void* tw, hipStream_t s, int w,
                        unsigned* tq) {
  if (w == 0) w = default_width(prec, n, KIND_X);
  if (!supported_n(n) || !in || !out || !tab || !tw || out_fstride < 0 || mode < 0 || mode > 3 || nr < 1)
    return hipErrorInvalidValue;
  const size_t cb = 2 * esize(prec), field = (size_t)nr * n * n * (n / 2);
  const int nout = mode == 0 ? 5 : (mode == 3 ? 3 : 2);
  if (field * cb > in_cap || ((size_t)(nout - 1) * out_fstride + field) * cb > out_cap) return hipErrorInvalidValue;
  if (nr > 65535) return hipErrorInvalidValue;  // grid.y
  const size_t n2cnt = 3 * (size_t)(n / 2) * (n / 2) + 1;
  if (n2cnt * esize(prec) * (mode == 1 ? 1 : 2) > tab_cap) return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? xdisp_t<float, NN>(w, nr, mode, in, out, out_fstride, tab, tw, s, tq) : xdisp_t<double, NN>(w, nr, mode, in, out, out_fstride, tab, tw, s, tq)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_xadj(int prec, int n, int mode, const void* in, size_t in_cap, long in_fstride, void* out,
                       size_t out_cap, const void* tab, size_t tab_cap, const void* tw, hipStream_t s, int w,
                       unsigned* tq) {
  if (w == 0) w = default_width(prec, n, KIND_X);
  if (!supported_n(n) || !in || !out || !tab || !tw || in_fstride < 0 || mode < 0 || mode > 1) return hipErrorInvalidValue;
  const int nin = mode == 0 ? 5 : 2;
  const size_t cb = 2 * esize(prec), field = (size_t)n * n * (n / 2);
  if (((size_t)(nin - 1) * in_fstride + field) * cb > in_cap || field * cb > out_cap) return hipErrorInvalidValue;
  // table entries up to |m|^2 = 3 (n/2)^2: pairs for mode 0, single values for mode 1
  const size_t n2cnt = 3 * (size_t)(n / 2) * (n / 2) + 1;
  if (n2cnt * esize(prec) * (mode == 0 ? 2 : 1) > tab_cap) return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? xadj_t<float, NN>(w, mode, in, in_fstride, out, tab, tw, s, tq) : xadj_t<double, NN>(w, mode, in, in_fstride, out, tab, tw, s, tq)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_xpass(int prec, int n, const void* in, size_t in_cap, long in_fstride, void* out, size_t out_cap,
                        long out_fstride, const XOp& op, long n2cnt, const void* tw, hipStream_t s) {
  if (op.nin < 1 || op.nout < 1 || (op.nin > 1 && op.nout > 1) || op.nin > XOP_MAX || op.nout > XOP_MAX)
    return hipErrorInvalidValue;
  if (!supported_n(n) || !in || !out || !tw || in_fstride < 0 || out_fstride < 0) return hipErrorInvalidValue;
  const size_t cb = 2 * esize(prec), field = (size_t)n * n * (n / 2);
  if (((size_t)(op.nin - 1) * in_fstride + field) * cb > in_cap) return hipErrorInvalidValue;
  if (((size_t)(op.nout - 1) * out_fstride + field) * cb > out_cap) return hipErrorInvalidValue;
  const long n2need = 3L * (n / 2) * (n / 2) + 1;
  const int ncodes = op.nin > op.nout ? op.nin : op.nout;
  for (int c = 0; c < ncodes; ++c) {
    if (op.kind[c] < MUL_REAL || op.kind[c] > MUL_MI) return hipErrorInvalidValue;
    if (op.ci[c] > 2 || op.cj[c] > 2) return hipErrorInvalidValue;
    if (op.table[c] >= 16) return hipErrorInvalidValue;
    if (op.table[c] >= 0 && (!op.tables[op.table[c]] || n2cnt < n2need)) return hipErrorInvalidValue;
  }
#define CALL(NN) return prec == PREC_F32 ? xpass_t<float, NN>(in, in_fstride, out, out_fstride, op, tw, s) : xpass_t<double, NN>(in, in_fstride, out, out_fstride, op, tw, s)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

}  // namespace lpt2


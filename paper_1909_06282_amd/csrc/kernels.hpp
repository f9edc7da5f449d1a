// Host-side launchers of the gfx950 kernels (one entry per kernel family;
// each dispatches on precision and grid size).  Every launcher is
// asynchronous on `s`, allocates nothing, and returns the launch status.
// Each takes the capacity in bytes of every buffer it is given (counted
// from the pointer passed) and refuses to launch, with
// hipErrorInvalidValue, if the grid would touch a byte beyond it.
//
// Spectral layout used throughout: a half spectrum of an n^3 real field is
// complex [n][n][n/2] (x slowest), i.e. the m_z = n/2 plane is not stored
// (every spectrum on the path has it masked to zero).
#pragma once
#include <hip/hip_runtime.h>

#include "physics.hpp"

namespace lpt2 {

enum { PREC_F64 = 0, PREC_F32 = 1 };

// Multiplier code of the fused x-pass.  The value applied to a mode
// (m_x, m_y, m_z) with |m|^2 = n2 is
//   scale * m_ci * m_cj * tables[table][n2]   (ci, cj, table < 0: factor 1)
// times 1, +i or -i (kind 0, 1, 2), and zero on DC and Nyquist planes.
enum { MUL_REAL = 0, MUL_PI = 1, MUL_MI = 2 };
constexpr int XOP_MAX = 12;
struct XOp {
  int nin, nout;   // nin == 1 (one input, nout outputs) or nout == 1 (sum over nin inputs)
  int inverse;     // 1: inverse x-FFT after the multiply; 0: store the k-space values
  int kind[XOP_MAX], ci[XOP_MAX], cj[XOP_MAX], table[XOP_MAX];
  double scale[XOP_MAX];
  const double* tables[16];
};

// Per-field power of m_z applied to a half-spectrum line before an inverse
// z transform: field f is multiplied by m_z^r[f] (r in {0, 1, 2}).
constexpr int ZPOW_MAX = 16;
struct ZPow {
  int r[ZPOW_MAX];
  int fmap[ZPOW_MAX];   // source pass: logical field f is stored at field fmap[f]
};
ZPow zpow_none();

// Realisation addressing of the z passes that read or write caller buffers:
// nf fields of nr realisations (nr <= BATCH_MAX), n^2 lines per field.
//   caller side: line l of field f of realisation r at ext[r] + f*ext_fstride + l*n   (reals)
//   workspace:   at ws + f*ws_fstride + r*ws_rstride + l*(n/2)                        (complex)
// Every ext[r] must hold ext_cap bytes.  Lines are numbered f-major, then r, then l.
constexpr int BATCH_MAX = 64;
struct Batch {
  int nf, nr;
  long ext_fstride;
  long ws_fstride, ws_rstride;
  const void* ext[BATCH_MAX];
};
// one realisation whose nf fields sit at ext + f*ext_fstride (reals); workspace fields at ws_fstride
Batch batch_one(const void* ext, int nf, long ext_fstride, long ws_fstride);

// Fused inverse y pass: output o = F^-1_y[ m_y^pw[o] * input src[o] ]
// (outputs grouped by source field).
constexpr int YOP_MAX = 16;
struct YOp {
  int nin, nout;
  int src[YOP_MAX], pw[YOP_MAX];
};

// z axis (contiguous): real lines of n values <-> n/2 complex modes
hipError_t launch_zr2c(int prec, int n, const Batch& b, size_t ext_cap, void* ws, size_t ws_cap, const void* tw,
                       hipStream_t s);
// (field f multiplied by m_z^zp.r[f] before the transform)
hipError_t launch_zc2r(int prec, int n, const void* ws, size_t ws_cap, const Batch& b, size_t ext_cap, const ZPow& zp,
                       const void* tw, hipStream_t s);
// strided complex column FFT in place: nplanes planes of ncols columns,
// element (row, col) of plane p at data + p*plane_stride + row*rowstride + col
// w: columns per block, one of col_width(n, 0..2); 0 picks default_width
hipError_t launch_colfft(int prec, int n, int dir, void* data, size_t cap, long nplanes, long plane_stride,
                         int ncols, long rowstride, const void* tw, hipStream_t s, int w = 0);
// pass kinds with a tile width of their own: single column FFTs, fused y
// passes, fused x passes (the index into a grid's tiles[])
enum { KIND_COL = 0, KIND_MULTI = 1, KIND_X = 2 };
int col_width(int prec, int n, int kind, int i);  // the three widths offered for (precision, n, kind); 0 if none
int default_width(int prec, int n, int kind);
// fused inverse y pass over the nr*n planes x n/2 columns of each field
// (nr realisations stored one after the other inside every field slot)
hipError_t launch_ycombo(int prec, int n, int nr, const void* in, size_t in_cap, long in_fstride, void* out,
                         size_t out_cap, long out_fstride, const YOp& op, const void* tw, hipStream_t s, int w = 0,
                         unsigned* tq = nullptr);
// adjoint x pass: mode 0 (tab = the PHI, PSI1 pair; inputs Ubar0..2, Vbar0..1)
// or mode 1 (tab = PSI2; inputs Qbar0..1), nin input fields in_fstride
// complex apart -> one output field (the transpose of the displacement x pass)
hipError_t launch_xadj(int prec, int n, int mode, const void* in, size_t in_cap, long in_fstride, void* out,
                       size_t out_cap, const void* tab, size_t tab_cap, const void* tw, hipStream_t s, int w = 0,
                       unsigned* tq = nullptr);
// fan-in y pass of the adjoint: output o sums terms first[o] .. first[o+1]-1;
// term k is the forward y-FFT of input field src[k] times m_y^py[k] m_z^pz[k]
// (powers 0..2; first[0] = 0, first[nout] = nterm, every output has a term)
constexpr int YFAN_MAX = 16;
struct YFan {
  int nin, nout, nterm;
  int first[YFAN_MAX + 1];
  int src[YFAN_MAX], py[YFAN_MAX], pz[YFAN_MAX];
};
hipError_t launch_yfanin(int prec, int n, int nr, const void* in, size_t in_cap, long in_fstride, void* out,
                         size_t out_cap, long out_fstride, const YFan& op, const void* tw, hipStream_t s, int w = 0,
                         unsigned* tq = nullptr);
// displacement x pass: mode 0 (tab = interleaved PHI, PSI1 per |m|^2; five
// outputs U0,U1,U2,V0,V1), mode 1 (tab = PSI2; outputs Q0,Q1), mode 2
// (tab = the PHI, PSI1 pair; outputs V0,V1) or mode 3 (the pair; outputs
// U0,U1,U2).  The table
// is in the working precision (pair: 2 values per |m|^2); tab_cap in bytes.
// nr realisations one after the other (n^2 (n/2) complex each) in the input
// and in every output field.
hipError_t launch_xdisp(int prec, int n, int nr, int mode, const void* in, size_t in_cap, void* out, size_t out_cap,
                        long out_fstride, const void* tab, size_t tab_cap, const void* tw, hipStream_t s, int w = 0,
                        unsigned* tq = nullptr);
// fused x pass over the n*(n/2) columns of each field
hipError_t launch_xpass(int prec, int n, const void* in, size_t in_cap, long in_fstride, void* out, size_t out_cap,
                        long out_fstride, const XOp& op, long n2cnt, const void* tw, hipStream_t s);
// z pass: 6 phi_,ij half-spectrum lines (xx,yy,zz,xy,xz,yz at fstride) -> S(k) line
// (field f of the six multiplied by m_z^zp.r[f] first)
hipError_t launch_zsource(int prec, int n, const void* phi, size_t phi_cap, long fstride, const ZPow& zp, void* sk,
                          size_t sk_cap, long nlines, const void* tw, hipStream_t s);
// z pass of the full MG source: kind 0 / 1 (diagonal / off-diagonal pairs,
// nt = 2 or 3 fields per pair), kind 2 (gradients and chi, f(R)); `in` holds
// the fields (half-spectrum lines, every k factor applied), `acc` the real
// accumulator fields acc_fstride reals apart (see k_zmg)
hipError_t launch_zmg(int prec, int n, int kind, int nt, const void* in, size_t in_cap, long fstride, void* acc,
                      size_t acc_cap, long acc_fstride, long nlines, const void* tw, hipStream_t s);
// z pass of the adjoint: 6 phi lines + real S_bar line -> 6 phi_bar half-spectrum lines
// (logical field f = xx,yy,zz,xy,xz,yz read and written at field zp.fmap[f],
// multiplied by m_z^zp.r[f] before its inverse transform)
hipError_t launch_zprodrule(int prec, int n, const void* phi, size_t phi_cap, long fstride, const void* sbar,
                            size_t sbar_cap, void* out, size_t out_cap, long out_fstride, long nlines, const ZPow& zp,
                            const void* tw, hipStream_t s);

// ---- auxiliary kernels (aux_kernels.hip) ----
struct GrowthSetup {
  Cosmo c;
  double a_init, a;
  int steps, nk;
  double lkmin, lkmax;
  double ratio, cs;     // triangle k1/k2 and cos(theta)
  int winther;
  int mode;             // 0: D2 = -3/7 D1^2; 1: D2 from the ODE; 2: Bouchet fit
};
// one block: raw ODE solves on the nk nodes and at k = 0, then normalised tables
hipError_t launch_growth(const GrowthSetup& g, double* d1n, double* d2n, hipStream_t s);

enum {
  TAB_PSI1 = 0, TAB_PHI, TAB_PSI2, TAB_A, TAB_R1, TAB_R2, TAB_R3, TAB_R4, TAB_R5, TAB_R6,
  TAB_C2, TAB_C4, TAB_C5, TAB_COUNT
};
// after the TAB_COUNT rows: the interleaved (PHI, PSI1) pair table (2 rows),
// then FP32 copies of the pair table (float2, 1 row) and of PSI2 (float,
// half a row): FP32 passes gather these (the same values rounded once).
constexpr int TAB_PAIR64 = TAB_COUNT, TAB_PAIR32 = TAB_COUNT + 2, TAB_PSI2_32 = TAB_COUNT + 3;
constexpr int TAB_ROWS = TAB_COUNT + 4;
struct RadialSetup {
  Cosmo c;
  int n;
  double box, amp, a;
  int nk;
  double lkmin, lkmax;
  int unit;   // 1: no sqrt(P n^3/V) shaping (the input is a density field, not white noise)
};
// per-|m|^2 FP64 tables: TAB_COUNT arrays of n2max + 1 = 3 (n/2)^2 + 1 entries,
// then the interleaved pair table (PHI, PSI1) of 2 (n2max + 1) entries
hipError_t launch_radial(const RadialSetup& r, const double* d1n, const double* d2n, double* tabs, long n2cnt,
                         hipStream_t s);

// deterministic shell binner: quantity 0 power (q = qscale |A|^2), 1 ratio
// (q = Re(A conj B)/|B|^2 where |B| > 0), 2 power divided by the squared
// CIC window.  partial: [nblk][nbins][4].
constexpr int BIN_BLOCKS = 512;
constexpr int BIN_MAXBINS = 512;
hipError_t launch_bin(int prec, int n, const void* A, size_t a_cap, const void* B, size_t b_cap, int quantity,
                      double qscale, int nbins, double kf, double* partial, double* out4, hipStream_t s);

// (every particle moved by `shift` cells along each axis before painting)
hipError_t launch_cic(int prec, int n, double box, const void* psi1, const void* psi2, void* delta, hipStream_t s,
                      double shift = 0.0);
// interlacing of two half-spectrum density transforms into a
hipError_t launch_interlace(int prec, int n, void* a, size_t a_cap, const void* b, size_t b_cap, hipStream_t s);
// x = (q + psi1 + psi2) mod box per particle and component ([3][n][n][n] each)
hipError_t launch_positions(int prec, int n, double box, const void* psi1, const void* psi2, void* pos, hipStream_t s);
hipError_t launch_cic_back(int prec, int n, double box, const void* psi1, const void* psi2, const void* gdelta,
                           void* gpsi, hipStream_t s);

// *out = number of non-finite values of x[0..count) (x holds count reals),
// zeroed by a kernel first
hipError_t launch_count_nonfinite(int prec, const void* x, long count, unsigned long long* out, hipStream_t s);
// x[0..count) = value (x must hold count values)
hipError_t launch_fill(int prec, void* x, long count, double value, hipStream_t s);

}  // namespace lpt2

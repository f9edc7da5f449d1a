// Axis-pass kernels of the 3D real FFTs, with the pointwise work of the
// 2LPT chain fused into them.
//
// A 3D transform of an n^3 real field is three passes over HBM:
//   z (contiguous): real lines of n values packed as n/2 complex, one complex
//     FFT of length n/2, then the split that yields modes 0..n/2-1;
//   y, x (strided): complex column FFTs of length n on tiles of W adjacent
//     columns, so every row access is a W-wide contiguous run.
// The k-space multipliers need all three wavenumbers, so they are applied
// in the x pass (the last forward / first inverse axis); real-space
// products are formed in the z pass (the last inverse / first forward
// axis), where a line sits in registers in real space.
#include <hip/hip_runtime.h>

#include "fft_core.hpp"
#include "kernels.hpp"

namespace lpt2 {

// ---------------------------------------------------------------------------
// z-line kernels.  A block owns whole lines and reads all of a line before
// any of its stores (barriers in between), so in == out is allowed.  The
// twiddle table (n entries) is staged in LDS at the start of every kernel.
// ---------------------------------------------------------------------------
template <int N>
struct LineCfg {
  static constexpr int L = N / 2;                       // complex length
  static constexpr int E = elems_per_thread(L);
  static constexpr int TPL = L / E;                     // threads per line
  static constexpr int BLOCK = 256;
  static constexpr int G = BLOCK / TPL;                 // lines per block
  static constexpr int R0F = plan_first(L, false);      // forward first radix
  static constexpr int RLF = plan_last(L, false);       // forward last radix
  static constexpr int R0I = plan_first(L, true);       // inverse first radix
  static constexpr int RLI = plan_last(L, true);        // inverse last radix (== R0F)
  static_assert(RLI == R0F, "inverse plan must end with the forward first radix");
};

template <typename T, int N>
__device__ __forceinline__ void stage_twiddles(Cx<T>* stw, const Cx<T>* __restrict__ tw) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) stw[i] = tw[i];
  __syncthreads();
}

// m^r for r = 0, 1, 2 (exact in T for |m| <= 512)
template <typename T>
__device__ __forceinline__ T mpow(int m, int r) {
  return r == 0 ? T(1) : (r == 1 ? T(m) : T(m) * T(m));
}

// Real line (n values, read as n/2 complex pairs) into the forward first-stage slots.
template <typename T, int N>
__device__ __forceinline__ void load_real_line(const T* src, Cx<T>* v, int t, bool act) {
  using C = LineCfg<N>;
  const Cx<T>* s2 = reinterpret_cast<const Cx<T>*>(src);
#pragma unroll
  for (int sl = 0; sl < C::E; ++sl) v[sl] = act ? s2[slot_elem<C::L, C::E, C::R0F>(t, sl)] : zero<T>();
}

// After a forward FFT of the packed line: split Z into the real line's modes
// X_k = (Z_k + Z*_{L-k})/2 - i W^k (Z_k - Z*_{L-k})/2, W = exp(-2 pi i/n),
// for k = 0..n/2-1 (the Nyquist mode is not kept), and store them.
template <typename T, int N>
__device__ __forceinline__ void r2c_finish(Cx<T>* v, int t, Cx<T>* lb, const Cx<T>* stw, Cx<T>* dst, bool act) {
  using C = LineCfg<N>;
  __syncthreads();
#pragma unroll
  for (int sl = 0; sl < C::E; ++sl) lb[slot_elem<C::L, C::E, C::RLF>(t, sl)] = v[sl];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < C::E; ++s) {
    const int k = t + s * C::TPL;
    const Cx<T> z = lb[k];
    const Cx<T> zc = conj(lb[(C::L - k) & (C::L - 1)]);
    const Cx<T> a = scale(z + zc, T(0.5));
    const Cx<T> wb = stw[k] * scale(z - zc, T(0.5));
    if (act) dst[k] = mk(a.x + wb.y, a.y - wb.x);
  }
}

// Load a half-spectrum line X_0..X_{n/2-1}, each mode multiplied by m_z^r,
// and form the packed spectrum Z_k = E_k + i O_k, E_k = X_k + X*_{L-k},
// O_k = (X_k - X*_{L-k}) conj(W^k), with X_{n/2} = 0 and Im X_0 ignored, in
// the inverse first-stage slots.  The unnormalised inverse FFT of Z then
// gives n x_{2j} + i n x_{2j+1}.
template <typename T, int N>
__device__ __forceinline__ void c2r_prepare(const Cx<T>* src, int r, Cx<T>* v, int t, Cx<T>* lb, const Cx<T>* stw,
                                            bool act) {
  using C = LineCfg<N>;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < C::E; ++s) {
    const int k = t + s * C::TPL;
    lb[k] = act ? scale(src[k], mpow<T>(k, r)) : zero<T>();
  }
  __syncthreads();
#pragma unroll
  for (int sl = 0; sl < C::E; ++sl) {
    const int e = slot_elem<C::L, C::E, C::R0I>(t, sl);
    Cx<T> x = lb[e];
    Cx<T> xc;
    if (e == 0) {
      x.y = T(0);
      xc = zero<T>();
    } else {
      xc = conj(lb[C::L - e]);
    }
    const Cx<T> ek = x + xc;
    const Cx<T> ok = (x - xc) * conj(stw[e]);
    v[sl] = mk(ek.x - ok.y, ek.y + ok.x);
  }
}

template <typename T, int N>
__global__ __launch_bounds__(256) void k_zr2c(const T* in, Cx<T>* out, long nlines, const Cx<T>* __restrict__ tw) {
  using C = LineCfg<N>;
  __shared__ Cx<T> lds[C::G * C::L];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int t = threadIdx.x % C::TPL, g = threadIdx.x / C::TPL;
  const long line = (long)blockIdx.x * C::G + g;
  const bool act = line < nlines;
  const long lsafe = act ? line : 0;
  Cx<T>* lb = lds + g * C::L;
  Cx<T> v[C::E];
  load_real_line<T, N>(in + lsafe * N, v, t, act);
  fft<T, C::L, -1, 1>(v, t, stw, 2, lb);
  r2c_finish<T, N>(v, t, lb, stw, out + lsafe * C::L, act);
}

// lines of field f = line / lines_per_field are multiplied by m_z^rpow[f]
template <typename T, int N>
__global__ __launch_bounds__(256) void k_zc2r(const Cx<T>* in, T* out, long nlines, ZPow zp,
                                              const Cx<T>* __restrict__ tw) {
  using C = LineCfg<N>;
  __shared__ Cx<T> lds[C::G * C::L];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int t = threadIdx.x % C::TPL, g = threadIdx.x / C::TPL;
  const long line = (long)blockIdx.x * C::G + g;
  const bool act = line < nlines;
  const long lsafe = act ? line : 0;
  const int f = (int)(lsafe / zp.lines_per_field);
  const int r = f < ZPOW_MAX ? zp.r[f] : 0;
  Cx<T>* lb = lds + g * C::L;
  Cx<T> v[C::E];
  c2r_prepare<T, N>(in + lsafe * C::L, r, v, t, lb, stw, act);
  fft<T, C::L, +1, 1>(v, t, stw, 2, lb);
  Cx<T>* d2 = reinterpret_cast<Cx<T>*>(out + lsafe * N);
  if (act) {
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) d2[slot_elem<C::L, C::E, C::RLI>(t, sl)] = v[sl];
  }
}

// S = phi_xx phi_yy + (phi_xx + phi_yy) phi_zz - phi_xy^2 - phi_xz^2 - phi_yz^2
// per real value (field f of the six multiplied by m_z^rpow[f] first), then
// the forward R2C of the S line.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_zsource(const Cx<T>* __restrict__ phi, long fstride, ZPow zp,
                                                 Cx<T>* __restrict__ sk, long nlines, const Cx<T>* __restrict__ tw) {
  using C = LineCfg<N>;
  __shared__ Cx<T> lds[C::G * C::L];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int t = threadIdx.x % C::TPL, g = threadIdx.x / C::TPL;
  const long line = (long)blockIdx.x * C::G + g;
  const bool act = line < nlines;
  const long lsafe = act ? line : 0;
  Cx<T>* lb = lds + g * C::L;
  Cx<T> a[C::E], s[C::E], v[C::E];
  const Cx<T>* src = phi + lsafe * C::L;
  c2r_prepare<T, N>(src, zp.r[0], v, t, lb, stw, act);
  fft<T, C::L, +1, 1>(v, t, stw, 2, lb);
#pragma unroll
  for (int i = 0; i < C::E; ++i) a[i] = v[i];
  c2r_prepare<T, N>(src + fstride, zp.r[1], v, t, lb, stw, act);
  fft<T, C::L, +1, 1>(v, t, stw, 2, lb);
#pragma unroll
  for (int i = 0; i < C::E; ++i) {
    s[i] = mk(a[i].x * v[i].x, a[i].y * v[i].y);
    a[i] = a[i] + v[i];
  }
  c2r_prepare<T, N>(src + 2 * fstride, zp.r[2], v, t, lb, stw, act);
  fft<T, C::L, +1, 1>(v, t, stw, 2, lb);
#pragma unroll
  for (int i = 0; i < C::E; ++i) s[i] = mk(s[i].x + a[i].x * v[i].x, s[i].y + a[i].y * v[i].y);
#pragma unroll 1
  for (int f = 3; f < 6; ++f) {
    c2r_prepare<T, N>(src + f * fstride, zp.r[f], v, t, lb, stw, act);
    fft<T, C::L, +1, 1>(v, t, stw, 2, lb);
#pragma unroll
    for (int i = 0; i < C::E; ++i) s[i] = mk(s[i].x - v[i].x * v[i].x, s[i].y - v[i].y * v[i].y);
  }
  fft<T, C::L, -1, 1>(s, t, stw, 2, lb);
  r2c_finish<T, N>(s, t, lb, stw, sk + lsafe * C::L, act);
}

// Adjoint of the source: with S_bar given per real value,
//   phi_bar_ii = S_bar (tr phi - phi_ii), phi_bar_ij = -2 S_bar phi_ij (i < j),
// each forward-transformed along z.  phi and out may be the same buffers.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_zprodrule(const Cx<T>* phi, long fstride, const T* __restrict__ sbar,
                                                   Cx<T>* out, long ofstride, long nlines,
                                                   const Cx<T>* __restrict__ tw) {
  using C = LineCfg<N>;
  __shared__ Cx<T> lds[C::G * C::L];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int t = threadIdx.x % C::TPL, g = threadIdx.x / C::TPL;
  const long line = (long)blockIdx.x * C::G + g;
  const bool act = line < nlines;
  const long lsafe = act ? line : 0;
  Cx<T>* lb = lds + g * C::L;
  Cx<T> sb[C::E], d0[C::E], d1[C::E], d2[C::E], v[C::E];
  load_real_line<T, N>(sbar + lsafe * N, sb, t, act);
  const Cx<T>* src = phi + lsafe * C::L;
  c2r_prepare<T, N>(src, 0, d0, t, lb, stw, act);
  fft<T, C::L, +1, 1>(d0, t, stw, 2, lb);
  c2r_prepare<T, N>(src + fstride, 0, d1, t, lb, stw, act);
  fft<T, C::L, +1, 1>(d1, t, stw, 2, lb);
  c2r_prepare<T, N>(src + 2 * fstride, 0, d2, t, lb, stw, act);
  fft<T, C::L, +1, 1>(d2, t, stw, 2, lb);
  Cx<T>* dst = out + lsafe * C::L;
#pragma unroll
  for (int i = 0; i < C::E; ++i) v[i] = mk(sb[i].x * (d1[i].x + d2[i].x), sb[i].y * (d1[i].y + d2[i].y));
  fft<T, C::L, -1, 1>(v, t, stw, 2, lb);
  r2c_finish<T, N>(v, t, lb, stw, dst, act);
#pragma unroll
  for (int i = 0; i < C::E; ++i) v[i] = mk(sb[i].x * (d0[i].x + d2[i].x), sb[i].y * (d0[i].y + d2[i].y));
  fft<T, C::L, -1, 1>(v, t, stw, 2, lb);
  r2c_finish<T, N>(v, t, lb, stw, dst + ofstride, act);
#pragma unroll
  for (int i = 0; i < C::E; ++i) v[i] = mk(sb[i].x * (d0[i].x + d1[i].x), sb[i].y * (d0[i].y + d1[i].y));
  fft<T, C::L, -1, 1>(v, t, stw, 2, lb);
  r2c_finish<T, N>(v, t, lb, stw, dst + 2 * ofstride, act);
#pragma unroll 1
  for (int f = 3; f < 6; ++f) {
    c2r_prepare<T, N>(src + f * fstride, 0, v, t, lb, stw, act);
    fft<T, C::L, +1, 1>(v, t, stw, 2, lb);
#pragma unroll
    for (int i = 0; i < C::E; ++i) v[i] = mk(T(-2) * sb[i].x * v[i].x, T(-2) * sb[i].y * v[i].y);
    fft<T, C::L, -1, 1>(v, t, stw, 2, lb);
    r2c_finish<T, N>(v, t, lb, stw, dst + f * ofstride, act);
  }
}

// ---------------------------------------------------------------------------
// strided column kernels: a block takes W adjacent columns of one plane
// (lane = column fastest), so every row access is W contiguous complex.
// ---------------------------------------------------------------------------
// EPT: complex values per thread (8, or 16 for the multi-transform kernels
// so that their blocks are half as large and two fit on a CU).
template <typename T, int N, int EPT = elems_per_thread(N)>
struct ColCfg {
  static constexpr int L = N;
  static constexpr int E = (EPT < L) ? EPT : L;
  static constexpr int TPC = L / E;                     // threads per column
  static constexpr int WMIN = sizeof(T) == 4 ? 16 : 8;  // 128-byte rows
  static constexpr int W = (256 / TPC > WMIN) ? 256 / TPC : WMIN;
  static constexpr int BLOCK = W * TPC;
  static constexpr int R0F = plan_first(L, false), RLF = plan_last(L, false);
  static constexpr int R0I = plan_first(L, true), RLI = plan_last(L, true);
  static_assert(RLF == R0I && RLI == R0F, "reversed plans");
};
// elements per thread of the fused x and y passes
template <int N>
constexpr int multi_ept() { return elems_per_thread(N); }

template <typename T, int N, int D>
__global__ __launch_bounds__((ColCfg<T, N>::BLOCK)) void k_colfft(Cx<T>* __restrict__ data, int ncols, int bpp,
                                                                  long plane_stride, long rowstride,
                                                                  const Cx<T>* __restrict__ tw) {
  using C = ColCfg<T, N>;
  __shared__ Cx<T> lds[C::L * C::W];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int c = threadIdx.x % C::W, t = threadIdx.x / C::W;
  const long plane = blockIdx.x / bpp;
  const int col = (blockIdx.x % bpp) * C::W + c;
  const bool act = col < ncols;
  Cx<T>* base = data + plane * plane_stride + (act ? col : 0);
  constexpr int RIN = (D < 0) ? C::R0F : C::R0I;
  constexpr int ROUT = (D < 0) ? C::RLF : C::RLI;
  Cx<T> v[C::E];
#pragma unroll
  for (int sl = 0; sl < C::E; ++sl) v[sl] = act ? base[slot_elem<C::L, C::E, RIN>(t, sl) * rowstride] : zero<T>();
  fft<T, C::L, D, C::W>(v, t, stw, 1, lds + c);
  if (act) {
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) base[slot_elem<C::L, C::E, ROUT>(t, sl) * rowstride] = v[sl];
  }
}

// Fused y pass of the inverse chain: output o is the inverse y-FFT of input
// field src[o] multiplied by m_y^pw[o] (outputs grouped by source, so each
// input column tile is read once).
template <typename T, int N>
__global__ __launch_bounds__((ColCfg<T, N, multi_ept<N>()>::BLOCK)) void k_ycombo(const Cx<T>* __restrict__ in, long fsi,
                                                                  Cx<T>* __restrict__ out, long fso, YOp op,
                                                                  const Cx<T>* __restrict__ tw) {
  using C = ColCfg<T, N, multi_ept<N>()>;
  constexpr int M = N / 2;
  constexpr int BPP = (M + C::W - 1) / C::W;
  __shared__ Cx<T> lds[C::L * C::W];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int c = threadIdx.x % C::W, t = threadIdx.x / C::W;
  const long plane = blockIdx.x / BPP;                    // x index
  const int col = (blockIdx.x % BPP) * C::W + c;          // z index
  const bool act = col < M;
  const long off = plane * (long)N * M + (act ? col : 0);
  Cx<T> v[C::E], y[C::E];
  int cur = -1;
#pragma unroll 1
  for (int o = 0; o < op.nout; ++o) {
    if (op.src[o] != cur) {
      cur = op.src[o];
      const Cx<T>* b = in + cur * fsi + off;
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) v[sl] = act ? b[slot_elem<C::L, C::E, C::R0I>(t, sl) * M] : zero<T>();
    }
    const int pw = op.pw[o];
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) {
      const int iy = slot_elem<C::L, C::E, C::R0I>(t, sl);
      y[sl] = scale(v[sl], mpow<T>(iy < N / 2 ? iy : iy - N, pw));
    }
    fft<T, C::L, +1, C::W, C::E>(y, t, stw, 1, lds + c);
    if (act) {
      Cx<T>* d = out + o * fso + off;
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) d[slot_elem<C::L, C::E, C::RLI>(t, sl) * M] = y[sl];
    }
  }
}

// Fused x pass: forward x-FFT of each input column, multiply by the codes of
// `op` (FP64, rounded once), then (op.inverse) inverse x-FFT, store.
template <typename T>
__device__ __forceinline__ Cx<T> xop_mul(const XOp& op, int c, int mx, int my, int mz, long n2, bool keep) {
  if (!keep) return zero<T>();
  double val = op.scale[c];
  const int ci = op.ci[c], cj = op.cj[c], tb = op.table[c];
  const int m3[3] = {mx, my, mz};
  if (ci >= 0) val *= (double)m3[ci];
  if (cj >= 0) val *= (double)m3[cj];
  if (tb >= 0) val *= op.tables[tb][n2];
  const int kd = op.kind[c];
  return kd == MUL_REAL ? mk(T(val), T(0)) : (kd == MUL_PI ? mk(T(0), T(val)) : mk(T(0), T(-val)));
}

template <typename T, int N>
__global__ __launch_bounds__((ColCfg<T, N, multi_ept<N>()>::BLOCK)) void k_xpass(const Cx<T>* __restrict__ in, long fsi,
                                                                 Cx<T>* __restrict__ out, long fso, XOp op,
                                                                 const Cx<T>* __restrict__ tw) {
  using C = ColCfg<T, N, multi_ept<N>()>;
  constexpr int M = N / 2;
  constexpr long NCOL = (long)N * M;
  __shared__ Cx<T> lds[C::L * C::W];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int c = threadIdx.x % C::W, t = threadIdx.x / C::W;
  const long col = (long)blockIdx.x * C::W + c;
  const bool act = col < NCOL;
  const long cs = act ? col : 0;
  const int iy = (int)(cs / M), iz = (int)(cs % M);
  const int my = iy < N / 2 ? iy : iy - N;
  const bool keep_y = iy != N / 2;
  const long n2yz = (long)my * my + (long)iz * iz;
  Cx<T> v[C::E], y[C::E];
  if (op.nin == 1) {
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) v[sl] = act ? in[cs + slot_elem<C::L, C::E, C::R0F>(t, sl) * NCOL] : zero<T>();
    fft<T, C::L, -1, C::W, C::E>(v, t, stw, 1, lds + c);
#pragma unroll 1
    for (int o = 0; o < op.nout; ++o) {
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) {
        const int ix = slot_elem<C::L, C::E, C::RLF>(t, sl);
        const int mx = ix < N / 2 ? ix : ix - N;
        const long n2 = (long)mx * mx + n2yz;
        y[sl] = xop_mul<T>(op, o, mx, my, iz, n2, keep_y && ix != N / 2 && n2 != 0) * v[sl];
      }
      Cx<T>* dst = out + o * fso + cs;
      if (op.inverse) {
        fft<T, C::L, +1, C::W, C::E>(y, t, stw, 1, lds + c);
        if (act) {
#pragma unroll
          for (int sl = 0; sl < C::E; ++sl) dst[slot_elem<C::L, C::E, C::RLI>(t, sl) * NCOL] = y[sl];
        }
      } else if (act) {
#pragma unroll
        for (int sl = 0; sl < C::E; ++sl) dst[slot_elem<C::L, C::E, C::RLF>(t, sl) * NCOL] = y[sl];
      }
    }
  } else {
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) y[sl] = zero<T>();
#pragma unroll 1
    for (int f = 0; f < op.nin; ++f) {
      const Cx<T>* src = in + f * fsi + cs;
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) v[sl] = act ? src[slot_elem<C::L, C::E, C::R0F>(t, sl) * NCOL] : zero<T>();
      fft<T, C::L, -1, C::W, C::E>(v, t, stw, 1, lds + c);
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) {
        const int ix = slot_elem<C::L, C::E, C::RLF>(t, sl);
        const int mx = ix < N / 2 ? ix : ix - N;
        const long n2 = (long)mx * mx + n2yz;
        y[sl] = y[sl] + xop_mul<T>(op, f, mx, my, iz, n2, keep_y && ix != N / 2 && n2 != 0) * v[sl];
      }
    }
    Cx<T>* dst = out + cs;
    if (op.inverse) {
      fft<T, C::L, +1, C::W, C::E>(y, t, stw, 1, lds + c);
      if (act) {
#pragma unroll
        for (int sl = 0; sl < C::E; ++sl) dst[slot_elem<C::L, C::E, C::RLI>(t, sl) * NCOL] = y[sl];
      }
    } else if (act) {
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) dst[slot_elem<C::L, C::E, C::RLF>(t, sl) * NCOL] = y[sl];
    }
  }
}

// ---------------------------------------------------------------------------
// launchers (footprint checks, then the launch)
// ---------------------------------------------------------------------------
#define LPT2_SWITCH_N(n, CALL)     \
  switch (n) {                     \
    case 8: CALL(8); break;        \
    case 16: CALL(16); break;      \
    case 32: CALL(32); break;      \
    case 64: CALL(64); break;      \
    case 128: CALL(128); break;    \
    case 256: CALL(256); break;    \
    case 512: CALL(512); break;    \
    default: return hipErrorInvalidValue; \
  }

static inline size_t esize(int prec) { return prec == PREC_F32 ? 4 : 8; }
static inline bool pow2n(int n) { return n >= 8 && n <= 512 && (n & (n - 1)) == 0; }

template <typename T, int N>
static hipError_t zr2c_t(const void* in, void* out, long nlines, const void* tw, hipStream_t s) {
  using C = LineCfg<N>;
  const long blocks = (nlines + C::G - 1) / C::G;
  hipLaunchKernelGGL((k_zr2c<T, N>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const T*)in, (Cx<T>*)out, nlines,
                     (const Cx<T>*)tw);
  return hipGetLastError();
}
hipError_t launch_zr2c(int prec, int n, const void* in, size_t in_cap, void* out, size_t out_cap, long nlines,
                       const void* tw, hipStream_t s) {
  if (nlines <= 0) return hipSuccess;
  if (!pow2n(n) || !in || !out || !tw) return hipErrorInvalidValue;
  const size_t line = (size_t)n * esize(prec);  // n reals = n/2 complex
  if ((size_t)nlines * line > in_cap || (size_t)nlines * line > out_cap) return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? zr2c_t<float, NN>(in, out, nlines, tw, s) : zr2c_t<double, NN>(in, out, nlines, tw, s)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

ZPow zpow_none(long lines_per_field) {
  ZPow z;
  z.lines_per_field = lines_per_field > 0 ? lines_per_field : 1;
  for (int i = 0; i < ZPOW_MAX; ++i) z.r[i] = 0;
  return z;
}
static bool zpow_ok(const ZPow& zp) {
  if (zp.lines_per_field <= 0) return false;
  for (int i = 0; i < ZPOW_MAX; ++i)
    if (zp.r[i] < 0 || zp.r[i] > 2) return false;
  return true;
}

template <typename T, int N>
static hipError_t zc2r_t(const void* in, void* out, long nlines, const ZPow& zp, const void* tw, hipStream_t s) {
  using C = LineCfg<N>;
  const long blocks = (nlines + C::G - 1) / C::G;
  hipLaunchKernelGGL((k_zc2r<T, N>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const Cx<T>*)in, (T*)out, nlines,
                     zp, (const Cx<T>*)tw);
  return hipGetLastError();
}
hipError_t launch_zc2r(int prec, int n, const void* in, size_t in_cap, void* out, size_t out_cap, long nlines,
                       const ZPow& zp, const void* tw, hipStream_t s) {
  if (nlines <= 0) return hipSuccess;
  if (!pow2n(n) || !in || !out || !tw || !zpow_ok(zp)) return hipErrorInvalidValue;
  const size_t line = (size_t)n * esize(prec);
  if ((size_t)nlines * line > in_cap || (size_t)nlines * line > out_cap) return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? zc2r_t<float, NN>(in, out, nlines, zp, tw, s) : zc2r_t<double, NN>(in, out, nlines, zp, tw, s)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

template <typename T, int N>
static hipError_t zsource_t(const void* phi, long fstride, const ZPow& zp, void* sk, long nlines, const void* tw,
                            hipStream_t s) {
  using C = LineCfg<N>;
  const long blocks = (nlines + C::G - 1) / C::G;
  hipLaunchKernelGGL((k_zsource<T, N>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const Cx<T>*)phi, fstride, zp,
                     (Cx<T>*)sk, nlines, (const Cx<T>*)tw);
  return hipGetLastError();
}
hipError_t launch_zsource(int prec, int n, const void* phi, size_t phi_cap, long fstride, const ZPow& zp, void* sk,
                          size_t sk_cap, long nlines, const void* tw, hipStream_t s) {
  if (nlines <= 0) return hipSuccess;
  if (!pow2n(n) || !phi || !sk || !tw || fstride < 0 || !zpow_ok(zp)) return hipErrorInvalidValue;
  const size_t cb = 2 * esize(prec), lc = (size_t)n / 2;
  if ((5 * (size_t)fstride + (size_t)nlines * lc) * cb > phi_cap || (size_t)nlines * lc * cb > sk_cap)
    return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? zsource_t<float, NN>(phi, fstride, zp, sk, nlines, tw, s) : zsource_t<double, NN>(phi, fstride, zp, sk, nlines, tw, s)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

template <typename T, int N>
static hipError_t zprod_t(const void* phi, long fstride, const void* sbar, void* out, long ofs, long nlines,
                          const void* tw, hipStream_t s) {
  using C = LineCfg<N>;
  const long blocks = (nlines + C::G - 1) / C::G;
  hipLaunchKernelGGL((k_zprodrule<T, N>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const Cx<T>*)phi, fstride,
                     (const T*)sbar, (Cx<T>*)out, ofs, nlines, (const Cx<T>*)tw);
  return hipGetLastError();
}
hipError_t launch_zprodrule(int prec, int n, const void* phi, size_t phi_cap, long fstride, const void* sbar,
                            size_t sbar_cap, void* out, size_t out_cap, long out_fstride, long nlines, const void* tw,
                            hipStream_t s) {
  if (nlines <= 0) return hipSuccess;
  if (!pow2n(n) || !phi || !sbar || !out || !tw || fstride < 0 || out_fstride < 0) return hipErrorInvalidValue;
  const size_t cb = 2 * esize(prec), lc = (size_t)n / 2;
  if ((5 * (size_t)fstride + (size_t)nlines * lc) * cb > phi_cap ||
      (size_t)nlines * n * esize(prec) > sbar_cap ||
      (5 * (size_t)out_fstride + (size_t)nlines * lc) * cb > out_cap)
    return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? zprod_t<float, NN>(phi, fstride, sbar, out, out_fstride, nlines, tw, s) : zprod_t<double, NN>(phi, fstride, sbar, out, out_fstride, nlines, tw, s)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

template <typename T, int N>
static hipError_t colfft_t(int dir, void* data, long nplanes, long plane_stride, int ncols, long rowstride,
                           const void* tw, hipStream_t s) {
  using C = ColCfg<T, N>;
  const int bpp = (ncols + C::W - 1) / C::W;
  const long blocks = nplanes * bpp;
  if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
  if (dir < 0)
    hipLaunchKernelGGL((k_colfft<T, N, -1>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (Cx<T>*)data, ncols, bpp,
                       plane_stride, rowstride, (const Cx<T>*)tw);
  else
    hipLaunchKernelGGL((k_colfft<T, N, +1>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (Cx<T>*)data, ncols, bpp,
                       plane_stride, rowstride, (const Cx<T>*)tw);
  return hipGetLastError();
}
hipError_t launch_colfft(int prec, int n, int dir, void* data, size_t cap, long nplanes, long plane_stride,
                         int ncols, long rowstride, const void* tw, hipStream_t s) {
  if (nplanes <= 0 || ncols <= 0) return hipSuccess;
  if (!pow2n(n) || !data || !tw || plane_stride < 0 || rowstride < ncols) return hipErrorInvalidValue;
  // one past the last element touched
  const size_t end = (size_t)(nplanes - 1) * plane_stride + (size_t)(n - 1) * rowstride + (size_t)ncols;
  if (end * 2 * esize(prec) > cap) return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? colfft_t<float, NN>(dir, data, nplanes, plane_stride, ncols, rowstride, tw, s) : colfft_t<double, NN>(dir, data, nplanes, plane_stride, ncols, rowstride, tw, s)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

template <typename T, int N>
static hipError_t ycombo_t(const void* in, long fsi, void* out, long fso, const YOp& op, const void* tw,
                           hipStream_t s) {
  using C = ColCfg<T, N, multi_ept<N>()>;
  constexpr int M = N / 2;
  const long blocks = (long)N * ((M + C::W - 1) / C::W);
  hipLaunchKernelGGL((k_ycombo<T, N>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const Cx<T>*)in, fsi,
                     (Cx<T>*)out, fso, op, (const Cx<T>*)tw);
  return hipGetLastError();
}
hipError_t launch_ycombo(int prec, int n, const void* in, size_t in_cap, long in_fstride, void* out, size_t out_cap,
                         long out_fstride, const YOp& op, const void* tw, hipStream_t s) {
  if (op.nin < 1 || op.nout < 1 || op.nin > YOP_MAX || op.nout > YOP_MAX) return hipErrorInvalidValue;
  if (!pow2n(n) || !in || !out || !tw || in_fstride < 0 || out_fstride < 0) return hipErrorInvalidValue;
  for (int o = 0; o < op.nout; ++o)
    if (op.src[o] < 0 || op.src[o] >= op.nin || op.pw[o] < 0 || op.pw[o] > 2) return hipErrorInvalidValue;
  const size_t cb = 2 * esize(prec), field = (size_t)n * n * (n / 2);
  if (((size_t)(op.nin - 1) * in_fstride + field) * cb > in_cap) return hipErrorInvalidValue;
  if (((size_t)(op.nout - 1) * out_fstride + field) * cb > out_cap) return hipErrorInvalidValue;
#define CALL(NN) return prec == PREC_F32 ? ycombo_t<float, NN>(in, in_fstride, out, out_fstride, op, tw, s) : ycombo_t<double, NN>(in, in_fstride, out, out_fstride, op, tw, s)
  LPT2_SWITCH_N(n, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

template <typename T, int N>
static hipError_t xpass_t(const void* in, long fsi, void* out, long fso, const XOp& op, const void* tw,
                          hipStream_t s) {
  using C = ColCfg<T, N, multi_ept<N>()>;
  const long ncol = (long)N * (N / 2);
  const long blocks = (ncol + C::W - 1) / C::W;
  hipLaunchKernelGGL((k_xpass<T, N>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const Cx<T>*)in, fsi,
                     (Cx<T>*)out, fso, op, (const Cx<T>*)tw);
  return hipGetLastError();
}
hipError_t launch_xpass(int prec, int n, const void* in, size_t in_cap, long in_fstride, void* out, size_t out_cap,
                        long out_fstride, const XOp& op, long n2cnt, const void* tw, hipStream_t s) {
  if (op.nin < 1 || op.nout < 1 || (op.nin > 1 && op.nout > 1) || op.nin > XOP_MAX || op.nout > XOP_MAX)
    return hipErrorInvalidValue;
  if (!pow2n(n) || !in || !out || !tw || in_fstride < 0 || out_fstride < 0) return hipErrorInvalidValue;
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

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
//
// This header holds the kernels and their per-size launchers; the public
// launchers (fft_kernels.hip) check their arguments and dispatch on n.
#pragma once
#include <hip/hip_runtime.h>

#include <cstring>

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
  static constexpr int G = 256 / TPL;                   // lines per block
  static constexpr int BLOCK = G * TPL;                 // 256, or just under for the lengths with a factor 5 or 7
  static constexpr int R0F = plan_first(L, false);      // forward first radix
  static constexpr int RLF = plan_last(L, false);       // forward last radix
  static constexpr int R0I = plan_first(L, true);       // inverse first radix
  static constexpr int RLI = plan_last(L, true);        // inverse last radix (== R0F)
  static_assert(RLI == R0F, "inverse plan must end with the forward first radix");
  // a line inside one wavefront synchronises at wave level; lines of 10,
  // 20, 30 or 35 threads (lengths with a factor 5 or 7) straddle wavefronts
  // and synchronise the block
  static constexpr bool WAVE = TPL <= 64 && 64 % TPL == 0;
  static constexpr int SY = WAVE ? SY_WAVE : SY_BLOCK;
  static_assert(G >= 1 && BLOCK <= 256, "lines per block");
  static constexpr int SPAN = lds_span<true>(L);       // LDS slots per line (room for padding)
};

template <typename T, int N>
__device__ __forceinline__ void stage_twiddles(Cx<T>* stw, const Cx<T>* __restrict__ tw) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) stw[i] = tw[i];
  __syncthreads();
}

// m^r for r = 0, 1, 2 as 1 + r d + r(r-1)/2 d^2 with d = m - 1: no branch on
// r, which is a runtime value uniform over the block in most callers and
// would otherwise become scalar branches that split the loads and LDS
// accesses around it (measured 3-5% on the fused passes at n = 512).  Exact
// in T for the |m| <= 384 of the grids here: every intermediate is an
// integer below 2^24.
template <typename T>
__device__ __forceinline__ T mpow(int m, int r) {
  const T d = T(m - 1);
  return T(1) + d * (T(r) + T((r * (r - 1)) >> 1) * d);
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
template <typename T, int N, bool PAD = true>
__device__ __forceinline__ void r2c_finish(Cx<T>* v, int t, Cx<T>* lb, const Cx<T>* stw, Cx<T>* dst, bool act) {
  using C = LineCfg<N>;
  lds_sync<C::SY>();
#pragma unroll
  for (int sl = 0; sl < C::E; ++sl) lb[lds_index<PAD>(slot_elem<C::L, C::E, C::RLF>(t, sl))] = v[sl];
  lds_sync<C::SY>();
#pragma unroll
  for (int s = 0; s < C::E; ++s) {
    const int k = t + s * C::TPL;
    const Cx<T> z = lb[lds_index<PAD>(k)];
    const Cx<T> zc = conj(lb[lds_index<PAD>(k == 0 ? 0 : C::L - k)]);
    const Cx<T> a = scale(z + zc, T(0.5));
    const Cx<T> wb = stw[k] * scale(z - zc, T(0.5));
    if (act) dst[k] = mk(a.x + wb.y, a.y - wb.x);
  }
}

// A half-spectrum line X_0..X_{n/2-1} into registers (raw[s] = X_{t + s*TPL}).
// Every load is issued before any is used, so they are in flight together;
// callers pass an address inside the buffer also for an inactive line.
template <typename T, int N>
__device__ __forceinline__ void load_cx_line(const Cx<T>* src, Cx<T>* raw, int t) {
  using C = LineCfg<N>;
#pragma unroll
  for (int s = 0; s < C::E; ++s) raw[s] = src[t + s * C::TPL];
}

// From a line in registers, each mode multiplied by m_z^r, form the packed
// spectrum Z_k = E_k + i O_k, E_k = X_k + X*_{L-k}, O_k = (X_k - X*_{L-k})
// conj(W^k), with X_{n/2} = 0 and Im X_0 ignored, in the inverse first-stage
// slots.  The unnormalised inverse FFT of Z then gives n x_{2j} + i n x_{2j+1}.
template <typename T, int N, bool PAD = true>
__device__ __forceinline__ void c2r_prepare_regs(const Cx<T>* raw, int r, Cx<T>* v, int t, Cx<T>* lb,
                                                 const Cx<T>* stw) {
  using C = LineCfg<N>;
  lds_sync<C::SY>();
#pragma unroll
  for (int s = 0; s < C::E; ++s) {
    const int k = t + s * C::TPL;
    lb[lds_index<PAD>(k)] = scale(raw[s], mpow<T>(k, r));
  }
  lds_sync<C::SY>();
#pragma unroll
  for (int sl = 0; sl < C::E; ++sl) {
    const int e = slot_elem<C::L, C::E, C::R0I>(t, sl);
    Cx<T> x = lb[lds_index<PAD>(e)];
    Cx<T> xc;
    if (e == 0) {
      x.y = T(0);
      xc = zero<T>();
    } else {
      xc = conj(lb[lds_index<PAD>(C::L - e)]);
    }
    const Cx<T> ek = x + xc;
    const Cx<T> ok = (x - xc) * conj(stw[e]);
    v[sl] = mk(ek.x - ok.y, ek.y + ok.x);
  }
}

// Line `line` of a Batch (f-major, then realisation, then line): where it
// sits in the caller's buffer (reals) and in the workspace (complex).
// With G lines per block and G dividing n^2, a block's lines never straddle
// a field, so (f, r) follow from the block index alone (scalar registers, and
// the pointer table and per-field powers are read as scalars).  The caller
// passes the block's first line for a line past the end.
template <int N, int G>
__device__ __forceinline__ void batch_line(const Batch& b, long line, int& f, int& r, long& ext_off, long& ws_off) {
  constexpr long NN = (long)N * N;
  const int fr = NN % G == 0 ? (int)(((long)blockIdx.x * G) / NN) : (int)(line / NN);  // < nf * nr
  const long l = line - (long)fr * NN;
  f = fr / b.nr;
  r = fr - f * b.nr;
  ext_off = f * b.ext_fstride + l * N;
  ws_off = f * b.ws_fstride + r * b.ws_rstride + l * (N / 2);
}

template <typename T, int N>
__global__ __launch_bounds__(256) void k_zr2c(Batch b, Cx<T>* ws, long nlines, const Cx<T>* __restrict__ tw) {
  using C = LineCfg<N>;
  __shared__ Cx<T> lds[C::G * C::SPAN];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int t = threadIdx.x % C::TPL, g = threadIdx.x / C::TPL;
  const long line = (long)blockIdx.x * C::G + g;
  const bool act = line < nlines;
  int f, r;
  long eo, wo;
  batch_line<N, C::G>(b, act ? line : (long)blockIdx.x * C::G, f, r, eo, wo);
  Cx<T>* lb = lds + g * C::SPAN;
  Cx<T> v[C::E];
  load_real_line<T, N>(static_cast<const T*>(b.ext[r]) + eo, v, t, act);
  fft<T, C::L, -1, 1, C::SY, false>(v, t, stw, 2, lb);
  r2c_finish<T, N, false>(v, t, lb, stw, ws + wo, act);
}

// field f of the batch is multiplied by m_z^zp.r[f] before the transform
template <typename T, int N>
__global__ __launch_bounds__(256) void k_zc2r(const Cx<T>* ws, Batch b, long nlines, ZPow zp,
                                              const Cx<T>* __restrict__ tw) {
  using C = LineCfg<N>;
  __shared__ Cx<T> lds[C::G * C::SPAN];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int t = threadIdx.x % C::TPL, g = threadIdx.x / C::TPL;
  const long line = (long)blockIdx.x * C::G + g;
  const bool act = line < nlines;
  int f, r;
  long eo, wo;
  batch_line<N, C::G>(b, act ? line : (long)blockIdx.x * C::G, f, r, eo, wo);
  const int rp = f < ZPOW_MAX ? zp.r[f] : 0;
  Cx<T>* lb = lds + g * C::SPAN;
  Cx<T> v[C::E], raw[C::E];
  load_cx_line<T, N>(ws + wo, raw, t);  // line 0 stands in for an inactive line
  c2r_prepare_regs<T, N, false>(raw, rp, v, t, lb, stw);
  fft<T, C::L, +1, 1, C::SY, false>(v, t, stw, 2, lb);
  Cx<T>* d2 = reinterpret_cast<Cx<T>*>(static_cast<T*>(const_cast<void*>(b.ext[r])) + eo);
  if (act) {
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) d2[slot_elem<C::L, C::E, C::RLI>(t, sl)] = v[sl];
  }
}

// S = phi_xx phi_yy + (phi_xx + phi_yy) phi_zz - phi_xy^2 - phi_xz^2 - phi_yz^2
// per real value (logical field f of the six, stored at field zp.fmap[f],
// multiplied by m_z^zp.r[f] first), then
// the forward R2C of the S line.  The field loop is not unrolled: unrolled,
// the six transforms need ~240 VGPRs (two waves per SIMD) in FP32, rolled
// ~165 (three), and measured 15% faster at n = 512.  Every load of a line is
// issued before any is used (the compiler then waits once per line, not per
// element).
template <typename T, int N>
__global__ __launch_bounds__(256) void k_zsource(const Cx<T>* __restrict__ phi, long fstride, ZPow zp,
                                                 Cx<T>* __restrict__ sk, long nlines, const Cx<T>* __restrict__ tw) {
  using C = LineCfg<N>;
  __shared__ Cx<T> lds[C::G * C::SPAN];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int t = threadIdx.x % C::TPL, g = threadIdx.x / C::TPL;
  const long line = (long)blockIdx.x * C::G + g;
  const bool act = line < nlines;
  const long lsafe = act ? line : 0;
  Cx<T>* lb = lds + g * C::SPAN;
  // FP32 loads the next field's line into raw as soon as raw has gone to
  // LDS, so it is in flight during this field's transform; FP64 loads it
  // after the transform (in flight during it, FP64 needs 256 VGPRs and ran
  // 11% slower at n = 512)
  constexpr bool PF = sizeof(T) == 4;
  Cx<T> a[C::E], s[C::E], v[C::E], raw[C::E];
  const Cx<T>* src = phi + lsafe * C::L;  // line 0 stands in for an inactive line
  auto load_field = [&](int f) {
#pragma unroll
    for (int q = 0; q < C::E; ++q) raw[q] = src[zp.fmap[f] * fstride + t + q * C::TPL];
  };
  load_field(0);
#pragma unroll 1
  for (int f = 0; f < 6; ++f) {
    const int tf = opaque_if<is_gen(C::L)>(t);
    c2r_prepare_regs<T, N>(raw, zp.r[f], v, tf, lb, stw);
    if (PF && f < 5) load_field(f + 1);
    fft<T, C::L, +1, 1, C::SY, true>(v, tf, stw, 2, lb);
    if (f == 0) {
#pragma unroll
      for (int i = 0; i < C::E; ++i) a[i] = v[i];
    } else if (f == 1) {
#pragma unroll
      for (int i = 0; i < C::E; ++i) {
        s[i] = mk(a[i].x * v[i].x, a[i].y * v[i].y);
        a[i] = a[i] + v[i];
      }
    } else if (f == 2) {
#pragma unroll
      for (int i = 0; i < C::E; ++i) s[i] = mk(s[i].x + a[i].x * v[i].x, s[i].y + a[i].y * v[i].y);
    } else {
#pragma unroll
      for (int i = 0; i < C::E; ++i) s[i] = mk(s[i].x - v[i].x * v[i].x, s[i].y - v[i].y * v[i].y);
    }
    if (!PF && f < 5) load_field(f + 1);
  }
  fft<T, C::L, -1, 1, C::SY, true>(s, t, stw, 2, lb);
  r2c_finish<T, N>(s, t, lb, stw, sk + lsafe * C::L, act);
}

// Products of the full modified-gravity source, per z line.  The input
// fields (inverse-transformed along x and y, every k factor applied) are
// transformed along z here and combined in registers into real accumulator
// lines (field k of `acc` at acc + k * afs reals):
//   KIND 0 (the diagonal pairs, weight 1) and KIND 1 (the off-diagonal
//   pairs, weight 2): per pair, NT fields a (R1), b (R2) [, c (R4)]:
//     acc0 += w a b, acc1 += w a^2 [, acc2 += 2 w a c]; KIND 0 also sums
//     the trace of a and adds its square to acc1, and writes the
//     accumulators (the first pass), KIND 1 adds to them;
//   KIND 2 (f(R) only): fields p_x, q_x, p_y, q_y, p_z, q_z, chi:
//     acc2 += sum_j p_j q_j, acc3 = chi^2.
// FP32 loads the next field's line while the current one transforms.
template <typename T, int N, int KIND, int NT>
__global__ __launch_bounds__(256) void k_zmg(const Cx<T>* __restrict__ in, long fstride, T* __restrict__ acc,
                                             long afs, long nlines, const Cx<T>* __restrict__ tw) {
  using C = LineCfg<N>;
  constexpr int NF = KIND == 2 ? 7 : 3 * NT;
  constexpr T W = KIND == 1 ? T(2) : T(1);
  __shared__ Cx<T> lds[C::G * C::SPAN];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int t = threadIdx.x % C::TPL, g = threadIdx.x / C::TPL;
  const long line = (long)blockIdx.x * C::G + g;
  const bool act = line < nlines;
  const long lsafe = act ? line : 0;
  Cx<T>* lb = lds + g * C::SPAN;
  constexpr bool PF = sizeof(T) == 4;
  Cx<T> raw[C::E], v[C::E], a[C::E], r0[C::E], r1[C::E], r2[C::E], tr[C::E];
  const Cx<T>* src = in + lsafe * C::L;  // line 0 stands in for an inactive line
  auto load_field = [&](int f) {
#pragma unroll
    for (int q = 0; q < C::E; ++q) raw[q] = src[f * fstride + t + q * C::TPL];
  };
  // accumulator k's real line as pairs, in the inverse transform's output slots
  auto acc_line = [&](int k) { return reinterpret_cast<Cx<T>*>(acc + k * afs + lsafe * N); };
#pragma unroll
  for (int i = 0; i < C::E; ++i) r0[i] = r1[i] = r2[i] = tr[i] = zero<T>();
  load_field(0);
#pragma unroll 1
  for (int f = 0; f < NF; ++f) {
    const int tf = opaque_if<true>(t);
    c2r_prepare_regs<T, N>(raw, 0, v, tf, lb, stw);
    if (PF && f < NF - 1) load_field(f + 1);
    fft<T, C::L, +1, 1, C::SY, true>(v, tf, stw, 2, lb);
    if constexpr (KIND == 2) {
      if (f == 6) {
#pragma unroll
        for (int i = 0; i < C::E; ++i) tr[i] = mk(v[i].x * v[i].x, v[i].y * v[i].y);  // chi^2
      } else if (f % 2 == 0) {
#pragma unroll
        for (int i = 0; i < C::E; ++i) a[i] = v[i];
      } else {
#pragma unroll
        for (int i = 0; i < C::E; ++i) r2[i] = mk(r2[i].x + a[i].x * v[i].x, r2[i].y + a[i].y * v[i].y);
      }
    } else {
      const int tb = f % NT;
      if (tb == 0) {
#pragma unroll
        for (int i = 0; i < C::E; ++i) {
          a[i] = v[i];
          if (KIND == 0) tr[i] = tr[i] + v[i];
        }
      } else if (tb == 1) {
#pragma unroll
        for (int i = 0; i < C::E; ++i) {
          r0[i] = mk(r0[i].x + W * a[i].x * v[i].x, r0[i].y + W * a[i].y * v[i].y);
          r1[i] = mk(r1[i].x + W * a[i].x * a[i].x, r1[i].y + W * a[i].y * a[i].y);
        }
      } else {
#pragma unroll
        for (int i = 0; i < C::E; ++i)
          r2[i] = mk(r2[i].x + T(2) * W * a[i].x * v[i].x, r2[i].y + T(2) * W * a[i].y * v[i].y);
      }
    }
    if (!PF && f < NF - 1) load_field(f + 1);
  }
  if (!act) return;
  if constexpr (KIND == 0) {
    Cx<T>* d0 = acc_line(0);
    Cx<T>* d1 = acc_line(1);
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) {
      const int e = slot_elem<C::L, C::E, C::RLI>(t, sl);
      d0[e] = r0[sl];
      d1[e] = mk(r1[sl].x + tr[sl].x * tr[sl].x, r1[sl].y + tr[sl].y * tr[sl].y);
    }
    if (NT == 3) {
      Cx<T>* d2 = acc_line(2);
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) d2[slot_elem<C::L, C::E, C::RLI>(t, sl)] = r2[sl];
    }
  } else if constexpr (KIND == 1) {
    Cx<T>* d0 = acc_line(0);
    Cx<T>* d1 = acc_line(1);
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) {
      const int e = slot_elem<C::L, C::E, C::RLI>(t, sl);
      d0[e] = d0[e] + r0[sl];
      d1[e] = d1[e] + r1[sl];
    }
    if (NT == 3) {
      Cx<T>* d2 = acc_line(2);
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) {
        const int e = slot_elem<C::L, C::E, C::RLI>(t, sl);
        d2[e] = d2[e] + r2[sl];
      }
    }
  } else {
    Cx<T>* d2 = acc_line(2);
    Cx<T>* d3 = acc_line(3);
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) {
      const int e = slot_elem<C::L, C::E, C::RLI>(t, sl);
      d2[e] = d2[e] + r2[sl];
      d3[e] = tr[sl];
    }
  }
}

// Adjoint of the source: with S_bar given per real value,
//   phi_bar_ii = S_bar (tr phi - phi_ii), phi_bar_ij = -2 S_bar phi_ij (i < j),
// each forward-transformed along z.  Logical field f of the six (xx, yy, zz,
// xy, xz, yz) is read at field zp.fmap[f], multiplied by m_z^zp.r[f] before
// its inverse transform, and its phi_bar is written at field zp.fmap[f] of
// `out` (so phi and out may be the same buffers: every line is read before
// it is written).
template <typename T, int N>
__global__ __launch_bounds__(256) void k_zprodrule(const Cx<T>* phi, long fstride, const T* __restrict__ sbar,
                                                   Cx<T>* out, long ofstride, long nlines, ZPow zp,
                                                   const Cx<T>* __restrict__ tw) {
  using C = LineCfg<N>;
  __shared__ Cx<T> lds[C::G * C::SPAN];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int t = threadIdx.x % C::TPL, g = threadIdx.x / C::TPL;
  const long line = (long)blockIdx.x * C::G + g;
  const bool act = line < nlines;
  const long lsafe = act ? line : 0;
  Cx<T>* lb = lds + g * C::SPAN;
  Cx<T> sb[C::E], d0[C::E], d1[C::E], d2[C::E], v[C::E];
  load_real_line<T, N>(sbar + lsafe * N, sb, t, true);
  const Cx<T>* src = phi + lsafe * C::L;
  load_cx_line<T, N>(src + zp.fmap[0] * fstride, v, t);
  c2r_prepare_regs<T, N>(v, zp.r[0], d0, t, lb, stw);
  fft<T, C::L, +1, 1, C::SY, true>(d0, t, stw, 2, lb);
  load_cx_line<T, N>(src + zp.fmap[1] * fstride, v, t);
  c2r_prepare_regs<T, N>(v, zp.r[1], d1, t, lb, stw);
  fft<T, C::L, +1, 1, C::SY, true>(d1, t, stw, 2, lb);
  load_cx_line<T, N>(src + zp.fmap[2] * fstride, v, t);
  c2r_prepare_regs<T, N>(v, zp.r[2], d2, t, lb, stw);
  fft<T, C::L, +1, 1, C::SY, true>(d2, t, stw, 2, lb);
  Cx<T>* dst = out + lsafe * C::L;
#pragma unroll
  for (int i = 0; i < C::E; ++i) v[i] = mk(sb[i].x * (d1[i].x + d2[i].x), sb[i].y * (d1[i].y + d2[i].y));
  fft<T, C::L, -1, 1, C::SY, true>(v, t, stw, 2, lb);
  r2c_finish<T, N>(v, t, lb, stw, dst + zp.fmap[0] * ofstride, act);
#pragma unroll
  for (int i = 0; i < C::E; ++i) v[i] = mk(sb[i].x * (d0[i].x + d2[i].x), sb[i].y * (d0[i].y + d2[i].y));
  fft<T, C::L, -1, 1, C::SY, true>(v, t, stw, 2, lb);
  r2c_finish<T, N>(v, t, lb, stw, dst + zp.fmap[1] * ofstride, act);
#pragma unroll
  for (int i = 0; i < C::E; ++i) v[i] = mk(sb[i].x * (d0[i].x + d1[i].x), sb[i].y * (d0[i].y + d1[i].y));
  fft<T, C::L, -1, 1, C::SY, true>(v, t, stw, 2, lb);
  r2c_finish<T, N>(v, t, lb, stw, dst + zp.fmap[2] * ofstride, act);
#pragma unroll 1
  for (int f = 3; f < 6; ++f) {
    Cx<T> raw[C::E];
    load_cx_line<T, N>(src + zp.fmap[f] * fstride, raw, t);
    c2r_prepare_regs<T, N>(raw, zp.r[f], v, t, lb, stw);
    fft<T, C::L, +1, 1, C::SY, true>(v, t, stw, 2, lb);
#pragma unroll
    for (int i = 0; i < C::E; ++i) v[i] = mk(T(-2) * sb[i].x * v[i].x, T(-2) * sb[i].y * v[i].y);
    fft<T, C::L, -1, 1, C::SY, true>(v, t, stw, 2, lb);
    r2c_finish<T, N>(v, t, lb, stw, dst + zp.fmap[f] * ofstride, act);
  }
}

// ---------------------------------------------------------------------------
// strided column kernels: a block takes W adjacent columns of one plane
// (lane = column fastest), so every row access is W contiguous complex.
// ---------------------------------------------------------------------------
// WW: columns per block; a block is WW * (N/E) threads.  Each (precision,
// grid size, pass kind) offers three widths for the tile tuner: half, one
// and two times the width that gives 128-byte row runs, clamped to blocks of
// 64..1024 threads and to tiles whose LDS fits in 150 KB -- two exchange
// buffers for the column FFT and x passes, one for the fused y passes (which
// keep two where they fit; at n = 768 in FP32 only one does at 128 bytes).
constexpr int col_tpc(int N) { return N / elems_per_thread(N); }
constexpr int pow2_floor(int x) { return x >= 1024 ? 1024 : x >= 512 ? 512 : x >= 256 ? 256 : x >= 128 ? 128 : x >= 64 ? 64 : x >= 32 ? 32 : x >= 16 ? 16 : x >= 8 ? 8 : x >= 4 ? 4 : x >= 2 ? 2 : 1; }
// at least one wavefront per block (tiles of several columns where one
// column has fewer than 64 threads)
template <typename T>
constexpr int col_wlo(int N) { return (64 + col_tpc(N) - 1) / col_tpc(N); }
template <typename T>
constexpr int col_whi(int N, int kind) {
  const int byblock = 1024 / col_tpc(N);
  const int bylds = pow2_floor((150 * 1024) / ((kind == KIND_MULTI ? 1 : 2) * N * (int)sizeof(Cx<T>)));
  return byblock < bylds ? byblock : bylds;
}
template <typename T>
constexpr int clampw(int N, int w, int kind) {
  return w < col_wlo<T>(N) ? col_wlo<T>(N) : (w > col_whi<T>(N, kind) ? col_whi<T>(N, kind) : w);
}
template <typename T>
constexpr int col_w(int N, int i, int kind) {
  return clampw<T>(N, i == 0 ? 64 / (int)sizeof(Cx<T>) : (i == 1 ? 128 / (int)sizeof(Cx<T>) : 256 / (int)sizeof(Cx<T>)),
                   kind);
}

template <typename T, int N, int WW>
struct ColCfg {
  static constexpr int L = N;
  static constexpr int E = elems_per_thread(L);
  static constexpr int TPC = L / E;                     // threads per column
  static constexpr int W = WW;
  static constexpr int BLOCK = W * TPC;
  static_assert(BLOCK >= 64 && BLOCK <= 1024, "block size");
  static constexpr int R0F = plan_first(L, false), RLF = plan_last(L, false);
  static constexpr int R0I = plan_first(L, true), RLI = plan_last(L, true);
  static_assert(RLF == R0I && RLI == R0F, "reversed plans");
  // the multi-transform passes keep two exchange buffers where they fit
  static constexpr bool ONE = 2 * L * W * (int)sizeof(Cx<T>) > 150 * 1024;
  // tiles of under 128 bytes per row share cache lines with their
  // neighbours: those are dealt XCD by XCD (xcd_block)
  static constexpr bool XCD = W * (int)sizeof(Cx<T>) < 128;
};

// Logical block index.  Workgroups are dealt to the 8 XCDs (each with its
// own L2) round robin, block b to XCD b % 8; this numbers them so that each
// XCD's blocks take one contiguous range, and neighbouring tiles meet in the
// same L2 (measured at n = 768, 64-byte rows: y passes 10-25% faster; with
// 128-byte rows the plain order was faster).
__device__ __forceinline__ long xcd_block(long b, long g) {
  const long q = g / 8;
  return b < 8 * q ? (b % 8) * q + b / 8 : b;
}
template <typename C>
__device__ __forceinline__ long block_index() {
  return C::XCD ? xcd_block(blockIdx.x, gridDim.x) : (long)blockIdx.x;
}

// Tile order of the persistent column passes.  Q = false: the grid-stride
// order from block_index.  Q = true: with a ticket array (q, 16 words, zero
// between launches) the workgroups fall into G = min(8, grid) groups,
// workgroup b into group b % G (the XCD it runs on, as dealt above); group x
// works through the contiguous tile range [x P, (x+1) P), P = ceil(ntiles /
// G), taking each next tile from a ticket counter.  The workgroups of one XCD
// then process neighbouring tiles at the same time; in the grid-stride order
// they drift apart within a few tiles, and tiles under 128 bytes per row
// fetch the cache lines they share with their neighbours twice (measured at
// n = 768, 64-byte rows: both x passes read 1.3-1.6x and write 1.1x their
// bytes).  The last workgroup of a group to find its range empty sets the
// group's words back to zero, so every launch starts from zero (graph
// replays included).
//
// Every thread of the block calls the members in the same order; cur and nxt
// are block-uniform (the tickets go through LDS: thread 0 asks for each one
// a tile before it reads the answer, so the atomic's latency hides behind a
// tile's work, and writes the tile to a ring slot two tiles ahead of its use;
// each tile's transforms hold block barriers between the writing and the
// reading of a slot).
template <typename C, bool Q>
struct TileOrder {
  static constexpr long END = 0x7fffffffL;
  unsigned* q;
  long ntiles, cur, nxt = END;
  int lo = 0, hi = 0, x = 0, it = 0;
  unsigned nblk = 0, pend = 0;  // thread 0: a ticket taken one tile ahead of its use
  bool out = false;             // thread 0: this workgroup's range is exhausted
  int* ring;                    // three LDS slots

  __device__ void ask() {  // thread 0: the next ticket (used a tile later, so its latency is hidden)
    if (!out) pend = atomicAdd(&q[x], 1u);
  }
  __device__ int tile_of_pend() {  // thread 0: the tile of the ticket asked for last
    if (out) return (int)END;
    const int t = lo + (int)pend;
    if (t < hi) return t;
    out = true;
    if (atomicAdd(&q[8 + x], 1u) == nblk - 1) {  // the group's last workgroup: reset for the next launch
      q[x] = 0u;
      q[8 + x] = 0u;
    }
    return (int)END;
  }
  // Q: ends with a block barrier, ntiles < 2^31
  __device__ TileOrder(unsigned* q_, long ntiles_, int* ring_) : q(q_), ntiles(ntiles_), ring(ring_) {
    if (Q && q) {
      const int g = gridDim.x < 8 ? (int)gridDim.x : 8;
      x = (int)(blockIdx.x % g);
      nblk = (gridDim.x - x + g - 1) / g;
      const int nt = (int)ntiles, per = (nt + g - 1) / g;
      lo = x < (nt + per - 1) / per ? x * per : nt;
      hi = lo < nt - per ? lo + per : nt;
      if (threadIdx.x == 0) {
        ask();
        ring[0] = tile_of_pend();
        ask();
        ring[1] = tile_of_pend();
        ask();
      }
      __syncthreads();
      cur = __builtin_amdgcn_readfirstlane(ring[0]);
      nxt = __builtin_amdgcn_readfirstlane(ring[1]);
    } else {
      cur = block_index<C>();
    }
  }
  __device__ bool valid() const { return cur < ntiles; }
  __device__ long next() const { return Q && q ? nxt : cur + gridDim.x; }
  __device__ bool has_next() const { return next() < ntiles; }
  // at the start of a tile (before its first block barrier)
  __device__ void begin() {
    if (Q && q && threadIdx.x == 0) {
      ring[(it + 2) % 3] = tile_of_pend();
      ask();
    }
  }
  // after the tile's last block barrier has been passed (a transform of one
  // stage exchanges nothing through LDS, so there the barrier is taken here)
  __device__ void advance() {
    if (Q && q) {
      if constexpr (!is_gen(C::L) && plan_stages(C::L) <= 1) __syncthreads();
      cur = nxt;
      nxt = __builtin_amdgcn_readfirstlane(ring[(it + 2) % 3]);
      ++it;
    } else {
      cur += gridDim.x;
    }
  }
};

template <typename T, int N, int WW, int D>
__global__ __launch_bounds__((ColCfg<T, N, WW>::BLOCK)) void k_colfft(Cx<T>* __restrict__ data, int ncols, int bpp,
                                                                  long plane_stride, long rowstride,
                                                                  const Cx<T>* __restrict__ tw) {
  using C = ColCfg<T, N, WW>;
  __shared__ Cx<T> lds[C::L * C::W];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int c = threadIdx.x % C::W, t = threadIdx.x / C::W;
  // (XCD-contiguous tiles at 128-byte rows make this pass 10% faster at
  // n = 512 but the x pass that reads its output 5% slower: the plain order
  // is kept there)
  const long bx = block_index<C>();
  const long plane = bx / bpp;
  const int col = (int)(bx % bpp) * C::W + c;
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
// field src[o] multiplied by m_y^pw[o], over `nplanes` x planes (the planes of
// several realisations follow each other).  Persistent over column tiles (the
// grid holds the resident blocks): the column of the next source, or of the
// next tile's first source, is loaded while the current outputs transform.
// Two LDS exchange buffers where they fit, else one (n = 768 FP32: the
// nine-output pass takes 7.3 ms with one buffer and 128-byte rows, 8.4 ms
// with two and 64-byte rows).
template <typename T, int N, int WW>
__global__ __launch_bounds__((ColCfg<T, N, WW>::BLOCK)) void k_ycombo(const Cx<T>* __restrict__ in, long fsi,
                                                                  Cx<T>* __restrict__ out, long fso, YOp op,
                                                                  long nplanes, const Cx<T>* __restrict__ tw,
                                                                  unsigned* tq) {
  using C = ColCfg<T, N, WW>;
  constexpr int M = N / 2;
  constexpr int BPP = (M + C::W - 1) / C::W;
  const long NTILES = nplanes * BPP;
  __shared__ Cx<T> lds[(C::ONE ? 1 : 2) * C::L * C::W];  // exchange buffers
  __shared__ Cx<T> stw[N];
  __shared__ int ring[3];
  stage_twiddles<T, N>(stw, tw);
  int phase = 0;
  const int c = threadIdx.x % C::W, t0 = threadIdx.x / C::W;
  // tile -> (x plane, z column); returns the element offset, act = column exists
  auto tile_off = [&](long tile, bool& act) -> long {
    const long plane = tile / BPP;
    const int col = (int)(tile % BPP) * C::W + c;
    act = col < M;
    return plane * (long)N * M + (act ? col : 0);
  };
  Cx<T> v[C::E], y[C::E], pf[C::E];
  auto load = [&](long tile, int src, int t) {
    bool a;
    const long off = tile_off(tile, a);
    const Cx<T>* b = in + src * fsi + off;
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) pf[sl] = b[slot_elem<C::L, C::E, C::R0I>(t, sl) * M];  // column 0 if missing
  };
  // tickets for tiles of 128-byte rows (n = 512 FP32: 2-4% faster; the
  // one-buffer tiles at n = 768 with the opaque index below, which keeps them
  // from spilling: 11% faster)
  TileOrder<C, !C::XCD> order(tq, NTILES, ring);
  if (order.valid()) load(order.cur, op.src[0], t0);
#pragma unroll 1
  for (; order.valid(); order.advance()) {
    order.begin();
    const long tile = order.cur;
    bool act;
    const long off = tile_off(tile, act);
#pragma unroll 1
    for (int o = 0; o < op.nout; ++o) {
      const int t = opaque_if<is_gen(C::L) || C::ONE>(t0);
      if (o == 0 || op.src[o] != op.src[o - 1]) {
#pragma unroll
        for (int sl = 0; sl < C::E; ++sl) v[sl] = pf[sl];
        int on = o + 1;
        while (on < op.nout && op.src[on] == op.src[o]) ++on;
        // always one load (after the last tile: the current column again), so
        // the compiler keeps it in flight instead of waiting at a merge
        const bool same = on < op.nout;
        const long nt = same || !order.has_next() ? tile : order.next();
        load(nt, op.src[same ? on : 0], t);
      }
      const int pw = op.pw[o];
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) {
        const int iy = slot_elem<C::L, C::E, C::R0I>(t, sl);
        y[sl] = scale(v[sl], mpow<T>(iy < N / 2 ? iy : iy - N, pw));
      }
      if constexpr (C::ONE)
        fft<T, C::L, +1, C::W, SY_BLOCK>(y, t, stw, 1, lds + c);
      else
        fft<T, C::L, +1, C::W, SY_PING>(y, t, stw, 1, lds + c, C::L * C::W, &phase);
      if (act) {
        Cx<T>* d = out + o * fso + off;
#pragma unroll
        for (int sl = 0; sl < C::E; ++sl) d[slot_elem<C::L, C::E, C::RLI>(t, sl) * M] = y[sl];
      }
    }
  }
}

// Fused y pass of the adjoint chain: output o sums its terms k (first[o] to
// first[o+1]-1), each the forward y-FFT of input field src[k] times
// m_y^py[k] m_z^pz[k] (m_z is the column's z mode, constant along it), over
// `nplanes` x planes.  Persistent over column tiles; the column of the next
// term, or of the next tile's first term, loads while the current one
// transforms.
template <typename T, int N, int WW>
__global__ __launch_bounds__((ColCfg<T, N, WW>::BLOCK)) void k_yfanin(const Cx<T>* __restrict__ in, long fsi,
                                                                  Cx<T>* __restrict__ out, long fso, YFan op,
                                                                  long nplanes, const Cx<T>* __restrict__ tw,
                                                                  unsigned* tq) {
  using C = ColCfg<T, N, WW>;
  constexpr int M = N / 2;
  constexpr int BPP = (M + C::W - 1) / C::W;
  const long NTILES = nplanes * BPP;
  __shared__ Cx<T> lds[(C::ONE ? 1 : 2) * C::L * C::W];  // exchange buffers
  __shared__ Cx<T> stw[N];
  __shared__ int ring[3];
  stage_twiddles<T, N>(stw, tw);
  int phase = 0;
  const int c = threadIdx.x % C::W, t0 = threadIdx.x / C::W;
  Cx<T> v[C::E], acc[C::E], pf[C::E];
  auto load = [&](long tile, int src, int t) {
    const long plane = tile / BPP;
    const int col = (int)(tile % BPP) * C::W + c;
    const bool a = col < M;
    const Cx<T>* b = in + src * fsi + plane * (long)N * M + (a ? col : 0);
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) pf[sl] = a ? b[slot_elem<C::L, C::E, C::R0F>(t, sl) * M] : zero<T>();
  };
  // the tile order and opaque index of the fused y pass of the displacement
  TileOrder<C, !C::XCD> order(tq, NTILES, ring);
  if (order.valid()) load(order.cur, op.src[0], t0);
#pragma unroll 1
  for (; order.valid(); order.advance()) {
    order.begin();
    const long tile = order.cur;
    const long plane = tile / BPP;
    const int col = (int)(tile % BPP) * C::W + c;
    const bool act = col < M;
    const long off = plane * (long)N * M + (act ? col : 0);
    int o = 0;
#pragma unroll 1
    for (int k = 0; k < op.nterm; ++k) {
      const int t = opaque_if<is_gen(C::L) || C::ONE>(t0);
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) v[sl] = pf[sl];
      if (k + 1 < op.nterm)
        load(tile, op.src[k + 1], t);
      else if (order.has_next())
        load(order.next(), op.src[0], t);
      if constexpr (C::ONE)
        fft<T, C::L, -1, C::W, SY_BLOCK>(v, t, stw, 1, lds + c);
      else
        fft<T, C::L, -1, C::W, SY_PING>(v, t, stw, 1, lds + c, C::L * C::W, &phase);
      const T fz = mpow<T>(col, op.pz[k]);
      const bool start = k == op.first[o];
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) {
        const int iy = slot_elem<C::L, C::E, C::RLF>(t, sl);
        const Cx<T> u = scale(v[sl], mpow<T>(iy < N / 2 ? iy : iy - N, op.py[k]) * fz);
        acc[sl] = start ? u : acc[sl] + u;
      }
      if (k + 1 == op.first[o + 1]) {
        if (act) {
          Cx<T>* d = out + o * fso + off;
#pragma unroll
          for (int sl = 0; sl < C::E; ++sl) d[slot_elem<C::L, C::E, C::RLF>(t, sl) * M] = acc[sl];
        }
        ++o;
      }
    }
  }
}

// Displacement x pass (the hot path's two x passes).  One input column X
// (z and y already forward-transformed), forward x-FFT, then one gather per
// mode of the radial table(s) (built in FP64, stored rounded once to T), then the outputs
// with their k_x powers (integer mode numbers, exact in T).  Realisation
// blockIdx.y (one after the other, in the input and in every output field);
// persistent over its column tiles; the next tile's input column loads while
// this one transforms.
//   MODE 0: tab = interleaved (PHI, PSI1) per |m|^2;
//           out 0..2: U_p = F_x^-1[-m_x^p PHI X], out 3..4: V_p = F_x^-1[i m_x^p PSI1 X]
//   MODE 1: tab = PSI2;  out 0..1: Q_p = F_x^-1[-i m_x^p PSI2 X]
//   MODE 2: tab = the (PHI, PSI1) pair; out 0..1: V_p (first order only, for
//           further epochs of the same realisation)
//   MODE 3: tab = the (PHI, PSI1) pair; out 0..2: U_p (the potential only, for
//           the adjoint)
// DC and Nyquist planes are zero in every output.  The column data are
// loaded and stored non-temporally, so the table stays in L2 for the gathers
// (measured 10% faster at n = 512).
//
// Paired gathers (where the last forward stage leaves slot s at element
// t + s L/E and a wavefront holds an even number of 16-column groups): the
// column threads are numbered so that t and L/E - t sit in neighbouring lane
// groups of one wavefront.  Their modes are each other's negatives (slot s of
// one, slot E-1-s of the other), and |m|^2 is even in m_x, so in gather k the
// second group asks for its slot E-1-k: both groups then ask for the same
// table entries and each line is fetched once for two lanes.  The second
// group reads its slots back in reverse (measured 2-6% faster at n = 512).
template <int L, int E, int RLF, int TPC, int W>
struct XPair {
  static constexpr bool ON = RLF == E && W <= 32 && 64 % W == 0 && (64 / W) % 2 == 0 && TPC % 2 == 0;
  // column thread index of lane group j, and whether it reads its slots reversed
  __device__ static int t_of(int j) {
    if (!ON) return j;
    const int p = j >> 1;
    return (j & 1) ? (p == 0 ? TPC / 2 : TPC - p) : p;
  }
  __device__ static bool rev(int j) { return ON && (j & 1); }
};

template <typename T, int N, int WW, int MODE>
__global__ __launch_bounds__((ColCfg<T, N, WW>::BLOCK)) void k_xdisp(const Cx<T>* __restrict__ in,
                                                                 Cx<T>* __restrict__ out, long fso,
                                                                 const T* __restrict__ tab,
                                                                 const Cx<T>* __restrict__ tw, int nr,
                                                                 unsigned* tq) {
  using C = ColCfg<T, N, WW>;
  constexpr int M = N / 2;
  constexpr long NCOL = (long)N * M;
  constexpr long FIELD = (long)N * NCOL;  // one realisation's half spectrum
  static_assert(!C::ONE, "x-pass widths keep two exchange buffers");
  // the two-output pass under 128-byte rows keeps one exchange buffer (two
  // barriers per exchange), so that two workgroups fit a CU, with the opaque
  // thread index that brings it to 125 VGPRs (n = 768 FP32: 2.47 -> 2.07-
  // 2.14 ms; the five-output pass, at 150 VGPRs one workgroup either way,
  // lost 15%, and n = 700 lost 13%)
  constexpr bool X1 = MODE == 1 && C::XCD && !is_gen(C::L);
  __shared__ Cx<T> lds[(X1 ? 1 : 2) * C::L * C::W];  // exchange buffers
  __shared__ Cx<T> stw[N];
  __shared__ int ring[3];
  stage_twiddles<T, N>(stw, tw);
  int phase = 0;
  using XP = XPair<C::L, C::E, C::RLF, C::TPC, C::W>;
  const int c = threadIdx.x % C::W, t0 = XP::t_of(threadIdx.x / C::W);
  const bool rev = XP::rev(threadIdx.x / C::W);
  constexpr long NTILES = (NCOL + C::W - 1) / C::W;  // per realisation
  // tickets for tiles under 128 bytes per row (n = 768 FP32, first x pass
  // 4.9 -> 4.3 ms), the realisations then flattened into one tile space
  // (tile r NTILES + j: realisation r); the grid-stride order otherwise
  // (realisation blockIdx.y)
  constexpr bool Q = C::XCD;
  Cx<T> va[C::E], y[C::E], pf[C::E];
  // radial factors per slot: MODE 0, 2 the (PHI, PSI1) pair, MODE 1 PSI2
  constexpr bool PAIR = MODE != 1;
  Cx<T> rf[PAIR ? C::E : 1];
  T rq[PAIR ? 1 : C::E];
  auto load = [&](long tile, int t) {
    const long r = Q ? tile / NTILES : blockIdx.y;
    const long col = (Q ? tile - r * NTILES : tile) * C::W + c;
    const bool a = col < NCOL;
    const Cx<T>* src = in + r * FIELD + (a ? col : 0);
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) pf[sl] = a ? ld_nt(&src[slot_elem<C::L, C::E, C::R0F>(t, sl) * NCOL]) : zero<T>();
  };
  TileOrder<C, Q> order(tq, Q ? nr * NTILES : NTILES, ring);
  if (order.valid()) load(order.cur, t0);
#pragma unroll 1
  for (; order.valid(); order.advance()) {
    order.begin();
    const int t = opaque_if<X1>(t0);
    const long tile = order.cur;
    const long r = Q ? tile / NTILES : blockIdx.y;
    const long col = (Q ? tile - r * NTILES : tile) * C::W + c;
    const bool act = col < NCOL;
    const long cs = act ? col : 0;
    const int iy = (int)(cs / M), iz = (int)(cs % M);
    const int my = iy < N / 2 ? iy : iy - N;
    const bool keep_y = iy != N / 2;
    const int n2yz = my * my + iz * iz;
    // the radial factors of the modes this thread holds after the forward
    // transform: gathered before it (latency hidden behind the transform), or
    // after it where that measured faster (the two-output FP32 pass, whose
    // early gathers compete with the next tile's prefetch)
    auto gather = [&]() {
  #pragma unroll
      for (int sl = 0; sl < C::E; ++sl) {
        const int ix = slot_elem<C::L, C::E, C::RLF>(t, rev ? C::E - 1 - sl : sl);
        const int mx = ix < N / 2 ? ix : ix - N;
        const int n2 = mx * mx + n2yz;
        const bool keep = keep_y && ix != N / 2 && n2 != 0;
        if constexpr (PAIR)
          rf[sl] = keep ? reinterpret_cast<const Cx<T>*>(tab)[n2] : zero<T>();
        else
          rq[sl] = keep ? tab[n2] : T(0);
      }
    };
    constexpr bool EARLY = PAIR || sizeof(T) == 8;
    if (EARLY) gather();
  #pragma unroll
    for (int sl = 0; sl < C::E; ++sl) va[sl] = pf[sl];
    if (order.has_next()) load(order.next(), t);  // next tile's column, in flight meanwhile
    if constexpr (X1)
      fft<T, C::L, -1, C::W, SY_BLOCK>(va, t, stw, 1, lds + c);
    else
      fft<T, C::L, -1, C::W, SY_PING>(va, t, stw, 1, lds + c, C::L * C::W, &phase);
    if (!EARLY) gather();
    constexpr int NOUT = MODE == 0 ? 5 : (MODE == 3 ? 3 : 2);
  #pragma unroll 1
    for (int o = 0; o < NOUT; ++o) {
      const int t = opaque_if<X1>(t0);
      // MODE 0: o < 3 -> -m_x^o PHI X ; o = 3, 4 -> i m_x^(o-3) PSI1 X.  MODE 1: -i m_x^o PSI2 X.
      // MODE 2: i m_x^o PSI1 X
      const bool second = (MODE == 0 && o >= 3) || MODE == 2;
      const int p = (MODE == 0 && o >= 3) ? o - 3 : o;
  #pragma unroll
      for (int sl = 0; sl < C::E; ++sl) {
        const int ix = slot_elem<C::L, C::E, C::RLF>(t, sl);
        const T f = mpow<T>(ix < N / 2 ? ix : ix - N, p);
        T r;
        if constexpr (PAIR) {
          const Cx<T> rr = rev ? rf[C::E - 1 - sl] : rf[sl];
          r = second ? rr.y : rr.x;
        } else {
          r = rev ? rq[C::E - 1 - sl] : rq[sl];
        }
        const Cx<T> a = scale(va[sl], r);
        if (PAIR)
          y[sl] = second ? mk(-a.y * f, a.x * f) : mk(-a.x * f, -a.y * f);
        else
          y[sl] = mk(a.y * f, -a.x * f);
      }
      if constexpr (X1)
        fft<T, C::L, +1, C::W, SY_BLOCK>(y, t, stw, 1, lds + c);
      else
        fft<T, C::L, +1, C::W, SY_PING>(y, t, stw, 1, lds + c, C::L * C::W, &phase);
      if (act) {
        Cx<T>* dst = out + r * FIELD + o * fso + cs;
  #pragma unroll
        for (int sl = 0; sl < C::E; ++sl) st_nt(&dst[slot_elem<C::L, C::E, C::RLI>(t, sl) * NCOL], y[sl]);
      }
    }
  }
}

// Adjoint x passes, the transposes of k_xdisp: NIN input columns (z and y
// already forward-transformed), each forward x-transformed and multiplied by
// its factor, summed, and the sum inverse x-transformed into one output.
//   MODE 0: tab = the (PHI, PSI1) pair; in 0..2: Ubar_p, factor -m_x^p PHI;
//           in 3..4: Vbar_p, factor -i m_x^p PSI1
//   MODE 1: tab = PSI2; in 0..1: Qbar_p, factor i m_x^p PSI2
// DC and Nyquist planes get no contribution.  Persistent over column tiles;
// the next input's column (or the next tile's first) loads while the
// current one transforms.
template <typename T, int N, int WW, int MODE>
__global__ __launch_bounds__((ColCfg<T, N, WW>::BLOCK)) void k_xadj(const Cx<T>* __restrict__ in, long fsi,
                                                                Cx<T>* __restrict__ out,
                                                                const T* __restrict__ tab,
                                                                const Cx<T>* __restrict__ tw, unsigned* tq) {
  using C = ColCfg<T, N, WW>;
  constexpr int M = N / 2;
  constexpr long NCOL = (long)N * M;
  constexpr int NIN = MODE == 0 ? 5 : 2;
  constexpr bool PAIR = MODE == 0;
  static_assert(!C::ONE, "x-pass widths keep two exchange buffers");
  __shared__ Cx<T> lds[2 * C::L * C::W];  // two exchange buffers
  __shared__ Cx<T> stw[N];
  __shared__ int ring[3];
  stage_twiddles<T, N>(stw, tw);
  int phase = 0;
  using XP = XPair<C::L, C::E, C::RLF, C::TPC, C::W>;  // paired gathers, as in k_xdisp
  const int c = threadIdx.x % C::W, t = XP::t_of(threadIdx.x / C::W);
  const bool rev = XP::rev(threadIdx.x / C::W);
  constexpr long NTILES = (NCOL + C::W - 1) / C::W;
  Cx<T> v[C::E], acc[C::E], pf[C::E];
  Cx<T> rf[PAIR ? C::E : 1];
  T rq[PAIR ? 1 : C::E];
  auto load = [&](long tile, int k) {
    const long col = tile * C::W + c;
    const bool a = col < NCOL;
    const long cs = a ? col : 0;
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl)
      pf[sl] = a ? ld_nt(&in[k * fsi + cs + slot_elem<C::L, C::E, C::R0F>(t, sl) * NCOL]) : zero<T>();
  };
  // the tile order of the displacement x pass
  TileOrder<C, C::XCD> order(tq, NTILES, ring);
  if (order.valid()) load(order.cur, 0);
#pragma unroll 1
  for (; order.valid(); order.advance()) {
    order.begin();
    const long tile = order.cur;
    const long col = tile * C::W + c;
    const bool act = col < NCOL;
    const long cs = act ? col : 0;
    const int iy = (int)(cs / M), iz = (int)(cs % M);
    const int my = iy < N / 2 ? iy : iy - N;
    const bool keep_y = iy != N / 2;
    const int n2yz = my * my + iz * iz;
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) {
      const int ix = slot_elem<C::L, C::E, C::RLF>(t, rev ? C::E - 1 - sl : sl);
      const int mx = ix < N / 2 ? ix : ix - N;
      const int n2 = mx * mx + n2yz;
      const bool keep = keep_y && ix != N / 2 && n2 != 0;
      if constexpr (PAIR)
        rf[sl] = keep ? reinterpret_cast<const Cx<T>*>(tab)[n2] : zero<T>();
      else
        rq[sl] = keep ? tab[n2] : T(0);
    }
#pragma unroll 1
    for (int k = 0; k < NIN; ++k) {
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) v[sl] = pf[sl];
      if (k + 1 < NIN)
        load(tile, k + 1);
      else if (order.has_next())
        load(order.next(), 0);
      fft<T, C::L, -1, C::W, SY_PING>(v, t, stw, 1, lds + c, C::L * C::W, &phase);
      const bool second = PAIR && k >= 3;
      const int pw = second ? k - 3 : k;
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) {
        const int ix = slot_elem<C::L, C::E, C::RLF>(t, sl);
        T r;
        if constexpr (PAIR) {
          const Cx<T> rr = rev ? rf[C::E - 1 - sl] : rf[sl];
          r = second ? rr.y : rr.x;
        } else {
          r = rev ? rq[C::E - 1 - sl] : rq[sl];
        }
        const T f = mpow<T>(ix < N / 2 ? ix : ix - N, pw) * r;
        // MODE 0: -f v (U) or -i f v (V); MODE 1: i f v
        const Cx<T> u = PAIR ? (second ? mk(v[sl].y * f, -v[sl].x * f) : mk(-v[sl].x * f, -v[sl].y * f))
                             : mk(-v[sl].y * f, v[sl].x * f);
        acc[sl] = k == 0 ? u : acc[sl] + u;
      }
    }
    fft<T, C::L, +1, C::W, SY_PING>(acc, t, stw, 1, lds + c, C::L * C::W, &phase);
    if (act) {
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) st_nt(&out[cs + slot_elem<C::L, C::E, C::RLI>(t, sl) * NCOL], acc[sl]);
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

template <typename T, int N, int WW>
__global__ __launch_bounds__((ColCfg<T, N, WW>::BLOCK)) void k_xpass(const Cx<T>* __restrict__ in, long fsi,
                                                                 Cx<T>* __restrict__ out, long fso, XOp op,
                                                                 const Cx<T>* __restrict__ tw) {
  using C = ColCfg<T, N, WW>;
  constexpr int M = N / 2;
  constexpr long NCOL = (long)N * M;
  __shared__ Cx<T> lds[C::L * C::W];
  __shared__ Cx<T> stw[N];
  stage_twiddles<T, N>(stw, tw);
  const int c = threadIdx.x % C::W, t0 = threadIdx.x / C::W;
  const long col = block_index<C>() * C::W + c;
  const bool act = col < NCOL;
  const long cs = act ? col : 0;
  const int iy = (int)(cs / M), iz = (int)(cs % M);
  const int my = iy < N / 2 ? iy : iy - N;
  const bool keep_y = iy != N / 2;
  const long n2yz = (long)my * my + (long)iz * iz;
  Cx<T> v[C::E], y[C::E];
  if (op.nin == 1) {
    const int t = t0;
#pragma unroll
    for (int sl = 0; sl < C::E; ++sl) v[sl] = act ? in[cs + slot_elem<C::L, C::E, C::R0F>(t, sl) * NCOL] : zero<T>();
    fft<T, C::L, -1, C::W>(v, t, stw, 1, lds + c);
#pragma unroll 1
    for (int o = 0; o < op.nout; ++o) {
      const int t = opaque_if<true>(t0);
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) {
        const int ix = slot_elem<C::L, C::E, C::RLF>(t, sl);
        const int mx = ix < N / 2 ? ix : ix - N;
        const long n2 = (long)mx * mx + n2yz;
        y[sl] = xop_mul<T>(op, o, mx, my, iz, n2, keep_y && ix != N / 2 && n2 != 0) * v[sl];
      }
      Cx<T>* dst = out + o * fso + cs;
      if (op.inverse) {
        fft<T, C::L, +1, C::W>(y, t, stw, 1, lds + c);
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
      const int t = opaque_if<true>(t0);
      const Cx<T>* src = in + f * fsi + cs;
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) v[sl] = act ? src[slot_elem<C::L, C::E, C::R0F>(t, sl) * NCOL] : zero<T>();
      fft<T, C::L, -1, C::W>(v, t, stw, 1, lds + c);
#pragma unroll
      for (int sl = 0; sl < C::E; ++sl) {
        const int ix = slot_elem<C::L, C::E, C::RLF>(t, sl);
        const int mx = ix < N / 2 ? ix : ix - N;
        const long n2 = (long)mx * mx + n2yz;
        y[sl] = y[sl] + xop_mul<T>(op, f, mx, my, iz, n2, keep_y && ix != N / 2 && n2 != 0) * v[sl];
      }
    }
    Cx<T>* dst = out + cs;
    const int t = t0;
    if (op.inverse) {
      fft<T, C::L, +1, C::W>(y, t, stw, 1, lds + c);
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

// Blocks of a persistent kernel that can be resident at once (occupancy of
// this kernel x compute units); the grid is this, at most one per tile.
static long resident_blocks(const void* kernel, int block) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return 1L << 30;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, 0) != hipSuccess || per < 1) per = 1;
  return (long)per * cus;
}

static inline long min_l(long a, long b) { return a < b ? a : b; }

// The ticket array for a persistent launch of `blocks` workgroups over
// `ntiles` tiles, or none (the grid-stride order) where a workgroup would
// take fewer than 8 tiles: there the tickets taken before the first tile
// cost more than the order gains (n = 128: fan-in y pass 12 -> 30 us).
static inline unsigned* tickets_for(unsigned* tq, long ntiles, long blocks) {
  return ntiles >= 8 * blocks ? tq : nullptr;
}

template <typename T, int N>
hipError_t zr2c_t(const Batch& b, void* ws, const void* tw, hipStream_t s) {
  using C = LineCfg<N>;
  const long nlines = (long)b.nf * b.nr * N * N;
  const long blocks = (nlines + C::G - 1) / C::G;
  hipLaunchKernelGGL((k_zr2c<T, N>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, b, (Cx<T>*)ws, nlines,
                     (const Cx<T>*)tw);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t zc2r_t(const void* ws, const Batch& b, const ZPow& zp, const void* tw, hipStream_t s) {
  using C = LineCfg<N>;
  const long nlines = (long)b.nf * b.nr * N * N;
  const long blocks = (nlines + C::G - 1) / C::G;
  hipLaunchKernelGGL((k_zc2r<T, N>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const Cx<T>*)ws, b, nlines, zp,
                     (const Cx<T>*)tw);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t zsource_t(const void* phi, long fstride, const ZPow& zp, void* sk, long nlines, const void* tw,
                            hipStream_t s) {
  using C = LineCfg<N>;
  const long blocks = (nlines + C::G - 1) / C::G;
  hipLaunchKernelGGL((k_zsource<T, N>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const Cx<T>*)phi, fstride, zp,
                     (Cx<T>*)sk, nlines, (const Cx<T>*)tw);
  return hipGetLastError();
}

template <typename T, int N, int KIND, int NT>
hipError_t zmg_t(const void* in, long fstride, void* acc, long afs, long nlines, const void* tw, hipStream_t s) {
  using C = LineCfg<N>;
  const long blocks = (nlines + C::G - 1) / C::G;
  hipLaunchKernelGGL((k_zmg<T, N, KIND, NT>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const Cx<T>*)in, fstride,
                     (T*)acc, afs, nlines, (const Cx<T>*)tw);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t zmg_k(int kind, int nt, const void* in, long fstride, void* acc, long afs, long nlines,
                        const void* tw, hipStream_t s) {
  if (kind == 0) return nt == 3 ? zmg_t<T, N, 0, 3>(in, fstride, acc, afs, nlines, tw, s) : zmg_t<T, N, 0, 2>(in, fstride, acc, afs, nlines, tw, s);
  if (kind == 1) return nt == 3 ? zmg_t<T, N, 1, 3>(in, fstride, acc, afs, nlines, tw, s) : zmg_t<T, N, 1, 2>(in, fstride, acc, afs, nlines, tw, s);
  return zmg_t<T, N, 2, 3>(in, fstride, acc, afs, nlines, tw, s);
}

template <typename T, int N>
hipError_t zprod_t(const void* phi, long fstride, const void* sbar, void* out, long ofs, long nlines,
                          const ZPow& zp, const void* tw, hipStream_t s) {
  using C = LineCfg<N>;
  const long blocks = (nlines + C::G - 1) / C::G;
  hipLaunchKernelGGL((k_zprodrule<T, N>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const Cx<T>*)phi, fstride,
                     (const T*)sbar, (Cx<T>*)out, ofs, nlines, zp, (const Cx<T>*)tw);
  return hipGetLastError();
}

template <typename T, int N, int WW>
hipError_t colfft_w(int dir, void* data, long nplanes, long plane_stride, int ncols, long rowstride,
                           const void* tw, hipStream_t s) {
  using C = ColCfg<T, N, WW>;
  const int bpp = (ncols + C::W - 1) / C::W;
  const long blocks = nplanes * bpp;
  if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
  if (dir < 0)
    hipLaunchKernelGGL((k_colfft<T, N, WW, -1>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (Cx<T>*)data, ncols,
                       bpp, plane_stride, rowstride, (const Cx<T>*)tw);
  else
    hipLaunchKernelGGL((k_colfft<T, N, WW, +1>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (Cx<T>*)data, ncols,
                       bpp, plane_stride, rowstride, (const Cx<T>*)tw);
  return hipGetLastError();
}

template <typename T, int N>
hipError_t colfft_t(int w, int dir, void* data, long nplanes, long plane_stride, int ncols, long rowstride,
                           const void* tw, hipStream_t s) {
  constexpr int K = KIND_COL;
  if (w == col_w<T>(N, 0, K)) return colfft_w<T, N, col_w<T>(N, 0, K)>(dir, data, nplanes, plane_stride, ncols, rowstride, tw, s);
  if (w == col_w<T>(N, 1, K)) return colfft_w<T, N, col_w<T>(N, 1, K)>(dir, data, nplanes, plane_stride, ncols, rowstride, tw, s);
  if (w == col_w<T>(N, 2, K)) return colfft_w<T, N, col_w<T>(N, 2, K)>(dir, data, nplanes, plane_stride, ncols, rowstride, tw, s);
  return hipErrorInvalidValue;
}

template <typename T, int N, int WW>
hipError_t ycombo_w(int nr, const void* in, long fsi, void* out, long fso, const YOp& op, const void* tw,
                           hipStream_t s, unsigned* tq) {
  using C = ColCfg<T, N, WW>;
  constexpr int M = N / 2;
  static const long res = resident_blocks(reinterpret_cast<const void*>(&k_ycombo<T, N, WW>), C::BLOCK);
  const long nplanes = (long)nr * N;
  const long ntiles = nplanes * ((M + C::W - 1) / C::W);
  const long blocks = min_l(res, ntiles);
  hipLaunchKernelGGL((k_ycombo<T, N, WW>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const Cx<T>*)in, fsi,
                     (Cx<T>*)out, fso, op, nplanes, (const Cx<T>*)tw, tickets_for(tq, ntiles, blocks));
  return hipGetLastError();
}

template <typename T, int N>
hipError_t ycombo_t(int w, int nr, const void* in, long fsi, void* out, long fso, const YOp& op, const void* tw,
                           hipStream_t s, unsigned* tq) {
  constexpr int K = KIND_MULTI;
  if (w == col_w<T>(N, 0, K)) return ycombo_w<T, N, col_w<T>(N, 0, K)>(nr, in, fsi, out, fso, op, tw, s, tq);
  if (w == col_w<T>(N, 1, K)) return ycombo_w<T, N, col_w<T>(N, 1, K)>(nr, in, fsi, out, fso, op, tw, s, tq);
  if (w == col_w<T>(N, 2, K)) return ycombo_w<T, N, col_w<T>(N, 2, K)>(nr, in, fsi, out, fso, op, tw, s, tq);
  return hipErrorInvalidValue;
}

template <typename T, int N, int WW>
hipError_t yfanin_w(int nr, const void* in, long fsi, void* out, long fso, const YFan& op, const void* tw,
                           hipStream_t s, unsigned* tq) {
  using C = ColCfg<T, N, WW>;
  constexpr int M = N / 2;
  static const long res = resident_blocks(reinterpret_cast<const void*>(&k_yfanin<T, N, WW>), C::BLOCK);
  const long nplanes = (long)nr * N;
  const long ntiles = nplanes * ((M + C::W - 1) / C::W);
  const long blocks = min_l(res, ntiles);
  hipLaunchKernelGGL((k_yfanin<T, N, WW>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const Cx<T>*)in, fsi,
                     (Cx<T>*)out, fso, op, nplanes, (const Cx<T>*)tw, tickets_for(tq, ntiles, blocks));
  return hipGetLastError();
}

template <typename T, int N>
hipError_t yfanin_t(int w, int nr, const void* in, long fsi, void* out, long fso, const YFan& op, const void* tw,
                           hipStream_t s, unsigned* tq) {
  constexpr int K = KIND_MULTI;
  if (w == col_w<T>(N, 0, K)) return yfanin_w<T, N, col_w<T>(N, 0, K)>(nr, in, fsi, out, fso, op, tw, s, tq);
  if (w == col_w<T>(N, 1, K)) return yfanin_w<T, N, col_w<T>(N, 1, K)>(nr, in, fsi, out, fso, op, tw, s, tq);
  if (w == col_w<T>(N, 2, K)) return yfanin_w<T, N, col_w<T>(N, 2, K)>(nr, in, fsi, out, fso, op, tw, s, tq);
  return hipErrorInvalidValue;
}

template <typename T, int N, int WW, int MODE>
hipError_t xdisp_m(int nr, const void* in, void* out, long fso, const void* tab, const void* tw,
                          hipStream_t s, unsigned* tq) {
  using C = ColCfg<T, N, WW>;
  const long ntiles = ((long)N * (N / 2) + C::W - 1) / C::W;  // per realisation
  static const long res = resident_blocks(reinterpret_cast<const void*>(&k_xdisp<T, N, WW, MODE>), C::BLOCK);
  // ticket order (rows under 128 bytes): one tile space over the
  // realisations; else the resident blocks shared out over them (grid.y)
  const dim3 grid = C::XCD ? dim3((unsigned)min_l(res, nr * ntiles), 1)
                           : dim3((unsigned)min_l((res + nr - 1) / nr, ntiles), (unsigned)nr);
  hipLaunchKernelGGL((k_xdisp<T, N, WW, MODE>), grid, dim3(C::BLOCK), 0, s, (const Cx<T>*)in, (Cx<T>*)out, fso,
                     (const T*)tab, (const Cx<T>*)tw, nr, tickets_for(tq, nr * ntiles, grid.x));
  return hipGetLastError();
}

template <typename T, int N, int WW>
hipError_t xdisp_w(int nr, int mode, const void* in, void* out, long fso, const void* tab, const void* tw,
                          hipStream_t s, unsigned* tq) {
  switch (mode) {
    case 0: return xdisp_m<T, N, WW, 0>(nr, in, out, fso, tab, tw, s, tq);
    case 1: return xdisp_m<T, N, WW, 1>(nr, in, out, fso, tab, tw, s, tq);
    case 2: return xdisp_m<T, N, WW, 2>(nr, in, out, fso, tab, tw, s, tq);
    case 3: return xdisp_m<T, N, WW, 3>(nr, in, out, fso, tab, tw, s, tq);
  }
  return hipErrorInvalidValue;
}

template <typename T, int N>
hipError_t xdisp_t(int w, int nr, int mode, const void* in, void* out, long fso, const void* tab,
                          const void* tw, hipStream_t s, unsigned* tq) {
  constexpr int K = KIND_X;
  if (w == col_w<T>(N, 0, K)) return xdisp_w<T, N, col_w<T>(N, 0, K)>(nr, mode, in, out, fso, tab, tw, s, tq);
  if (w == col_w<T>(N, 1, K)) return xdisp_w<T, N, col_w<T>(N, 1, K)>(nr, mode, in, out, fso, tab, tw, s, tq);
  if (w == col_w<T>(N, 2, K)) return xdisp_w<T, N, col_w<T>(N, 2, K)>(nr, mode, in, out, fso, tab, tw, s, tq);
  return hipErrorInvalidValue;
}

template <typename T, int N, int WW, int MODE>
hipError_t xadj_m(const void* in, long fsi, void* out, const void* tab, const void* tw, hipStream_t s, unsigned* tq) {
  using C = ColCfg<T, N, WW>;
  const long ntiles = ((long)N * (N / 2) + C::W - 1) / C::W;
  static const long res = resident_blocks(reinterpret_cast<const void*>(&k_xadj<T, N, WW, MODE>), C::BLOCK);
  const long blocks = min_l(res, ntiles);
  hipLaunchKernelGGL((k_xadj<T, N, WW, MODE>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const Cx<T>*)in, fsi,
                     (Cx<T>*)out, (const T*)tab, (const Cx<T>*)tw, tickets_for(tq, ntiles, blocks));
  return hipGetLastError();
}

template <typename T, int N, int WW>
hipError_t xadj_w(int mode, const void* in, long fsi, void* out, const void* tab, const void* tw,
                         hipStream_t s, unsigned* tq) {
  return mode == 0 ? xadj_m<T, N, WW, 0>(in, fsi, out, tab, tw, s, tq) : xadj_m<T, N, WW, 1>(in, fsi, out, tab, tw, s, tq);
}

template <typename T, int N>
hipError_t xadj_t(int w, int mode, const void* in, long fsi, void* out, const void* tab, const void* tw,
                         hipStream_t s, unsigned* tq) {
  constexpr int K = KIND_X;
  if (w == col_w<T>(N, 0, K)) return xadj_w<T, N, col_w<T>(N, 0, K)>(mode, in, fsi, out, tab, tw, s, tq);
  if (w == col_w<T>(N, 1, K)) return xadj_w<T, N, col_w<T>(N, 1, K)>(mode, in, fsi, out, tab, tw, s, tq);
  if (w == col_w<T>(N, 2, K)) return xadj_w<T, N, col_w<T>(N, 2, K)>(mode, in, fsi, out, tab, tw, s, tq);
  return hipErrorInvalidValue;
}

template <typename T, int N>
hipError_t xpass_t(const void* in, long fsi, void* out, long fso, const XOp& op, const void* tw,
                          hipStream_t s) {
  constexpr int WW = col_w<T>(N, 1, KIND_X);
  using C = ColCfg<T, N, WW>;
  const long ncol = (long)N * (N / 2);
  const long blocks = (ncol + C::W - 1) / C::W;
  hipLaunchKernelGGL((k_xpass<T, N, WW>), dim3((unsigned)blocks), dim3(C::BLOCK), 0, s, (const Cx<T>*)in, fsi,
                     (Cx<T>*)out, fso, op, (const Cx<T>*)tw);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// grid sizes and the per-size launchers
// ---------------------------------------------------------------------------
// Supported grid sizes n: powers of two 8..512, three times a power of two
// 24..768, and the sizes with a factor 5 or 7 (40, 56, 200, 400, 600, 700).
#define LPT2_GRID_SIZES(X) \
  X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(24) X(48) X(96) X(192) X(384) X(768) \
  X(40) X(56) X(200) X(400) X(600) X(700)

// The per-size launchers of one precision and size.  Each is instantiated in
// one of the size translation units (compiled in parallel) and declared
// extern where the public launchers dispatch on n.
#define LPT2_PASSES(PREFIX, T, N)                                                                              \
  PREFIX hipError_t zr2c_t<T, N>(const Batch&, void*, const void*, hipStream_t);                              \
  PREFIX hipError_t zc2r_t<T, N>(const void*, const Batch&, const ZPow&, const void*, hipStream_t);           \
  PREFIX hipError_t zsource_t<T, N>(const void*, long, const ZPow&, void*, long, const void*, hipStream_t);   \
  PREFIX hipError_t zmg_k<T, N>(int, int, const void*, long, void*, long, long, const void*, hipStream_t);    \
  PREFIX hipError_t zprod_t<T, N>(const void*, long, const void*, void*, long, long, const ZPow&, const void*, \
                                  hipStream_t);                                                                \
  PREFIX hipError_t colfft_t<T, N>(int, int, void*, long, long, int, long, const void*, hipStream_t);          \
  PREFIX hipError_t ycombo_t<T, N>(int, int, const void*, long, void*, long, const YOp&, const void*,          \
                                   hipStream_t, unsigned*);                                                    \
  PREFIX hipError_t yfanin_t<T, N>(int, int, const void*, long, void*, long, const YFan&, const void*,         \
                                   hipStream_t, unsigned*);                                                    \
  PREFIX hipError_t xdisp_t<T, N>(int, int, int, const void*, void*, long, const void*, const void*,          \
                                  hipStream_t, unsigned*);                                                     \
  PREFIX hipError_t xadj_t<T, N>(int, int, const void*, long, void*, const void*, const void*, hipStream_t,    \
                                 unsigned*);                                                                   \
  PREFIX hipError_t xpass_t<T, N>(const void*, long, void*, long, const XOp&, const void*, hipStream_t);
#define LPT2_DECLARE_SIZE(N) LPT2_PASSES(extern template, float, N) LPT2_PASSES(extern template, double, N)
#define LPT2_INSTANTIATE_SIZE(N) LPT2_PASSES(template, float, N) LPT2_PASSES(template, double, N)

}  // namespace lpt2

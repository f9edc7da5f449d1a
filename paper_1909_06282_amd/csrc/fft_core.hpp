// Register/LDS Stockham FFT engine shared by the axis-pass kernels.
//
// One transform of length L (a power of two, 4..512) is carried by L/E
// threads, each holding E complex values in registers.  A stage of radix R
// (R in {4, 8}, R divides E) runs E/R butterflies per thread; between stages
// the values go through LDS once (write in the stage's output order, read in
// the next stage's input order).  The Stockham ordering needs no bit
// reversal: after the last stage thread t holds, in slot u*R+q, element
// t + u*(L/E) + q*(L/R) of the natural-order result.  The same formula with
// the first stage's radix gives the element a thread must supply in each
// slot before the first stage, so a forward transform whose last radix
// equals the next inverse transform's first radix can hand its registers
// straight over (the inverse plan is the forward plan reversed).
//
// Twiddles come from a table tw[m] = exp(-2 pi i m / Ntab) built in FP64 on
// the host (rounded once for FP32); a transform of length L reads every
// (Ntab/L)-th entry.  The butterflies are unnormalised: forward uses
// exp(-2 pi i ...), inverse exp(+2 pi i ...), no 1/L.
#pragma once
#include "cx.hpp"

namespace lpt2 {

// ---- radix plans -----------------------------------------------------------
constexpr int plan_stages(int L) {
  return L == 4 ? 1 : L == 8 ? 1 : L == 16 ? 2 : L == 32 ? 2 : L == 64 ? 2 : L == 128 ? 3 : L == 256 ? 3 : 3;
}
// radix of forward stage s (0-based)
constexpr int plan_radix_fwd(int L, int s) {
  return L == 4     ? (s == 0 ? 4 : 0)
         : L == 8   ? (s == 0 ? 8 : 0)
         : L == 16  ? (s < 2 ? 4 : 0)
         : L == 32  ? (s == 0 ? 8 : s == 1 ? 4 : 0)
         : L == 64  ? (s < 2 ? 8 : 0)
         : L == 128 ? (s == 0 ? 8 : s < 3 ? 4 : 0)
         : L == 256 ? (s < 2 ? 8 : s == 2 ? 4 : 0)
                    : (s < 3 ? 8 : 0);
}
constexpr int plan_radix(int L, int s, bool inv) {
  return s >= plan_stages(L) ? 0 : (inv ? plan_radix_fwd(L, plan_stages(L) - 1 - s) : plan_radix_fwd(L, s));
}
constexpr int plan_first(int L, bool inv) { return plan_radix(L, 0, inv); }
constexpr int plan_last(int L, bool inv) { return plan_radix(L, plan_stages(L) - 1, inv); }
// elements per thread: 8, except the single radix-4 length
constexpr int elems_per_thread(int L) { return L == 4 ? 4 : 8; }

// Element index held in `slot` of thread t for a pattern of radix R.
template <int L, int E, int R>
__device__ __forceinline__ int slot_elem(int t, int slot) {
  return t + (slot / R) * (L / E) + (slot % R) * (L / R);
}

// ---- butterflies (in place, natural order in and out) -----------------------
template <int D, typename T>
__device__ __forceinline__ void dft4(Cx<T>& x0, Cx<T>& x1, Cx<T>& x2, Cx<T>& x3) {
  const Cx<T> t0 = x0 + x2, t1 = x0 - x2, t2 = x1 + x3;
  const Cx<T> t3 = mul_si<D>(x1 - x3);
  x0 = t0 + t2;
  x2 = t0 - t2;
  x1 = t1 + t3;
  x3 = t1 - t3;
}

template <int D, typename T>
__device__ __forceinline__ void dft8(Cx<T>* x) {
  Cx<T> e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  Cx<T> o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4<D>(e0, e1, e2, e3);
  dft4<D>(o0, o1, o2, o3);
  const T h = T(0.70710678118654752440084436210484903928483593768847);
  // w = exp(D 2 pi i / 8)
  const Cx<T> w1o = mk((o1.x - T(D) * o1.y) * h, (o1.y + T(D) * o1.x) * h);
  const Cx<T> w2o = mul_si<D>(o2);
  const Cx<T> w3o = mk((-o3.x - T(D) * o3.y) * h, (-o3.y + T(D) * o3.x) * h);
  x[0] = e0 + o0;
  x[4] = e0 - o0;
  x[1] = e1 + w1o;
  x[5] = e1 - w1o;
  x[2] = e2 + w2o;
  x[6] = e2 - w2o;
  x[3] = e3 + w3o;
  x[7] = e3 - w3o;
}

template <int R, int D, typename T>
__device__ __forceinline__ void butterfly(Cx<T>* x) {
  if constexpr (R == 8) {
    dft8<D>(x);
  } else {
    static_assert(R == 4, "radix 4 or 8");
    dft4<D>(x[0], x[1], x[2], x[3]);
  }
}

// ---- one stage in registers ---------------------------------------------------
// Butterfly b = t + u*(L/E) reads elements b + j*(L/R); with k = b mod NS the
// inputs are twiddled by exp(D 2 pi i k j / (NS R)).
template <typename T, int L, int E, int R, int NS, int D>
__device__ __forceinline__ void stage(Cx<T>* v, int t, const Cx<T>* __restrict__ tw, int tws) {
  constexpr int TP = L / E;
#pragma unroll
  for (int u = 0; u < E / R; ++u) {
    Cx<T>* x = v + u * R;
    if constexpr (NS > 1) {
      const int b = t + u * TP;
      const int k = b & (NS - 1);
      const int step = k * (L / (NS * R)) * tws;
#pragma unroll
      for (int j = 1; j < R; ++j) {
        Cx<T> w = tw[step * j];
        if (D > 0) w.y = -w.y;
        x[j] = x[j] * w;
      }
    }
    butterfly<R, D>(x);
  }
}

// ---- LDS exchange between stages ------------------------------------------------
// lb points at element 0 of this thread's transform; element e lives at
// lb[lds_index<PAD>(e) * ES].  PAD inserts one spare slot after every 8
// elements, which makes the stride-8 write of a first radix-8 stage
// bank-conflict free when one transform's threads sit in adjacent lanes.
//
// Synchronisation (SY):
//   SY_BLOCK: a transform spans several wavefronts; a workgroup barrier
//             before the writes (protects the previous reads) and after them;
//   SY_WAVE:  a transform lies inside one wavefront; LDS operations of a
//             wavefront complete in order, so only the compiler must be kept
//             from moving loads and stores across the exchange;
//   SY_PING:  as SY_BLOCK but alternating between two LDS buffers (`phase`
//             counts exchanges), so the barrier before the writes is not needed.
enum { SY_BLOCK = 0, SY_WAVE = 1, SY_PING = 2 };

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int SY>
__device__ __forceinline__ void lds_sync() {
  if constexpr (SY == SY_WAVE)
    wave_sync();
  else
    __syncthreads();
}

template <bool PAD>
__device__ __forceinline__ int lds_index(int e) {
  return PAD ? e + (e >> 3) : e;
}
// LDS slots needed by one transform of length L
template <bool PAD>
constexpr int lds_span(int L) { return PAD ? L + L / 8 : L; }

template <typename T, int L, int E, int ROUT, int NSOUT, int RIN, int ES, int SY, bool PAD>
__device__ __forceinline__ void exchange(Cx<T>* v, int t, Cx<T>* lb, int pingstride, int& phase) {
  constexpr int TP = L / E;
  if constexpr (SY == SY_PING) {
    lb += (phase & 1) * pingstride;
    ++phase;
  } else {
    lds_sync<SY>();
  }
#pragma unroll
  for (int u = 0; u < E / ROUT; ++u) {
    const int b = t + u * TP;
    const int k = b & (NSOUT - 1);
    const int base = (b - k) * ROUT + k;
#pragma unroll
    for (int q = 0; q < ROUT; ++q) lb[lds_index<PAD>(base + q * NSOUT) * ES] = v[u * ROUT + q];
  }
  lds_sync<SY>();
#pragma unroll
  for (int u = 0; u < E / RIN; ++u)
#pragma unroll
    for (int j = 0; j < RIN; ++j) v[u * RIN + j] = lb[lds_index<PAD>(t + u * TP + j * (L / RIN)) * ES];
}

// ---- full transform -----------------------------------------------------------
// In: slots in the first-stage pattern of the direction's plan.
// Out: slots in the last-stage pattern.  D = -1 forward, +1 inverse.
// For SY_PING, lb + pingstride is the second buffer and `phase` persists
// across the transforms of a kernel.
template <typename T, int L, int D, int ES, int SY = SY_BLOCK, bool PAD = false, int E = elems_per_thread(L)>
__device__ __forceinline__ void fft(Cx<T>* v, int t, const Cx<T>* __restrict__ tw, int tws, Cx<T>* lb,
                                    int pingstride = 0, int* phase = nullptr) {
  constexpr bool INV = D > 0;
  static_assert(E % plan_radix(L, 0, INV) == 0 && L % E == 0, "E must be a multiple of every radix");
  constexpr int NST = plan_stages(L);
  constexpr int R0 = plan_radix(L, 0, INV);
  constexpr int R1 = plan_radix(L, 1, INV);
  constexpr int R2 = plan_radix(L, 2, INV);
  int dummy = 0;
  int& ph = phase ? *phase : dummy;
  stage<T, L, E, R0, 1, D>(v, t, tw, tws);
  if constexpr (NST > 1) {
    exchange<T, L, E, R0, 1, R1, ES, SY, PAD>(v, t, lb, pingstride, ph);
    stage<T, L, E, R1, R0, D>(v, t, tw, tws);
  }
  if constexpr (NST > 2) {
    exchange<T, L, E, R1, R0, R2, ES, SY, PAD>(v, t, lb, pingstride, ph);
    stage<T, L, E, R2, R0 * R1, D>(v, t, tw, tws);
  }
}

}  // namespace lpt2

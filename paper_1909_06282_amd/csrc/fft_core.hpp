// Register/LDS Stockham FFT engine shared by the axis-pass kernels.
//
// One transform of length L (a power of two, 4..512, three times one,
// 12..768, or a length of the table of lengths with a factor 5 or 7) is
// carried by L/E threads, each holding E complex values in
// registers.  A stage of radix R (R in {2, 4, 8, 12}, R divides E) runs E/R
// butterflies per thread; between stages
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
// Lengths 2^k (4..512): radix-8/4 stages, 8 values per thread.
// Lengths 3 * 2^k (12..768): one radix-12 stage first (3 x 4 in registers),
// then radix 4 (and one radix 2 where the power of two is odd), 12 values
// per thread.  (A separate radix-3 stage would cost one more LDS exchange:
// the 768-point transforms measured 5% faster over a whole 768^3 step.)
constexpr bool is_pow2(int L) { return L > 0 && (L & (L - 1)) == 0; }
constexpr int log2i(int L) { return L <= 1 ? 0 : 1 + log2i(L / 2); }
constexpr int plan_stages(int L) {
  return is_pow2(L) ? (L == 4 ? 1 : L == 8 ? 1 : L == 16 ? 2 : L == 32 ? 2 : L == 64 ? 2 : 3)
                    : 1 + log2i(L / 12) / 2 + (log2i(L / 12) % 2);
}
// radix of forward stage s (0-based)
constexpr int plan_radix_fwd(int L, int s) {
  return !is_pow2(L)     ? (s == 0 ? 12 : (s >= plan_stages(L) ? 0 : ((log2i(L / 12) % 2) && s == plan_stages(L) - 1 ? 2 : 4)))
         : L == 4   ? (s == 0 ? 4 : 0)
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
// product of the radices of stages 0..s-1
constexpr int plan_span(int L, int s, bool inv) { return s <= 0 ? 1 : plan_span(L, s - 1, inv) * plan_radix(L, s - 1, inv); }

// Lengths with a factor 5 or 7 (the grids 40, 56, 200, 400, 600 and 700 and
// their half lengths along z).  E values per thread, T = L/E threads; the
// stages (radices 2, 3, 4, 5, 7, 8) need not divide E: stage s has L/R_s
// butterflies, thread t takes butterflies t, t + T, ... (the last round
// partly), and every stage reads its inputs from and writes its outputs to
// LDS.  On entry and exit thread t holds elements t + s T (s < E) in
// registers ("natural" slots); the first stage reads straight from those
// registers when its radix divides E, and the last stage writes straight
// into them when its radix divides E.  Forward and inverse use the same
// stage order.
struct GenPlan {
  int L, E, ns, r[4];
};
constexpr GenPlan kGenPlans[] = {
    {20, 5, 2, {5, 4, 0, 0}},   {28, 7, 2, {7, 4, 0, 0}},   {40, 8, 2, {8, 5, 0, 0}},
    {56, 8, 2, {8, 7, 0, 0}},   {100, 10, 3, {5, 4, 5, 0}}, {200, 10, 3, {5, 8, 5, 0}},
    {300, 10, 4, {5, 4, 3, 5}}, {350, 10, 4, {5, 7, 2, 5}}, {400, 10, 4, {5, 4, 4, 5}},
    {600, 10, 4, {5, 8, 3, 5}}, {700, 10, 4, {5, 7, 4, 5}},
};
constexpr int kNGenPlans = (int)(sizeof(kGenPlans) / sizeof(kGenPlans[0]));
constexpr int gen_find(int L, int i = 0) {
  return i >= kNGenPlans ? -1 : (kGenPlans[i].L == L ? i : gen_find(L, i + 1));
}
constexpr bool is_gen(int L) { return gen_find(L) >= 0; }
constexpr int gen_E(int L) { return kGenPlans[gen_find(L)].E; }
constexpr int gen_stages(int L) { return kGenPlans[gen_find(L)].ns; }
constexpr int gen_radix(int L, int s) { return kGenPlans[gen_find(L)].r[s]; }
constexpr int gen_span(int L, int s) { return s <= 0 ? 1 : gen_span(L, s - 1) * gen_radix(L, s - 1); }
constexpr bool gen_ok(int L) {
  bool ok = gen_span(L, gen_stages(L)) == L && L % gen_E(L) == 0;
  for (int s = 0; s < gen_stages(L); ++s) ok = ok && L % gen_radix(L, s) == 0;
  return ok;
}

// Radix pattern of the registers on entry (first) and exit (last): for the
// lengths with a factor 5 or 7 the natural slots, i.e. the pattern of radix E.
constexpr int plan_first(int L, bool inv) { return is_gen(L) ? gen_E(L) : plan_radix(L, 0, inv); }
constexpr int plan_last(int L, bool inv) { return is_gen(L) ? gen_E(L) : plan_radix(L, plan_stages(L) - 1, inv); }
// elements per thread: 8 (12 for lengths 3 * 2^k), except the single radix-4
// length; the table above for lengths with a factor 5 or 7
constexpr int elems_per_thread(int L) { return is_gen(L) ? gen_E(L) : (L == 4 ? 4 : (is_pow2(L) ? 8 : 12)); }
// the plan multiplies out to L and every radix divides E
constexpr bool plan_ok(int L) {
  bool ok = plan_span(L, plan_stages(L), false) == L;
  for (int s = 0; s < plan_stages(L); ++s) ok = ok && elems_per_thread(L) % plan_radix(L, s, false) == 0;
  return ok;
}

// Element index held in `slot` of thread t for a pattern of radix R.
template <int L, int E, int R>
__device__ __forceinline__ int slot_elem(int t, int slot) {
  return t + (slot / R) * (L / E) + (slot % R) * (L / R);
}

// v, passed through an empty asm statement when ON.  Everything a transform
// derives from its thread index (element indices, LDS addresses, mode
// factors: a few operations per slot) is then worked out again from the
// opaque copy instead of being hoisted out of a rolled loop and held in VGPRs
// across it.  Measured per kernel: for the lengths with a factor 5 or 7 the
// fused y passes stop spilling (n = 700 FP32: 128 VGPRs + 80 bytes of scratch
// per lane -> 95 VGPRs, the nine-output pass 7.7 -> 5.9 ms) and the source
// pass drops from 227 to 145 VGPRs (3% faster); so do the one-buffer fused y
// passes at n = 768 (with the ticket tile order: 128 VGPRs + 60 bytes ->
// 110 VGPRs); so do the z and x passes of the full modified-gravity source
// (n = 256: the z pass of the f(R) pairs 200 -> 166 VGPRs, three waves per
// SIMD instead of two; the ratio spectrum 3.65 -> 3.26 ms); elsewhere the
// recomputation costs more than the registers it frees (n = 512: the source
// pass at 116 instead of 162 VGPRs, four waves per SIMD instead of three,
// still ran 9% slower), so there it stays off.
template <bool ON>
__device__ __forceinline__ int opaque_if(int v) {
  if constexpr (ON) asm volatile("" : "+v"(v));
  return v;
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
__device__ __forceinline__ void dft2(Cx<T>& x0, Cx<T>& x1) {
  const Cx<T> t = x0 - x1;
  x0 = x0 + x1;
  x1 = t;
}

// X_j = sum_m x_m w^(jm), w = exp(D 2 pi i / 3) = -1/2 + D i sqrt(3)/2
template <int D, typename T>
__device__ __forceinline__ void dft3(Cx<T>& x0, Cx<T>& x1, Cx<T>& x2) {
  const T h = T(0.86602540378443864676372317075293618347140262690519);  // sqrt(3)/2
  const Cx<T> s = x1 + x2, d = x1 - x2;
  const Cx<T> m = mk(x0.x - T(0.5) * s.x, x0.y - T(0.5) * s.y);
  const Cx<T> r = mk(-T(D) * h * d.y, T(D) * h * d.x);  // D i sqrt(3)/2 (x1 - x2)
  x0 = x0 + s;
  x1 = m + r;
  x2 = m - r;
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

// 12 points as 3 x 4: m = 4 m1 + m2, k = k1 + 3 k2.  A 3-point DFT over m1
// for each m2, the twiddle w^(m2 k1) (w = exp(D 2 pi i / 12)), then a
// 4-point DFT over m2 for each k1.
template <int D, typename T>
__device__ __forceinline__ void dft12(Cx<T>* x) {
  const T h = T(0.86602540378443864676372317075293618347140262690519);  // sqrt(3)/2
  Cx<T> y[12];  // y[3 m2 + k1]
#pragma unroll
  for (int m2 = 0; m2 < 4; ++m2) {
    Cx<T> a = x[m2], b = x[4 + m2], c = x[8 + m2];
    dft3<D>(a, b, c);
    y[3 * m2] = a;
    y[3 * m2 + 1] = b;
    y[3 * m2 + 2] = c;
  }
  const Cx<T> w1 = mk(h, T(D) * T(0.5)), w2 = mk(T(0.5), T(D) * h), w4 = mk(T(-0.5), T(D) * h);
  y[4] = y[4] * w1;            // m2 = 1, k1 = 1
  y[5] = y[5] * w2;            // m2 = 1, k1 = 2
  y[7] = y[7] * w2;            // m2 = 2, k1 = 1
  y[8] = y[8] * w4;            // m2 = 2, k1 = 2
  y[10] = mul_si<D>(y[10]);    // m2 = 3, k1 = 1: w^3 = D i
  y[11] = mk(-y[11].x, -y[11].y);  // m2 = 3, k1 = 2: w^6 = -1
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    Cx<T> p0 = y[k1], p1 = y[3 + k1], p2 = y[6 + k1], p3 = y[9 + k1];
    dft4<D>(p0, p1, p2, p3);
    x[k1] = p0;
    x[k1 + 3] = p1;
    x[k1 + 6] = p2;
    x[k1 + 9] = p3;
  }
}

// X_k = sum_m x_m w^(km), w = exp(D 2 pi i / P), P = 5 or 7 (odd prime): the
// inputs pair up as s_m = x_m + x_{P-m}, d_m = x_m - x_{P-m} (m = 1..(P-1)/2),
// and for k = 1..(P-1)/2
//   X_k, X_{P-k} = x_0 + sum_m s_m cos(2 pi km/P) +/- D i sum_m d_m sin(2 pi km/P).
// cos and sin of 2 pi j / P for P = 5, 7 and 0 <= j < P
__host__ __device__ constexpr double odd_cos(int P, int j) {
  return P == 5 ? (j == 0 ? 1.0 : (j == 1 || j == 4) ? 0.30901699437494742410229341718281905886436444230012
                                                      : -0.80901699437494742410229341718281905886436444230012)
                : (j == 0 ? 1.0 : (j == 1 || j == 6) ? 0.62348980185873353052500488400423981063227473089640
                                : (j == 2 || j == 5) ? -0.22252093395631440428890256449679475946635556876452
                                                     : -0.90096886790241912623610231950744505116591916213188);
}
__host__ __device__ constexpr double odd_sin(int P, int j) {
  return P == 5 ? (j == 0 ? 0.0 : j == 1 ? 0.95105651629515357211643933337938214340569863412575
                                : j == 2 ? 0.58778525229247312916870595463907276859765243764314
                                : j == 3 ? -0.58778525229247312916870595463907276859765243764314
                                         : -0.95105651629515357211643933337938214340569863412575)
                : (j == 0 ? 0.0 : j == 1 ? 0.78183148246802980870844452667405775023233451870869
                                : j == 2 ? 0.97492791218182360701813168299393121723278580062000
                                : j == 3 ? 0.43388373911755812047576833284835875460999072778746
                                : j == 4 ? -0.43388373911755812047576833284835875460999072778746
                                : j == 5 ? -0.97492791218182360701813168299393121723278580062000
                                         : -0.78183148246802980870844452667405775023233451870869);
}

template <int P, int D, typename T>
__device__ __forceinline__ void dft_odd(Cx<T>* x) {
  constexpr int H = (P - 1) / 2;
  Cx<T> sm[H], dm[H];
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    sm[m - 1] = x[m] + x[P - m];
    dm[m - 1] = x[m] - x[P - m];
  }
  const Cx<T> x0 = x[0];
  Cx<T> tot = x0;
#pragma unroll
  for (int m = 0; m < H; ++m) tot = tot + sm[m];
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    Cx<T> a = x0, b = zero<T>();
#pragma unroll
    for (int m = 1; m <= H; ++m) {
      const int j = (k * m) % P;
      const T c = T(odd_cos(P, j)), sn = T(odd_sin(P, j));
      a = mk(a.x + c * sm[m - 1].x, a.y + c * sm[m - 1].y);
      b = mk(b.x + sn * dm[m - 1].x, b.y + sn * dm[m - 1].y);
    }
    const Cx<T> ib = mul_si<D>(b);  // D i b
    x[k] = a + ib;
    x[P - k] = a - ib;
  }
  x[0] = tot;
}

template <int R, int D, typename T>
__device__ __forceinline__ void butterfly(Cx<T>* x) {
  if constexpr (R == 7 || R == 5) {
    dft_odd<R, D>(x);
  } else if constexpr (R == 12) {
    dft12<D>(x);
  } else if constexpr (R == 8) {
    dft8<D>(x);
  } else if constexpr (R == 4) {
    dft4<D>(x[0], x[1], x[2], x[3]);
  } else if constexpr (R == 3) {
    dft3<D>(x[0], x[1], x[2]);
  } else {
    static_assert(R == 2, "radix 2, 3, 4, 5, 7, 8 or 12");
    dft2<D>(x[0], x[1]);
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
      const int k = (int)((unsigned)b % (unsigned)NS);
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
    const int k = (int)((unsigned)b % (unsigned)NSOUT);
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
// Stages S.. of a transform whose stage S-1 has just run.
template <typename T, int L, int E, int D, int ES, int SY, bool PAD, int S>
__device__ __forceinline__ void fft_from(Cx<T>* v, int t, const Cx<T>* __restrict__ tw, int tws, Cx<T>* lb,
                                         int pingstride, int& ph) {
  constexpr bool INV = D > 0;
  if constexpr (S < plan_stages(L)) {
    constexpr int RP = plan_radix(L, S - 1, INV), NSP = plan_span(L, S - 1, INV);
    constexpr int R = plan_radix(L, S, INV);
    exchange<T, L, E, RP, NSP, R, ES, SY, PAD>(v, t, lb, pingstride, ph);
    stage<T, L, E, R, NSP * RP, D>(v, t, tw, tws);
    fft_from<T, L, E, D, ES, SY, PAD, S + 1>(v, t, tw, tws, lb, pingstride, ph);
  }
}

// ---- lengths with a factor 5 or 7 ----------------------------------------------
// One radix-R butterfly b of a stage of span NS (inputs twiddled as in `stage`).
template <typename T, int L, int R, int NS, int D>
__device__ __forceinline__ void gen_butterfly(Cx<T>* x, int b, const Cx<T>* __restrict__ tw, int tws) {
  if constexpr (NS > 1) {
    const int k = (int)((unsigned)b % (unsigned)NS);
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

// The LDS buffer of an exchange, after the synchronisation its writes need
// (SY_PING: the other buffer, no barrier).
template <typename T, int SY>
__device__ __forceinline__ Cx<T>* gen_buffer(Cx<T>* lb, int pingstride, int& ph) {
  if constexpr (SY == SY_PING) {
    Cx<T>* b = lb + (ph & 1) * pingstride;
    ++ph;
    return b;
  } else {
    lds_sync<SY>();
    return lb;
  }
}

// Stage S: its inputs are in `in` (U butterflies x R values); the outputs go
// to the next stage's inputs through LDS, or (last stage) to the natural
// slots v.
template <typename T, int L, int D, int ES, int SY, bool PAD, int S>
__device__ __forceinline__ void gen_from(Cx<T>* in, Cx<T>* v, int t, const Cx<T>* __restrict__ tw, int tws,
                                         Cx<T>* lb, int pingstride, int& ph) {
  constexpr int E = gen_E(L), TP = L / E;
  constexpr int R = gen_radix(L, S), NS = gen_span(L, S), NB = L / R;
  constexpr int U = (NB + TP - 1) / TP;
  constexpr bool FULL = NB % TP == 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int b = t + u * TP;
    if (FULL || b < NB) gen_butterfly<T, L, R, NS, D>(in + u * R, b, tw, tws);
  }
  constexpr bool LAST = S == gen_stages(L) - 1;
  if constexpr (LAST && E % R == 0) {
    // outputs b + q L/R, b = t + u TP: natural slot u + q U
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < R; ++q) v[u + q * U] = in[u * R + q];
  } else {
    Cx<T>* buf = gen_buffer<T, SY>(lb, pingstride, ph);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = t + u * TP;
      if (FULL || b < NB) {
        const int k = (int)((unsigned)b % (unsigned)NS);
        const int base = (b - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) buf[lds_index<PAD>(base + q * NS) * ES] = in[u * R + q];
      }
    }
    lds_sync<SY>();
    if constexpr (LAST) {
#pragma unroll
      for (int sl = 0; sl < E; ++sl) v[sl] = buf[lds_index<PAD>(t + sl * TP) * ES];
    } else {
      constexpr int R2 = gen_radix(L, S + 1), NB2 = L / R2, U2 = (NB2 + TP - 1) / TP;
      Cx<T> nx[U2 * R2];
#pragma unroll
      for (int u = 0; u < U2; ++u) {
        const int b = t + u * TP;
        if (NB2 % TP == 0 || b < NB2) {
#pragma unroll
          for (int j = 0; j < R2; ++j) nx[u * R2 + j] = buf[lds_index<PAD>(b + j * NB2) * ES];
        } else {
#pragma unroll
          for (int j = 0; j < R2; ++j) nx[u * R2 + j] = zero<T>();
        }
      }
      gen_from<T, L, D, ES, SY, PAD, S + 1>(nx, v, t, tw, tws, lb, pingstride, ph);
    }
  }
}

template <typename T, int L, int D, int ES, int SY, bool PAD>
__device__ __forceinline__ void gen_fft(Cx<T>* v, int t, const Cx<T>* __restrict__ tw, int tws, Cx<T>* lb,
                                        int pingstride, int& ph) {
  constexpr int E = gen_E(L), TP = L / E;
  constexpr int R = gen_radix(L, 0), NB = L / R, U = (NB + TP - 1) / TP;
  Cx<T> x[U * R];
  if constexpr (E % R == 0) {
    // inputs b + j L/R of butterfly b = t + u TP: natural slot u + j U
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < R; ++j) x[u * R + j] = v[u + j * U];
  } else {
    Cx<T>* buf = gen_buffer<T, SY>(lb, pingstride, ph);
#pragma unroll
    for (int sl = 0; sl < E; ++sl) buf[lds_index<PAD>(t + sl * TP) * ES] = v[sl];
    lds_sync<SY>();
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = t + u * TP;
      if (NB % TP == 0 || b < NB) {
#pragma unroll
        for (int j = 0; j < R; ++j) x[u * R + j] = buf[lds_index<PAD>(b + j * NB) * ES];
      } else {
#pragma unroll
        for (int j = 0; j < R; ++j) x[u * R + j] = zero<T>();
      }
    }
  }
  gen_from<T, L, D, ES, SY, PAD, 0>(x, v, t, tw, tws, lb, pingstride, ph);
}

// In: slots in the first-stage pattern of the direction's plan.
// Out: slots in the last-stage pattern.  D = -1 forward, +1 inverse.
// For SY_PING, lb + pingstride is the second buffer and `phase` persists
// across the transforms of a kernel.
template <typename T, int L, int D, int ES, int SY = SY_BLOCK, bool PAD = false, int E = elems_per_thread(L)>
__device__ __forceinline__ void fft(Cx<T>* v, int t, const Cx<T>* __restrict__ tw, int tws, Cx<T>* lb,
                                    int pingstride = 0, int* phase = nullptr) {
  int dummy = 0;
  int& ph = phase ? *phase : dummy;
  if constexpr (is_gen(L)) {
    static_assert(gen_ok(L) && E == gen_E(L), "the stages must multiply out to L");
    gen_fft<T, L, D, ES, SY, PAD>(v, t, tw, tws, lb, pingstride, ph);
  } else {
    constexpr bool INV = D > 0;
    static_assert(plan_ok(L) && L % E == 0, "every radix must divide E and the plan must multiply out to L");
    stage<T, L, E, plan_radix(L, 0, INV), 1, D>(v, t, tw, tws);
    fft_from<T, L, E, D, ES, SY, PAD, 1>(v, t, tw, tws, lb, pingstride, ph);
  }
}

}  // namespace lpt2

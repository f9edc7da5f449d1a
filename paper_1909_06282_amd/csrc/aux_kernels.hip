// Auxiliary kernels: FP64 growth ODE, per-|m|^2 radial tables, the
// deterministic shell binner, cloud-in-cell paint and its transpose, and
// real-space helpers of the full modified-gravity source.
#include <hip/hip_runtime.h>

#include "cx.hpp"
#include "kernels.hpp"

namespace lpt2 {

// ---------------------------------------------------------------------------
// growth ODE (eq. d1, eq. full-d2): one wave per block, lanes 0..62 each run
// one k node's chain and lane 63 the k = 0 normalisation run to a = 1 (every
// block repeats it, so no block waits on another); then normalised D1, D2
// tables.  The factors that depend on a alone (GrowthAFac) are the same for
// every node: the wave works them out for GROWTH_CHUNK steps at a time into
// LDS (the three times of each RK4 step, for the nodes' time grid and for the
// normalisation's), and each chain keeps only its own arithmetic, with 1/Pi
// from the hardware reciprocal and two Newton steps.  A single wave per block
// leaves the whole register file to the chain's 48-double state.
// ---------------------------------------------------------------------------
constexpr int GROWTH_CHUNK = 128;
constexpr int GROWTH_NODES = 63;  // nodes per block; the last lane normalises

// 1/p: v_rcp_f64 refined by two Newton steps (each squares the relative
// error; the result is within an ulp or two of the rounded quotient)
__device__ __forceinline__ double fast_rcp(double p) {
  double r = __builtin_amdgcn_rcp(p);
  double e = fma(-p, r, 1.0);
  r = fma(r, e, r);
  e = fma(-p, r, 1.0);
  return fma(r, e, r);
}

__global__ __launch_bounds__(64) void k_growth(GrowthSetup g, double* __restrict__ d1n, double* __restrict__ d2n) {
  __shared__ GrowthAFac tab[2][3 * GROWTH_CHUNK];  // [0]: to g.a, [1]: the normalisation run to a = 1
  const int lane = threadIdx.x;
  const bool norm = lane == GROWTH_NODES;
  const int i = blockIdx.x * GROWTH_NODES + lane;
  const bool node = !norm && i < g.nk;
  GrowthTri tri;
  if (node) {
    const double k = exp(g.lkmin + (g.lkmax - g.lkmin) * (double)i / (double)(g.nk - 1));
    tri.k = k;
    triangle(k, g.ratio, g.cs, tri.k1, tri.k2);
    tri.cs = g.cs;
    tri.bgr = 1.0 - g.cs * g.cs;
    tri.winther = g.winther;
    tri.with_d2 = (g.mode == 1);
  } else {
    tri.k = tri.k1 = tri.k2 = 0.0;
    tri.cs = 0.0;
    tri.bgr = 1.0;
    tri.winther = 0;
    tri.with_d2 = 0;
  }
  GrowthRhs f;
  f.init(g.c, tri);
  double y[8], k1[8], k2[8], k3[8], k4[8], t[8];
  growth_start(g.c, g.a_init, y);
  const double x0 = log(g.a_init);
  const double h0 = (log(g.a) - x0) / g.steps, h1 = (0.0 - x0) / g.steps;
  const double h = norm ? h1 : h0;
  const GrowthAFac* my = tab[norm ? 1 : 0];
  for (int s0 = 0; s0 < g.steps; s0 += GROWTH_CHUNK) {
    const int ns = g.steps - s0 < GROWTH_CHUNK ? g.steps - s0 : GROWTH_CHUNK;
    __syncthreads();  // the previous chunk's factors are no longer read
    for (int e = lane; e < 2 * 3 * ns; e += blockDim.x) {
      const int grid = e / (3 * ns), r = e % (3 * ns), st = r / 3, kind = r % 3;
      const double hh = grid ? h1 : h0;
      double x = x0 + (s0 + st) * hh;
      if (kind == 1) x = x + 0.5 * hh;
      if (kind == 2) x = x + hh;
      tab[grid][r] = f.afac(x);
    }
    __syncthreads();
    if (node || norm) {
      for (int st = 0; st < ns; ++st) {
        const GrowthAFac a0 = my[3 * st], am = my[3 * st + 1], a1 = my[3 * st + 2];
        f.eval_at(a0, y, k1, fast_rcp);
        for (int q = 0; q < 8; ++q) t[q] = y[q] + 0.5 * h * k1[q];
        f.eval_at(am, t, k2, fast_rcp);
        for (int q = 0; q < 8; ++q) t[q] = y[q] + 0.5 * h * k2[q];
        f.eval_at(am, t, k3, fast_rcp);
        for (int q = 0; q < 8; ++q) t[q] = y[q] + h * k3[q];
        f.eval_at(a1, t, k4, fast_rcp);
        for (int q = 0; q < 8; ++q) y[q] = y[q] + (h / 6.0) * (k1[q] + 2.0 * k2[q] + 2.0 * k3[q] + k4[q]);
      }
    }
  }
  const double nrm = __shfl(y[0], GROWTH_NODES);
  if (node) {
    const double d1v = y[0] / nrm;
    double d2v;
    if (g.mode == 1)
      d2v = y[6] / (nrm * nrm);
    else if (g.mode == 0)
      d2v = -3.0 / 7.0 * d1v * d1v;
    else
      d2v = -3.0 / 7.0 * d1v * d1v * pow(omega_m_a(g.c, g.a), -1.0 / 143.0);
    d1n[i] = d1v;
    d2n[i] = d2v;
  }
}

hipError_t launch_growth(const GrowthSetup& g, double* d1n, double* d2n, hipStream_t s) {
  if (g.nk < 2 || g.nk > 1023) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_growth, dim3((g.nk + GROWTH_NODES - 1) / GROWTH_NODES), dim3(64), 0, s, g, d1n, d2n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// radial tables per integer |m|^2 (FP64).  k = (2 pi/L) sqrt(n2),
// A = sqrt(P(k) n^3 / V), 1/n^3 of the inverse DFT folded in:
//   PSI1 = A D1 (L/2pi) / n2 / n^3    (times  i m_i)
//   PHI  = A / n2 / n^3               (times -m_i m_j)
//   PSI2 = D2 (L/2pi) / n2 / n^3      (times -i m_i)
//   A    = A / n^3
//   R1 = A D1/n2/n^3, R2 = A D1 mu/n2/n^3, R3 = A D1/Pi/n^3,
//   R4 = (2pi/L)^2 A D1/Pi/n^3, R5 = (2pi/L) A D1/n^3, R6 = (2pi/L) A D1/Pi/n^3,
//   C2 = -(G/2) mu, C4 = (2G/3)^2 (M2/12)(k^2/a^2)/Pi, C5 = -(2G/3)(m^2/(2a^2))/Pi.
// ---------------------------------------------------------------------------
__global__ void k_radial(RadialSetup r, const double* __restrict__ d1n, const double* __restrict__ d2n,
                         double* __restrict__ tabs, long n2cnt) {
  const long n2 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n2 >= n2cnt) return;
  double v[TAB_COUNT];
  for (int i = 0; i < TAB_COUNT; ++i) v[i] = 0.0;
  if (n2 > 0) {
    const double kf = 2.0 * kPi / r.box;
    const double k = kf * sqrt((double)n2);
    const double n3 = (double)r.n * (double)r.n * (double)r.n;
    const double t = bbks(r.c, k);
    const double p = r.amp * pow(k, r.c.ns) * t * t;
    const double A = r.unit ? 1.0 : sqrt(p * n3 / (r.box * r.box * r.box));
    const double d1 = interp_lnk(d1n, r.nk, r.lkmin, r.lkmax, k);
    const double d2 = interp_lnk(d2n, r.nk, r.lkmin, r.lkmax, k);
    const double inv = 1.0 / n3;
    const double lf = r.box / (2.0 * kPi);
    v[TAB_PSI1] = A * d1 * lf / (double)n2 * inv;
    v[TAB_PHI] = A / (double)n2 * inv;
    v[TAB_PSI2] = d2 * lf / (double)n2 * inv;
    v[TAB_A] = A * inv;
    const double ad = A * d1 * inv;
    const double a = r.a;
    const double m2 = (r.c.gravity == GRAV_FR) ? hs_m2(r.c, a) : 0.0;
    const double mu = mu_of(r.c, k, a, m2);
    const double G = four_pi_g_rho(r.c, a);
    v[TAB_R1] = ad / (double)n2;
    v[TAB_R2] = ad * mu / (double)n2;
    v[TAB_C2] = -0.5 * G * mu;
    if (r.c.gravity == GRAV_FR) {
      const double pk = big_pi(k, a, m2);
      v[TAB_R3] = ad / pk;
      v[TAB_R4] = kf * kf * ad / pk;
      v[TAB_R5] = kf * ad;
      v[TAB_R6] = kf * ad / pk;
      const double g3 = 2.0 * G / 3.0;
      v[TAB_C4] = g3 * g3 * (hs_M2(r.c, a) / 12.0) * (k * k / (a * a)) / pk;
      v[TAB_C5] = -g3 * (m2 / (2.0 * a * a)) / pk;
    }
  }
  for (int i = 0; i < TAB_COUNT; ++i) tabs[i * n2cnt + n2] = v[i];
  double* pair = tabs + (long)TAB_PAIR64 * n2cnt;
  pair[2 * n2] = v[TAB_PHI];
  pair[2 * n2 + 1] = v[TAB_PSI1];
  float* pair32 = reinterpret_cast<float*>(tabs + (long)TAB_PAIR32 * n2cnt);
  pair32[2 * n2] = (float)v[TAB_PHI];
  pair32[2 * n2 + 1] = (float)v[TAB_PSI1];
  float* psi2_32 = reinterpret_cast<float*>(tabs + (long)TAB_PSI2_32 * n2cnt);
  psi2_32[n2] = (float)v[TAB_PSI2];
}

hipError_t launch_radial(const RadialSetup& r, const double* d1n, const double* d2n, double* tabs, long n2cnt,
                         hipStream_t s) {
  const long blocks = (n2cnt + 255) / 256;
  hipLaunchKernelGGL(k_radial, dim3((unsigned)blocks), dim3(256), 0, s, r, d1n, d2n, tabs, n2cnt);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shell binner.  Along z the shell index of a half-spectrum line is
// non-decreasing, so a wave taking CH consecutive m_z of one line sees
// sorted keys: a segmented inclusive scan (fixed shuffle tree) gives each
// segment's sums in its last lane, which adds them to the wave's private LDS
// histogram.  Waves walk a fixed list of chunks, blocks combine their waves
// in a fixed order, and a second kernel sums the block partials in block
// order with Neumaier compensation: the result is bitwise reproducible.
// ---------------------------------------------------------------------------
// the largest divisor of m that is at most 64 (a chunk of a line in one wavefront)
constexpr int bin_chunk(int m, int c = 64) { return c <= 1 ? 1 : (m % c == 0 ? c : bin_chunk(m, c - 1)); }

template <typename T, int N>
__global__ __launch_bounds__(256) void k_bin1(const Cx<T>* __restrict__ A, const Cx<T>* __restrict__ B, int quantity,
                                              double qscale, int nbins, double kf, double* __restrict__ partial) {
  constexpr int M = N / 2;
  constexpr int CH = bin_chunk(M);  // chunk of a line: divides M
  constexpr int CPL = M / CH;  // chunks per line
  static_assert(M % CH == 0, "a line must split into whole chunks");
  __shared__ double hist[4][BIN_MAXBINS][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 4 * BIN_MAXBINS * 4; i += blockDim.x) (&hist[0][0][0])[i] = 0.0;
  __syncthreads();
  const long nchunks = (long)N * N * CPL;
  const long nw = (long)gridDim.x * 4;
  const long nb2 = (long)nbins * nbins, h2 = (long)(N / 2) * (N / 2);
  for (long ch = (long)blockIdx.x * 4 + wave; ch < nchunks; ch += nw) {
    const long line = ch / CPL;
    const int iz = (int)(ch % CPL) * CH + lane;
    const int ix = (int)(line / N), iy = (int)(line % N);
    const long mx = ix < N / 2 ? ix : ix - N, my = iy < N / 2 ? iy : iy - N;
    int key = -1;
    double w = 0.0, wk = 0.0, wq = 0.0, wq2 = 0.0;
    if (lane < CH) {
      const long n2 = mx * mx + my * my + (long)iz * iz;
      const long v = (n2 * nb2) / h2;
      long b = (long)sqrt((double)v);
      while (b * b > v) --b;
      while ((b + 1) * (b + 1) <= v) ++b;
      if (n2 > 0 && b < nbins) {
        const Cx<T> a = A[line * M + iz];
        double q = 0.0;
        bool ok = true;
        if (quantity == 0 || quantity == 2) {
          q = qscale * ((double)a.x * (double)a.x + (double)a.y * (double)a.y);
          if (quantity == 2) {  // divided by the squared CIC window prod_i sinc^2(pi m_i / N)
            const double h = kPi / (double)N;
            const double sx = mx == 0 ? 1.0 : sin(h * (double)mx) / (h * (double)mx);
            const double sy = my == 0 ? 1.0 : sin(h * (double)my) / (h * (double)my);
            const double sz = iz == 0 ? 1.0 : sin(h * (double)iz) / (h * (double)iz);
            const double w = sx * sx * sy * sy * sz * sz;
            q /= w * w;
          }
        } else {
          const Cx<T> bb = B[line * M + iz];
          const double den = (double)bb.x * (double)bb.x + (double)bb.y * (double)bb.y;
          ok = den > 0.0;
          q = ok ? ((double)a.x * (double)bb.x + (double)a.y * (double)bb.y) / den : 0.0;
        }
        key = (int)b;  // a left-out mode keeps its key (with zero sums) so keys stay contiguous
        if (ok) {
          w = iz == 0 ? 1.0 : 2.0;
          wk = w * kf * sqrt((double)n2);
          wq = w * q;
          wq2 = w * q * q;
        }
      }
    }
    // keys are non-decreasing along the chunk; -1 (DC, beyond the last shell)
    // can only open or close it, so every key forms one contiguous segment.
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int ok_ = __shfl_up(key, off);
      const double a0 = __shfl_up(w, off), a1 = __shfl_up(wk, off), a2 = __shfl_up(wq, off), a3 = __shfl_up(wq2, off);
      if (lane >= off && ok_ == key) {
        w += a0;
        wk += a1;
        wq += a2;
        wq2 += a3;
      }
    }
    const int next = __shfl_down(key, 1);
    const bool tail = (lane == 63) || (next != key);
    if (tail && key >= 0) {
      double* hb = hist[wave][key];
      hb[0] += w;
      hb[1] += wk;
      hb[2] += wq;
      hb[3] += wq2;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nbins * 4; i += blockDim.x) {
    const int b = i >> 2, c = i & 3;
    partial[((long)blockIdx.x * nbins + b) * 4 + c] = ((hist[0][b][c] + hist[1][b][c]) + hist[2][b][c]) + hist[3][b][c];
  }
}

__global__ void k_bin2(const double* __restrict__ partial, int nblk, int nbins, double* __restrict__ out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  double s[4], cmp[4];
  for (int c = 0; c < 4; ++c) s[c] = cmp[c] = 0.0;
  for (int k = 0; k < nblk; ++k) {
    for (int c = 0; c < 4; ++c) {
      const double x = partial[((long)k * nbins + b) * 4 + c];
      const double tt = s[c] + x;
      cmp[c] += (fabs(s[c]) >= fabs(x)) ? (s[c] - tt) + x : (x - tt) + s[c];
      s[c] = tt;
    }
  }
  for (int c = 0; c < 4; ++c) s[c] += cmp[c];
  const double cnt = s[0];
  double km = 0.0, mean = 0.0, sd = 0.0;
  if (cnt > 0.0) {
    km = s[1] / cnt;
    mean = s[2] / cnt;
    const double var = s[3] / cnt - mean * mean;
    sd = sqrt(var > 0.0 ? var : 0.0);
  }
  out[0 * nbins + b] = km;
  out[1 * nbins + b] = cnt;
  out[2 * nbins + b] = mean;
  out[3 * nbins + b] = sd;
}

template <typename T, int N>
static hipError_t bin_t(const void* A, const void* B, int quantity, double qscale, int nbins, double kf,
                        double* partial, double* out4, hipStream_t s) {
  hipLaunchKernelGGL((k_bin1<T, N>), dim3(BIN_BLOCKS), dim3(256), 0, s, (const Cx<T>*)A, (const Cx<T>*)B, quantity,
                     qscale, nbins, kf, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bin2, dim3((nbins + 63) / 64), dim3(64), 0, s, (const double*)partial, BIN_BLOCKS, nbins, out4);
  return hipGetLastError();
}

hipError_t launch_bin(int prec, int n, const void* A, size_t a_cap, const void* B, size_t b_cap, int quantity,
                      double qscale, int nbins, double kf, double* partial, double* out4, hipStream_t s) {
  if (nbins < 1 || nbins > BIN_MAXBINS || !A || !partial || !out4 || quantity < 0 || quantity > 2)
    return hipErrorInvalidValue;
  const size_t field = (size_t)n * n * (n / 2) * 2 * (prec == PREC_F32 ? 4 : 8);
  if (a_cap < field || (quantity == 1 && (!B || b_cap < field))) return hipErrorInvalidValue;
#define CALL(NN)                                                                                      \
  return prec == PREC_F32 ? bin_t<float, NN>(A, B, quantity, qscale, nbins, kf, partial, out4, s)     \
                          : bin_t<double, NN>(A, B, quantity, qscale, nbins, kf, partial, out4, s)
  switch (n) {
    case 8: CALL(8); case 16: CALL(16); case 32: CALL(32); case 64: CALL(64);
    case 128: CALL(128); case 256: CALL(256); case 512: CALL(512);
    case 24: CALL(24); case 48: CALL(48); case 96: CALL(96); case 192: CALL(192);
    case 384: CALL(384); case 768: CALL(768);
    case 40: CALL(40); case 56: CALL(56); case 200: CALL(200); case 400: CALL(400);
    case 600: CALL(600); case 700: CALL(700);
    default: return hipErrorInvalidValue;
  }
#undef CALL
}

// ---------------------------------------------------------------------------
// Cloud-in-cell paint (scatter with atomics) and its transpose (gather).
// Particle p = (ix,iy,iz) moves to u = (ix,iy,iz) + (psi1 + psi2)/cell in
// cell units; per axis the two nearest nodes get 1 - f and f, f = u - floor(u).
// ---------------------------------------------------------------------------
// Scatter: a workgroup of 256 threads takes a Lagrangian tile of
// CIC_TX x CIC_TY x CIC_TZ particles (z fastest, four per thread, held in
// registers) and accumulates their clouds in an LDS window of
// CIC_RX x CIC_RY x CIC_RZ cells placed on the tile shifted by the tile's mean
// displacement (a bulk flow of several cells moves the whole tile; a window
// fixed to the Lagrangian tile would lose it).  Only the non-zero window
// cells are then added to the grid, one coalesced global atomic each; a
// corner outside the window goes to the grid directly, so any displacement is
// painted.  FP32: the window accumulates fixed point in 32-bit integers
// (LDS float atomics run at about half the integer rate here): a weight w is
// added as round(w S), S = 2^22 - 1, and the cell value is recovered as the
// sum / S, within 0.5 / S (1.2e-7) per added weight.  The integer sums are exact and
// cannot wrap: a tile's weights add up to at most its 1024 particles, so a
// cell holds at most 1024 S + 512 < 2^32.  FP64: the window holds doubles.
// Tiles at the high end of an axis are partial when the tile does not
// divide n.  Measured at 512^3 (L = 1024 Mpc/h): 5.6 ms with an 8x8x32 tile,
// a fixed 4-cell halo and float LDS atomics; 2.6 ms like this.
constexpr int CIC_TX = 8, CIC_TY = 8, CIC_TZ = 16;
constexpr int CIC_RX = 16, CIC_RY = 16, CIC_RZ = 28;
constexpr int CIC_BLOCK = 256, CIC_NPT = CIC_TX * CIC_TY * CIC_TZ / CIC_BLOCK;
// a particle farther than this from the origin (in cells), or at a
// non-finite position, is not painted and has no gradient
constexpr double CIC_UMAX = 1073741824.0;
static_assert(CIC_NPT * CIC_BLOCK == CIC_TX * CIC_TY * CIC_TZ, "particles per thread");

template <typename T>
struct CicAcc;
template <>
struct CicAcc<float> {
  using A = unsigned int;
  static constexpr double S = 4194303.0;  // 2^22 - 1
  static_assert(CIC_TX * CIC_TY * CIC_TZ * 4194303.0 + 0.5 * CIC_TX * CIC_TY * CIC_TZ < 4294967296.0, "no wrap");
  __device__ static A to(float w) { return (A)((double)w * S + 0.5); }
  __device__ static float from(A v) { return (float)((double)v * (1.0 / S)); }
};
template <>
struct CicAcc<double> {
  using A = double;
  __device__ static A to(double w) { return w; }
  __device__ static double from(A v) { return v; }
};

template <typename T>
__global__ __launch_bounds__(CIC_BLOCK) void k_cic(int n, double inv_cell, double shift, const T* __restrict__ p1,
                                                   const T* __restrict__ p2, T* __restrict__ rho) {
  using Acc = CicAcc<T>;
  using A = typename Acc::A;
  constexpr int R3 = CIC_RX * CIC_RY * CIC_RZ;
  constexpr int NW = CIC_BLOCK / 64;
  __shared__ A acc[R3];
  __shared__ long long red[4][NW];
  const long n3 = (long)n * n * n;
  const int tpy = (n + CIC_TY - 1) / CIC_TY, tpz = (n + CIC_TZ - 1) / CIC_TZ;
  const int bt = blockIdx.x;
  const int tx = bt / (tpy * tpz), ty = (bt / tpz) % tpy, tz = bt % tpz;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // this thread's particles: base cell and fractional offset per axis
  int i0[CIC_NPT][3];
  T f[CIC_NPT][3];
  bool ok[CIC_NPT];
  long long sx = 0, sy = 0, sz = 0, cnt = 0;
#pragma unroll
  for (int k = 0; k < CIC_NPT; ++k) {
    const int q = threadIdx.x + k * CIC_BLOCK;
    const int id[3] = {tx * CIC_TX + q / (CIC_TY * CIC_TZ), ty * CIC_TY + (q / CIC_TZ) % CIC_TY, tz * CIC_TZ + q % CIC_TZ};
    bool v = id[0] < n && id[1] < n && id[2] < n;  // beyond a partial tile
    const long p = v ? ((long)id[0] * n + id[1]) * n + id[2] : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double u = (double)id[c] + ((double)p1[c * n3 + p] + (double)p2[c * n3 + p]) * inv_cell + shift;
      v = v && fabs(u) < CIC_UMAX;
      const double fl = v ? floor(u) : 0.0;
      f[k][c] = v ? (T)(u - fl) : T(0);
      i0[k][c] = (int)fl;
    }
    ok[k] = v;
    if (v) {
      sx += i0[k][0] - id[0];
      sy += i0[k][1] - id[1];
      sz += i0[k][2] - id[2];
      ++cnt;
    }
  }
  // the window: the tile moved by its mean displacement (whole cells),
  // clamped to a few boxes so every index below stays in int range
  for (int off = 32; off > 0; off >>= 1) {
    sx += __shfl_xor(sx, off);
    sy += __shfl_xor(sy, off);
    sz += __shfl_xor(sz, off);
    cnt += __shfl_xor(cnt, off);
  }
  if (lane == 0) {
    red[0][wv] = sx;
    red[1][wv] = sy;
    red[2][wv] = sz;
    red[3][wv] = cnt;
  }
  for (int i = threadIdx.x; i < R3; i += CIC_BLOCK) acc[i] = A(0);
  __syncthreads();
  long long ts[3] = {0, 0, 0}, tc = 0;
  for (int w = 0; w < NW; ++w) {
    ts[0] += red[0][w];
    ts[1] += red[1][w];
    ts[2] += red[2][w];
    tc += red[3][w];
  }
  int o0[3];
  const int tile0[3] = {tx * CIC_TX - (CIC_RX - CIC_TX) / 2, ty * CIC_TY - (CIC_RY - CIC_TY) / 2,
                        tz * CIC_TZ - (CIC_RZ - CIC_TZ) / 2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    long long m = tc > 0 ? (ts[c] >= 0 ? (ts[c] + tc / 2) / tc : -((-ts[c] + tc / 2) / tc)) : 0;
    m = m < -4LL * n ? -4LL * n : (m > 4LL * n ? 4LL * n : m);
    o0[c] = tile0[c] + (int)m;
  }
  auto wrap = [n](int g) {
    const int r = g % n;
    return r < 0 ? r + n : r;
  };
#pragma unroll
  for (int k = 0; k < CIC_NPT; ++k) {
    if (!ok[k]) continue;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
      const int ox = (o >> 2) & 1, oy = (o >> 1) & 1, oz = o & 1;
      const T w = (ox ? f[k][0] : T(1) - f[k][0]) * (oy ? f[k][1] : T(1) - f[k][1]) * (oz ? f[k][2] : T(1) - f[k][2]);
      const int gx = i0[k][0] + ox, gy = i0[k][1] + oy, gz = i0[k][2] + oz;
      const int rx = gx - o0[0], ry = gy - o0[1], rz = gz - o0[2];
      if (rx >= 0 && rx < CIC_RX && ry >= 0 && ry < CIC_RY && rz >= 0 && rz < CIC_RZ)
        atomicAdd(&acc[(rx * CIC_RY + ry) * CIC_RZ + rz], Acc::to(w));
      else
        atomicAdd(&rho[((long)wrap(gx) * n + wrap(gy)) * n + wrap(gz)], w);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R3; i += CIC_BLOCK) {
    const A v = acc[i];
    if (v != A(0)) {
      const int gx = o0[0] + i / (CIC_RY * CIC_RZ), gy = o0[1] + (i / CIC_RZ) % CIC_RY, gz = o0[2] + i % CIC_RZ;
      atomicAdd(&rho[((long)wrap(gx) * n + wrap(gy)) * n + wrap(gz)], Acc::from(v));
    }
  }
}

template <typename T>
__global__ void k_cic_back(int n, double inv_cell, const T* __restrict__ p1, const T* __restrict__ p2,
                           const T* __restrict__ gd, T* __restrict__ gp) {
  const long n3 = (long)n * n * n;
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n3) return;
  const int ix = (int)(p / ((long)n * n)), iy = (int)((p / n) % n), iz = (int)(p % n);
  const int id[3] = {ix, iy, iz};
  int i0[3];
  double f[3];
  for (int c = 0; c < 3; ++c) {
    const double u = (double)id[c] + ((double)p1[c * n3 + p] + (double)p2[c * n3 + p]) * inv_cell;
    if (!(fabs(u) < CIC_UMAX)) {  // same rule as the paint: the particle has no gradient
      for (int q = 0; q < 3; ++q) gp[q * n3 + p] = (T)0;
      return;
    }
    const double fl = floor(u);
    f[c] = u - fl;
    long ii = (long)fl % n;
    if (ii < 0) ii += n;
    i0[c] = (int)ii;
  }
  double g[3] = {0.0, 0.0, 0.0};
  for (int o = 0; o < 8; ++o) {
    const int ox = (o >> 2) & 1, oy = (o >> 1) & 1, oz = o & 1;
    const double wx = ox ? f[0] : 1.0 - f[0], wy = oy ? f[1] : 1.0 - f[1], wz = oz ? f[2] : 1.0 - f[2];
    const double dx = ox ? 1.0 : -1.0, dy = oy ? 1.0 : -1.0, dz = oz ? 1.0 : -1.0;
    const int gx = (i0[0] + ox) % n, gy = (i0[1] + oy) % n, gz = (i0[2] + oz) % n;
    const double v = (double)gd[((long)gx * n + gy) * n + gz];
    g[0] += v * dx * wy * wz;
    g[1] += v * wx * dy * wz;
    g[2] += v * wx * wy * dz;
  }
  for (int c = 0; c < 3; ++c) gp[c * n3 + p] = (T)(g[c] * inv_cell);
}

// number of non-finite values (NaN, +-inf) of x[0..count), added to *out
template <typename T>
__global__ __launch_bounds__(256) void k_count_nonfinite(const T* __restrict__ x, long count,
                                                         unsigned long long* __restrict__ out) {
  unsigned long long c = 0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x)
    c += __builtin_isfinite(x[i]) ? 0ull : 1ull;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

template <typename T>
__global__ void k_fill(T* __restrict__ x, long count, T value) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) x[i] = value;
}

static unsigned grid_for(long count) {
  long b = (count + 255) / 256;
  return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

hipError_t launch_fill(int prec, void* x, long count, double value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (prec == PREC_F32)
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(count)), dim3(256), 0, s, (float*)x, count, (float)value);
  else
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(count)), dim3(256), 0, s, (double*)x, count, value);
  return hipGetLastError();
}

__global__ void k_zero_u64(unsigned long long* out) { *out = 0ull; }

// *out is set to zero first (by a kernel, so that a caller may capture the
// sequence in a graph), then the count is added to it
hipError_t launch_count_nonfinite(int prec, const void* x, long count, unsigned long long* out, hipStream_t s) {
  if (!x || !out) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, out);
  if (count <= 0) return hipGetLastError();
  const unsigned blocks = grid_for(count) < 4096 ? grid_for(count) : 4096;
  if (prec == PREC_F32)
    hipLaunchKernelGGL(k_count_nonfinite<float>, dim3(blocks), dim3(256), 0, s, (const float*)x, count, out);
  else
    hipLaunchKernelGGL(k_count_nonfinite<double>, dim3(blocks), dim3(256), 0, s, (const double*)x, count, out);
  return hipGetLastError();
}

hipError_t launch_cic(int prec, int n, double box, const void* psi1, const void* psi2, void* delta, hipStream_t s,
                      double shift) {
  const long n3 = (long)n * n * n;
  hipError_t e = launch_fill(prec, delta, n3, -1.0, s);
  if (e != hipSuccess) return e;
  const double ic = n / box;
  if (n < 2) return hipErrorInvalidValue;
  const long tpx = (n + CIC_TX - 1) / CIC_TX, tpy = (n + CIC_TY - 1) / CIC_TY, tpz = (n + CIC_TZ - 1) / CIC_TZ;
  const unsigned blocks = (unsigned)(tpx * tpy * tpz);  // one per tile
  if (prec == PREC_F32)
    hipLaunchKernelGGL(k_cic<float>, dim3(blocks), dim3(CIC_BLOCK), 0, s, n, ic, shift, (const float*)psi1, (const float*)psi2,
                       (float*)delta);
  else
    hipLaunchKernelGGL(k_cic<double>, dim3(blocks), dim3(CIC_BLOCK), 0, s, n, ic, shift, (const double*)psi1, (const double*)psi2,
                       (double*)delta);
  return hipGetLastError();
}

// Interlacing: a = (a + b exp(i pi (m_x + m_y + m_z) / n)) / 2 over the half
// spectrum (x, y, then m_z = 0 .. n/2 - 1), where b is the transform of the
// density painted with every particle moved by half a cell along each axis:
// the phase undoes that move and the alias images with an odd index sum
// cancel in the average.
template <typename T>
__global__ void k_interlace(int n, Cx<T>* __restrict__ a, const Cx<T>* __restrict__ b) {
  const long m = n / 2, count = (long)n * n * m;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long)gridDim.x * blockDim.x) {
    const int ix = (int)(i / ((long)n * m)), iy = (int)((i / m) % n), iz = (int)(i % m);
    const int sm = (ix < n / 2 ? ix : ix - n) + (iy < n / 2 ? iy : iy - n) + iz;  // in (-n, n)
    double sn, cs;
    sincos(kPi * (double)sm / (double)n, &sn, &cs);
    const Cx<T> u = a[i], v = b[i];
    a[i] = mk(T(0.5 * ((double)u.x + cs * (double)v.x - sn * (double)v.y)),
              T(0.5 * ((double)u.y + cs * (double)v.y + sn * (double)v.x)));
  }
}

hipError_t launch_interlace(int prec, int n, void* a, size_t a_cap, const void* b, size_t b_cap, hipStream_t s) {
  const long count = (long)n * n * (n / 2);
  const size_t bytes = (size_t)count * 2 * (prec == PREC_F32 ? 4 : 8);
  if (n < 2 || !a || !b || bytes > a_cap || bytes > b_cap) return hipErrorInvalidValue;
  if (prec == PREC_F32)
    hipLaunchKernelGGL(k_interlace<float>, dim3(grid_for(count)), dim3(256), 0, s, n, (Cx<float>*)a,
                       (const Cx<float>*)b);
  else
    hipLaunchKernelGGL(k_interlace<double>, dim3(grid_for(count)), dim3(256), 0, s, n, (Cx<double>*)a,
                       (const Cx<double>*)b);
  return hipGetLastError();
}

// Eulerian positions (eq. position): particle (ix, iy, iz) starts at
// q = (ix, iy, iz) L/n; x = q + psi1 + psi2 wrapped into [0, L).
template <typename T>
__global__ void k_positions(int n, double box, const T* __restrict__ p1, const T* __restrict__ p2,
                            T* __restrict__ x) {
  const long n3 = (long)n * n * n;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n3) return;
  const int c = (int)(i / n3);
  const long p = i - c * n3;
  const long id = c == 0 ? p / ((long)n * n) : (c == 1 ? (p / n) % n : p % n);
  const T L = (T)box;
  const T q = (T)id * (T)(box / n);
  T v = (q + p1[i]) + p2[i];
  v = v - floor(v / L) * L;
  if (v >= L) v -= L;  // rounding at the upper edge
  if (v < T(0)) v += L;
  x[i] = v;
}

hipError_t launch_positions(int prec, int n, double box, const void* psi1, const void* psi2, void* pos, hipStream_t s) {
  const long cnt = 3L * n * n * n;
  const unsigned blocks = (unsigned)((cnt + 255) / 256);
  if (prec == PREC_F32)
    hipLaunchKernelGGL(k_positions<float>, dim3(blocks), dim3(256), 0, s, n, box, (const float*)psi1,
                       (const float*)psi2, (float*)pos);
  else
    hipLaunchKernelGGL(k_positions<double>, dim3(blocks), dim3(256), 0, s, n, box, (const double*)psi1,
                       (const double*)psi2, (double*)pos);
  return hipGetLastError();
}

hipError_t launch_cic_back(int prec, int n, double box, const void* psi1, const void* psi2, const void* gdelta,
                           void* gpsi, hipStream_t s) {
  const long n3 = (long)n * n * n;
  const double ic = n / box;
  const unsigned blocks = (unsigned)((n3 + 255) / 256);
  if (prec == PREC_F32)
    hipLaunchKernelGGL(k_cic_back<float>, dim3(blocks), dim3(256), 0, s, n, ic, (const float*)psi1,
                       (const float*)psi2, (const float*)gdelta, (float*)gpsi);
  else
    hipLaunchKernelGGL(k_cic_back<double>, dim3(blocks), dim3(256), 0, s, n, ic, (const double*)psi1,
                       (const double*)psi2, (const double*)gdelta, (double*)gpsi);
  return hipGetLastError();
}

}  // namespace lpt2

// Memory-pattern references of the strided and line passes (a measurement
// companion of the library, built as libmembench.so; not part of the C ABI
// of liblpt2).  Each pattern moves the bytes of one pass of the 3D FFT chain
// with the pass's access shape and no arithmetic: nin FP32 half-spectrum
// fields read, nout written, per tile of W adjacent columns (the strided
// passes) or per contiguous run (the line passes), every load of a tile
// before its stores.  A pass near its pattern's rate is bound by its
// traffic and access shape rather than by its arithmetic; the fused passes,
// which overlap the next tile's loads with their transforms, can beat this
// plain form by a few percent.
//
//   kind 0: line pass (z): element i of every field, contiguous;
//   kind 1: y columns: field [n][n][n/2] complex, column (x plane, z mode),
//           rows along y (stride n/2 elements), tiles of W columns in a plane;
//   kind 2: x columns: column (y, z mode), rows along x (stride n^2/2).
// Strided tiles: 64 threads per column, n/64 rows per thread (rows t + 64 s;
// n = 512 or 768), persistent over tiles like the library's fused passes:
// kind 1 or 2 in the grid-stride order (XCD-contiguous under 128-byte rows),
// kind 9 or 10 (kind + 8) in the ticket order (the workgroups of each XCD
// take the tiles of one contiguous range from a counter, in step), the two
// orders the library's column passes use.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

typedef float V2 __attribute__((ext_vector_type(2)));  // one complex value

constexpr int MB_MAXF = 16;

struct Fields {
  const V2* in[MB_MAXF];
  V2* out[MB_MAXF];
};

// ticket of group x: tiles lo.. of the group's range, then -1 once it is
// exhausted (the group's last workgroup out sets its two words back to zero)
__device__ long mb_ticket(unsigned* tq, int x, long lo, long hi, unsigned nblk, bool& out) {
  if (out) return -1;
  const long t = lo + (long)atomicAdd(&tq[x], 1u);
  if (t < hi) return t;
  out = true;
  if (atomicAdd(&tq[8 + x], 1u) == nblk - 1) {
    tq[x] = 0u;
    tq[8 + x] = 0u;
  }
  return -1;
}

template <int W, int R>
__global__ __launch_bounds__(W * 64) void k_columns(Fields f, int nin, int nout, long plane_stride, long row_stride,
                                                   int ncol, int nplanes, unsigned* tq) {
  __shared__ long s_tile;
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  const int bpp = (ncol + W - 1) / W;
  const long ntiles = (long)nplanes * bpp;
  // grid-stride order: rows under 128 bytes, each XCD's workgroups take one
  // contiguous range of tiles (workgroup b runs on XCD b % 8)
  long first = blockIdx.x;
  if (!tq && W * (int)sizeof(V2) < 128) {
    const long q = gridDim.x / 8;
    if (first < 8 * q) first = (first % 8) * q + first / 8;
  }
  // ticket order: group x = b % g works through [x per, (x+1) per)
  const int g = gridDim.x < 8 ? (int)gridDim.x : 8, x = (int)(blockIdx.x % g);
  const unsigned nblk = (gridDim.x - x + g - 1) / g;
  const long per = (ntiles + g - 1) / g;
  const long lo = x * per < ntiles ? x * per : ntiles, hi = lo + per < ntiles ? lo + per : ntiles;
  bool out = false;
  for (long tile = first;;) {
    if (tq) {
      __syncthreads();
      if (threadIdx.x == 0) s_tile = mb_ticket(tq, x, lo, hi, nblk, out);
      __syncthreads();
      tile = s_tile;
      if (tile < 0) break;
    } else if (tile >= ntiles) {
      break;
    }
    const long p = tile / bpp;
    const int col = (int)(tile % bpp) * W + c;
    if (!tq) tile += gridDim.x;
    if (col >= ncol) continue;
    const long base = p * plane_stride + col;
    V2 acc[R];
#pragma unroll
    for (int s = 0; s < R; ++s) acc[s] = V2{0.f, 0.f};
    for (int k = 0; k < nin; ++k) {
#pragma unroll
      for (int s = 0; s < R; ++s) acc[s] += __builtin_nontemporal_load(&f.in[k][base + (t + 64 * s) * row_stride]);
    }
    for (int o = 0; o < nout; ++o) {
#pragma unroll
      for (int s = 0; s < R; ++s) {
        V2 v = acc[s];
        v.x += (float)o;
        __builtin_nontemporal_store(v, &f.out[o][base + (t + 64 * s) * row_stride]);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_lines(Fields f, int nin, int nout, long count) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count; i += (long)gridDim.x * 256) {
    V2 acc = V2{0.f, 0.f};
    for (int k = 0; k < nin; ++k) acc += f.in[k][i];
    for (int o = 0; o < nout; ++o) {
      V2 v = acc;
      v.x += (float)o;
      f.out[o][i] = v;
    }
  }
}

template <int W, int R>
hipError_t launch_columns(const Fields& f, int nin, int nout, long ps, long rs, int ncol, int nplanes, unsigned* tq,
                          hipStream_t s) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_columns<W, R>), W * 64, 0);
  if (e != hipSuccess) return e;
  const long ntiles = (long)nplanes * ((ncol + W - 1) / W);
  long blocks = (long)(per > 0 ? per : 1) * cus;
  if (blocks > ntiles) blocks = ntiles;
  hipLaunchKernelGGL((k_columns<W, R>), dim3((unsigned)blocks), dim3(W * 64), 0, s, f, nin, nout, ps, rs, ncol, nplanes,
                     tq);
  return hipGetLastError();
}

}  // namespace

// Time one pattern on the current device: kind 0/1/2/9/10 as above, grid n
// (the strided kinds need n = 512 or 768: 64 threads x n/64 rows), nin + nout
// <= 16 fields of n^3 floats each (allocated and freed here), tile width W in
// {8, 16, 32} columns for the strided kinds.  Writes the mean milliseconds
// per launch over `reps` timed launches (after two untimed ones).  Returns 0,
// or -1 for bad arguments, -3 if the fields cannot be allocated, -4 for a HIP
// error.
extern "C" int membench_pattern(int kind, int n, int nin, int nout, int width, int reps, double* ms) {
  const bool tickets = kind == 9 || kind == 10;
  if (tickets) kind -= 8;
  if (!ms || kind < 0 || kind > 2 || nin < 1 || nout < 1 || nin + nout > MB_MAXF || reps < 1) return -1;
  if (kind != 0 && !((n == 512 || n == 768) && (width == 8 || width == 16 || width == 32))) return -1;
  if (kind == 0 && (n < 8 || n > 1024)) return -1;
  const long count = (long)n * n * (n / 2);  // complex values per field
  Fields f{};
  void* mem[MB_MAXF] = {};
  unsigned* tq = nullptr;  // ticket words (16), zero between launches
  int status = 0;
  if (tickets && (hipMalloc(&tq, 16 * sizeof(unsigned)) != hipSuccess || hipMemset(tq, 0, 16 * sizeof(unsigned)) != hipSuccess))
    status = -3;
  hipEvent_t a = nullptr, b = nullptr;
  for (int i = 0; i < nin + nout && status == 0; ++i) {
    if (hipMalloc(&mem[i], count * sizeof(V2)) != hipSuccess) status = -3;
    else if (hipMemset(mem[i], 0, count * sizeof(V2)) != hipSuccess) status = -4;
  }
  if (status == 0) {
    for (int i = 0; i < nin; ++i) f.in[i] = static_cast<const V2*>(mem[i]);
    for (int o = 0; o < nout; ++o) f.out[o] = static_cast<V2*>(mem[nin + o]);
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) status = -4;
  }
  auto launch = [&]() -> hipError_t {
    const int m = n / 2;
    if (kind == 0) {
      hipLaunchKernelGGL(k_lines, dim3(2048), dim3(256), 0, nullptr, f, nin, nout, count);
      return hipGetLastError();
    }
    const long ps = kind == 1 ? (long)n * m : 0;
    const long rs = kind == 1 ? m : (long)n * m;
    const int ncol = kind == 1 ? m : n * m;
    const int np = kind == 1 ? n : 1;
    if (n == 768) {
      if (width == 8) return launch_columns<8, 12>(f, nin, nout, ps, rs, ncol, np, tq, nullptr);
      if (width == 16) return launch_columns<16, 12>(f, nin, nout, ps, rs, ncol, np, tq, nullptr);
      return launch_columns<32, 12>(f, nin, nout, ps, rs, ncol, np, tq, nullptr);
    }
    if (width == 8) return launch_columns<8, 8>(f, nin, nout, ps, rs, ncol, np, tq, nullptr);
    if (width == 16) return launch_columns<16, 8>(f, nin, nout, ps, rs, ncol, np, tq, nullptr);
    return launch_columns<32, 8>(f, nin, nout, ps, rs, ncol, np, tq, nullptr);
  };
  if (status == 0) {
    for (int i = 0; i < 2 && status == 0; ++i)
      if (launch() != hipSuccess) status = -4;
    if (status == 0 && hipEventRecord(a, nullptr) != hipSuccess) status = -4;
    for (int i = 0; i < reps && status == 0; ++i)
      if (launch() != hipSuccess) status = -4;
    float t = 0.f;
    if (status == 0 && (hipEventRecord(b, nullptr) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                        hipEventElapsedTime(&t, a, b) != hipSuccess))
      status = -4;
    if (status == 0) *ms = (double)t / reps;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  for (int i = 0; i < MB_MAXF; ++i)
    if (mem[i]) (void)hipFree(mem[i]);
  if (tq) (void)hipFree(tq);
  return status;
}

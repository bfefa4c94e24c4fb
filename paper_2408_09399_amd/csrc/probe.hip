// Dependent-load latency probe: the floor of a chain of memory trips.
//
// The insertion loop is a serial chain in which every step waits for loads whose addresses
// come from the previous loads (list entries, then the similarities they name). Its floor
// is the number of such trips times the latency of one. This kernel measures that latency
// from one wave: each lane follows its own cyclic chain of 32-bit indices (next[p] is the
// element read after p), and the wave issues its next load only when every lane's load has
// returned, as the loop's walks do. Lanes may share one chain (every lane reads the same
// address: one cache line per trip) or follow 64 chains (64 lines per trip, a gather).
#include "../../include/tmfg.h"
#include "common.h"
#include "internal.h"

namespace tmfg {

namespace {
__global__ __launch_bounds__(64) void chase_kernel(const uint32_t* __restrict__ next, const uint32_t* __restrict__ start,
                                                   int steps, int warm, unsigned long long* __restrict__ ticks,
                                                   uint32_t* __restrict__ sink) {
  const int lane = threadIdx.x;
  uint32_t p = start[lane];
  // warm: read the same chain once untimed, so that the timed pass finds it in this CU's L2
  for (int i = 0; warm && i < steps; ++i) p = next[p];
  const uint32_t w = warm ? p : 0u;
  p = start[lane];
  const uint64_t t0 = wall_clock64();
  // a load's address is the previous load's value, so the wave waits for all of its lanes'
  // data before it can issue the next one
  for (int i = 0; i < steps; ++i) p = next[p];
  const uint64_t t1 = wall_clock64();
  if (lane == 0) *ticks = t1 - t0;
  sink[lane] = p ^ w;           // keeps both passes live
}

// next[32 x] = 32 y with y = (a x + c) mod lines: one cycle through every 128-byte line of
// the buffer (a full-period linear congruential map: lines a power of two, a = 1 mod 4, c odd).
constexpr uint64_t kLcgA = 6364136223846793005ull, kLcgC = 1442695040888963407ull;
__host__ __device__ inline uint64_t lcg_next(uint64_t x, uint64_t lines) { return (x * kLcgA + kLcgC) & (lines - 1); }

__global__ void chain_fill_kernel(uint32_t* __restrict__ next, uint64_t lines) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < lines; x += (uint64_t)gridDim.x * blockDim.x)
    next[x * 32] = (uint32_t)(lcg_next(x, lines) * 32);
}
}  // namespace

constexpr uint64_t kWarmBytes = 2u << 20;   // chains this small are read once untimed first

hipError_t probe_latency(int64_t bytes, int lanes, int steps, double* ns_per_trip) {
  uint64_t lines = 64;
  while (lines * 2 * 128 <= (uint64_t)bytes && lines * 2 * 32 <= 0xffffffffull) lines *= 2;
  // lane l starts l * steps lines along the cycle, so that no two lanes read one line
  uint32_t h_start[64];
  uint64_t x = 0;
  for (int l = 0; l < 64; ++l) {
    h_start[l] = (uint32_t)(x * 32);
    if (lanes > 1)
      for (int i = 0; i < steps; ++i) x = lcg_next(x, lines);
  }
  uint32_t* next = nullptr;
  uint32_t* aux = nullptr;
  hipError_t e = hipMalloc((void**)&next, lines * 128);
  if (e != hipSuccess) return e;
  if ((e = hipMalloc((void**)&aux, 64 * 4 * 2 + 16)) != hipSuccess) {
    hipFree(next);
    return e;
  }
  uint32_t* d_start = aux;
  uint32_t* sink = aux + 64;
  unsigned long long* ticks = (unsigned long long*)(aux + 128);
  unsigned long long h_ticks = 0;
  int khz = 0;
  int dev = 0;
  if ((e = hipGetDevice(&dev)) == hipSuccess &&
      (e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev)) == hipSuccess &&
      (e = hipMemcpy(d_start, h_start, sizeof(h_start), hipMemcpyHostToDevice)) == hipSuccess) {
    hipLaunchKernelGGL(chain_fill_kernel, dim3(1024), dim3(256), 0, 0, next, lines);
    if ((e = hipGetLastError()) == hipSuccess) {
      const int warm = lines * 128 <= kWarmBytes ? 1 : 0;
      hipLaunchKernelGGL(chase_kernel, dim3(1), dim3(64), 0, 0, next, d_start, steps, warm, ticks, sink);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpy(&h_ticks, ticks, sizeof(h_ticks), hipMemcpyDeviceToHost);
  }
  hipFree(next);
  hipFree(aux);
  if (e == hipSuccess) *ns_per_trip = khz > 0 ? (double)h_ticks * 1e6 / khz / steps : 0.0;
  return e;
}


}  // namespace tmfg

extern "C" tmfg_status tmfg_probe_load_latency(int64_t bytes, int32_t lanes, int32_t steps, double* ns_per_trip) {
  if (!ns_per_trip || (lanes != 1 && lanes != 64)) return TMFG_E_INVALID;
  if (bytes < 64 * 128 || bytes > ((int64_t)16 << 30) || steps < 1 || steps > (1 << 24)) return TMFG_E_SIZE;
  const hipError_t e = tmfg::probe_latency(bytes, lanes, steps, ns_per_trip);
  if (e == hipErrorOutOfMemory) {
    tmfg::record_hip_error((int)e);
    return TMFG_E_NOMEM;
  }
  if (e != hipSuccess) {
    tmfg::record_hip_error((int)e);
    return TMFG_E_HIP;
  }
  return TMFG_OK;
}

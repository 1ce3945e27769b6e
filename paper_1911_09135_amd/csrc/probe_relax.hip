// Measurement probe, not part of the traversal: the edge-relaxation inner
// loop of SSSP alone (column and weight streamed in CSR order, a gather of
// the destination's label, an atomic minimum when the candidate is smaller),
// over every edge of a graph once, perfectly balanced (256-edge chunks
// claimed from 64 striped counters), with no inspection, bins, pushes or
// barriers.  It bounds what a label layout can gain: labels in one array
// relaxed by any XCD ("flat"), or split into eight destination slices, XCD x
// relaxing only the edges into slice x, whose labels are contiguous
// ("sliced", the caller passes the edges grouped by slice and the column
// entries renumbered into the sliced label array).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kStripes = 64;

__device__ __forceinline__ uint32_t xcd_of_wave() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u;  // XCC_ID[2:0]
}

// V: 0 = 8-byte label word, atomic minimum; 1 = 8-byte gather only;
// 2 = 4-byte label, atomic minimum; 3 = 4-byte gather only.
template <int V>
__global__ __launch_bounds__(256) void k_probe(const int32_t *col, const int32_t *w, void *labels, int64_t m,
                                               const int64_t *list_off, int sliced, int32_t c0,
                                               unsigned long long *claim, unsigned long long *lowered) {
  __shared__ uint32_t s_x;
  if (threadIdx.x == 0) s_x = sliced ? xcd_of_wave() : 0u;
  __syncthreads();
  const uint32_t x = s_x;
  const int64_t b0 = sliced ? list_off[x] : 0, b1 = sliced ? list_off[x + 1] : m;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = blockIdx.x * (blockDim.x / 64u) + (threadIdx.x >> 6);
  const int64_t chunks = (b1 - b0 + 255) / 256;
  unsigned long long low = 0;
  unsigned long long *L64 = (unsigned long long *)labels;
  int32_t *L32 = (int32_t *)labels;
  for (int t = 0; t < kStripes; ++t) {
    const int k = (int)((wave + (uint32_t)t) % kStripes);
    for (;;) {
      unsigned long long j = 0;
      if (lane == 0) j = atomicAdd(&claim[((size_t)x * kStripes + k) * 32], 1ull);
      j = __shfl(j, 0);
      const int64_t chunk = k + (int64_t)kStripes * (int64_t)j;
      if (chunk >= chunks) break;
      const int64_t base = b0 + chunk * 256;
      bool act[4];
      int32_t d[4], ww[4], cur[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t e = base + u * 64 + lane;
        act[u] = e < b1;
        d[u] = col[act[u] ? e : b0];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) ww[u] = w[act[u] ? base + u * 64 + lane : b0];
#pragma unroll
      for (int u = 0; u < 4; ++u) cur[u] = V < 2 ? (int32_t)(L64[d[u]] >> 32) : L32[d[u]];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t cand = ww[u] + c0;
        if (!act[u] || cand >= cur[u]) continue;
        if (V == 0) {
          const unsigned long long old = __hip_atomic_fetch_min(
              &L64[d[u]], ((unsigned long long)(uint32_t)cand << 32) | 1ull, __ATOMIC_RELAXED,
              __HIP_MEMORY_SCOPE_AGENT);
          low += cand < (int32_t)(old >> 32);
        } else if (V == 2) {
          const int32_t old = __hip_atomic_fetch_min(&L32[d[u]], cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          low += cand < old;
        } else {
          low += 1;
        }
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) low += __shfl_xor(low, o);
  if (lane == 0 && low) atomicAdd(lowered, low);
}

}  // namespace

// Run one probe launch of `grid` workgroups of 256 threads on `stream`.
// labels: 8-byte words (variants 0, 1) or 4-byte labels (2, 3), indexed by
// the column entries; list_off: 9 entries (sliced) or unused; claim: at
// least 8 * 64 * 32 zeroed 64-bit counters; lowered: one 64-bit counter.
extern "C" int alb_probe_relax(int variant, const int32_t *col, const int32_t *w, void *labels, int64_t m,
                               const int64_t *list_off, int sliced, int32_t c0, unsigned long long *claim,
                               unsigned long long *lowered, int grid, void *stream) {
  hipStream_t s = (hipStream_t)stream;
  switch (variant) {
    case 0: hipLaunchKernelGGL(k_probe<0>, dim3(grid), dim3(256), 0, s, col, w, labels, m, list_off, sliced, c0, claim, lowered); break;
    case 1: hipLaunchKernelGGL(k_probe<1>, dim3(grid), dim3(256), 0, s, col, w, labels, m, list_off, sliced, c0, claim, lowered); break;
    case 2: hipLaunchKernelGGL(k_probe<2>, dim3(grid), dim3(256), 0, s, col, w, labels, m, list_off, sliced, c0, claim, lowered); break;
    case 3: hipLaunchKernelGGL(k_probe<3>, dim3(grid), dim3(256), 0, s, col, w, labels, m, list_off, sliced, c0, claim, lowered); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

// Calibration kernels for the roofline of the traversal kernels (measurement
// only; not part of the traversal library).  Each measures one memory
// primitive the level kernels are built from, so that the achieved rate of a
// kernel can be set against what the chip sustains for that primitive:
//
//   random 4-byte loads from a table of 2^k words (a BFS visited bitmap, an
//     SSSP distance array), 8 independent loads in flight per lane;
//   a streaming read of int32 and of int4 elements (the col_idx stream);
//   a streaming int32 read with one dependent probe of a table per element
//     (the child body: v = col[e], then visited[v]);
//   random atomicOr on a table (the BFS claim), with and without its return;
//   random plain stores (the level writes, the per-XCD visited copies);
//   random loads of a table while some workgroups update it, or a second
//     table, with atomics (a probed bitmap that is also claimed in, against
//     probed and claimed copies);
//   atomics of every workgroup on one address (a shared queue counter).
//
// Every index is masked into its buffer (table sizes are powers of two) or
// bounded by the element count, so each access stays in bounds.  Timing is by
// HIP events around the launch; results are written to `out` so that no load
// is dead.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint32_t xorshift(uint32_t x) {
  x ^= x << 13;
  x ^= x >> 17;
  x ^= x << 5;
  return x;
}

// iters x 8 loads per lane at pseudo-random indices in [0, mask].
__global__ __launch_bounds__(256) void random_loads(const uint32_t* __restrict__ table, uint32_t mask,
                                                    uint32_t iters, uint32_t* __restrict__ out) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t x = tid * 0x9E3779B9u + 0x7F4A7C15u;
  uint32_t acc = 0;
  for (uint32_t i = 0; i < iters; ++i) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x = xorshift(x);
      v[u] = table[x & mask];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  out[tid] = acc;
}

// The same with agent-scope (device-coherent) loads, as the kernels' checks of
// a copy that other workgroups update during a level.
__global__ __launch_bounds__(256) void random_coherent_loads(const uint32_t* __restrict__ table,
                                                             uint32_t mask, uint32_t iters,
                                                             uint32_t* __restrict__ out) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t x = tid * 0x9E3779B9u + 0x7F4A7C15u;
  uint32_t acc = 0;
  for (uint32_t i = 0; i < iters; ++i) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x = xorshift(x);
      v[u] = __hip_atomic_load(&table[x & mask], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  out[tid] = acc;
}

// Grid-stride sum of n int32 elements, 8 per lane per step.
__global__ __launch_bounds__(256) void stream_int(const int32_t* __restrict__ a, uint32_t n,
                                                  uint32_t* __restrict__ out) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t acc = 0;
  for (uint32_t i = tid; i < n; i += 8 * stride) {
    int32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t j = i + (uint32_t)u * stride;
      v[u] = j < n ? a[j] : 0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += (uint32_t)v[u];
  }
  out[tid] = acc;
}

// Grid-stride sum of n int4 elements, 4 per lane per step.
__global__ __launch_bounds__(256) void stream_int4(const int4* __restrict__ a, uint32_t n,
                                                   uint32_t* __restrict__ out) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t acc = 0;
  for (uint32_t i = tid; i < n; i += 4 * stride) {
    int4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t j = i + (uint32_t)u * stride;
      v[u] = j < n ? a[j] : make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc += (uint32_t)(v[u].x + v[u].y + v[u].z + v[u].w);
  }
  out[tid] = acc;
}

// Streaming read of n int32 elements, each followed by one probe of a table
// at the element's value (masked): the child body's col load and visited probe.
__global__ __launch_bounds__(256) void stream_probe(const int32_t* __restrict__ a, uint32_t n,
                                                    const uint32_t* __restrict__ table, uint32_t mask,
                                                    uint32_t* __restrict__ out) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t stride = gridDim.x * blockDim.x;
  uint32_t acc = 0;
  for (uint32_t i = tid; i < n; i += 8 * stride) {
    int32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t j = i + (uint32_t)u * stride;
      v[u] = j < n ? a[j] : 0;
    }
    uint32_t w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) w[u] = table[(uint32_t)v[u] & mask];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += w[u];
  }
  out[tid] = acc;
}

// iters x 8 atomicOr per lane on pseudo-random words of the table.
__global__ __launch_bounds__(256) void random_atomic_or(uint32_t* __restrict__ table, uint32_t mask,
                                                        uint32_t iters) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t x = tid * 0x9E3779B9u + 0x2545F491u;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x = xorshift(x);
      atomicOr(&table[x & mask], 1u << (x >> 27));
    }
  }
}

// The same, returning each old word (summed into out, so none is dead).
__global__ __launch_bounds__(256) void random_atomic_or_ret(uint32_t* __restrict__ table, uint32_t mask,
                                                            uint32_t iters, uint32_t* __restrict__ out) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t x = tid * 0x9E3779B9u + 0x2545F491u, acc = 0;
  for (uint32_t i = 0; i < iters; ++i) {
    uint32_t r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x = xorshift(x);
      r[u] = atomicOr(&table[x & mask], 1u << (x >> 27));
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += r[u];
  }
  out[tid] = acc;
}

// iters x 8 plain stores per lane at pseudo-random words of the table.
__global__ __launch_bounds__(256) void random_stores(uint32_t* __restrict__ table, uint32_t mask,
                                                     uint32_t iters) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t x = tid * 0x9E3779B9u + 0x68E31DA4u;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x = xorshift(x);
      table[x & mask] = x;
    }
  }
}

// Workgroups w with w % every == 0 run iters x 8 returning atomicOr on `at`
// (if mode & 2), the others iters x 8 loads of `lt` (if mode & 1); a part
// whose bit is clear returns at once.  `at` may be `lt` or another table of
// the same size.
__global__ __launch_bounds__(256) void loads_and_atomics(const uint32_t* __restrict__ lt,
                                                         uint32_t* __restrict__ at, uint32_t mask,
                                                         uint32_t iters, uint32_t every, uint32_t mode,
                                                         uint32_t* __restrict__ out) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const bool atom = blockIdx.x % every == 0;
  if (atom ? !(mode & 2u) : !(mode & 1u)) return;
  uint32_t x = tid * 0x9E3779B9u + 0x1B873593u, acc = 0;
  for (uint32_t i = 0; i < iters; ++i) {
    uint32_t r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x = xorshift(x);
      r[u] = atom ? atomicOr(&at[x & mask], 1u << (x >> 27)) : lt[x & mask];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += r[u];
  }
  out[tid] = acc;
}

// One lane per workgroup adds `iters` times to one of `naddr` counters
// (workgroup % naddr): same-address atomics serialise at the L2.
__global__ __launch_bounds__(64) void workgroup_atomics(uint32_t* __restrict__ ctr, uint32_t naddr,
                                                        uint32_t iters) {
  if (threadIdx.x != 0) return;
  uint32_t* c = ctr + (blockIdx.x % naddr) * 32;  // 128-byte apart
  for (uint32_t i = 0; i < iters; ++i) atomicAdd(c, 1u);
}

// The XCC (XCD) each workgroup runs on, from the hardware register, and the
// compute unit: out[2 * w] = XCC id, out[2 * w + 1] = HW_ID bits.
__global__ void workgroup_placement(uint32_t* __restrict__ out) {
  if (threadIdx.x != 0) return;
  uint32_t xcc, hw;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_HW_ID)" : "=s"(hw));
  out[2 * blockIdx.x] = xcc;
  out[2 * blockIdx.x + 1] = hw;
}

}  // namespace

extern "C" {

// out: device uint32[2 * grid].
int dpo_calib_workgroup_placement(int grid, int block, uint32_t* out, void* stream) {
  if (!out || grid < 1 || block < 1 || block > 1024) return -1;
  hipLaunchKernelGGL(workgroup_placement, dim3(grid), dim3(block), 0, (hipStream_t)stream, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}


// Each entry point launches one kernel on `stream` and returns 0, or -1 when
// the launch fails or an argument is outside what the kernel assumes.
// grid x 256 lanes; out: device uint32[grid * 256].  table_words a power of two.
int dpo_calib_random_loads(const uint32_t* table, uint32_t table_words, uint32_t iters, int grid,
                           uint32_t* out, void* stream) {
  if (!table || !out || grid < 1 || table_words == 0 || (table_words & (table_words - 1))) return -1;
  hipLaunchKernelGGL(random_loads, dim3(grid), dim3(256), 0, (hipStream_t)stream, table,
                     table_words - 1, iters, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int dpo_calib_random_coherent_loads(const uint32_t* table, uint32_t table_words, uint32_t iters,
                                    int grid, uint32_t* out, void* stream) {
  if (!table || !out || grid < 1 || table_words == 0 || (table_words & (table_words - 1))) return -1;
  hipLaunchKernelGGL(random_coherent_loads, dim3(grid), dim3(256), 0, (hipStream_t)stream, table,
                     table_words - 1, iters, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int dpo_calib_stream(const void* a, uint32_t n, int int4_elems, int grid, uint32_t* out,
                     void* stream) {
  if (!a || !out || grid < 1) return -1;
  if (int4_elems)
    hipLaunchKernelGGL(stream_int4, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const int4*)a, n,
                       out);
  else
    hipLaunchKernelGGL(stream_int, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const int32_t*)a,
                       n, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int dpo_calib_stream_probe(const int32_t* a, uint32_t n, const uint32_t* table, uint32_t table_words,
                           int grid, uint32_t* out, void* stream) {
  if (!a || !table || !out || grid < 1 || table_words == 0 || (table_words & (table_words - 1)))
    return -1;
  hipLaunchKernelGGL(stream_probe, dim3(grid), dim3(256), 0, (hipStream_t)stream, a, n, table,
                     table_words - 1, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int dpo_calib_random_atomic_or(uint32_t* table, uint32_t table_words, uint32_t iters, int grid,
                               void* stream) {
  if (!table || grid < 1 || table_words == 0 || (table_words & (table_words - 1))) return -1;
  hipLaunchKernelGGL(random_atomic_or, dim3(grid), dim3(256), 0, (hipStream_t)stream, table,
                     table_words - 1, iters);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// out: device uint32[grid * 256] (ret != 0 only).
int dpo_calib_random_atomic_or_ret(uint32_t* table, uint32_t table_words, uint32_t iters, int grid,
                                   uint32_t* out, void* stream) {
  if (!table || !out || grid < 1 || table_words == 0 || (table_words & (table_words - 1))) return -1;
  hipLaunchKernelGGL(random_atomic_or_ret, dim3(grid), dim3(256), 0, (hipStream_t)stream, table,
                     table_words - 1, iters, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int dpo_calib_random_stores(uint32_t* table, uint32_t table_words, uint32_t iters, int grid,
                            void* stream) {
  if (!table || grid < 1 || table_words == 0 || (table_words & (table_words - 1))) return -1;
  hipLaunchKernelGGL(random_stores, dim3(grid), dim3(256), 0, (hipStream_t)stream, table,
                     table_words - 1, iters);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// lt, at: device uint32[table_words] (may be the same buffer); out: device
// uint32[grid * 256]; every >= 1; mode in 1..3.
int dpo_calib_loads_and_atomics(const uint32_t* lt, uint32_t* at, uint32_t table_words,
                                uint32_t iters, uint32_t every, uint32_t mode, int grid,
                                uint32_t* out, void* stream) {
  if (!lt || !at || !out || grid < 1 || every < 1 || mode < 1 || mode > 3 || table_words == 0 ||
      (table_words & (table_words - 1)))
    return -1;
  hipLaunchKernelGGL(loads_and_atomics, dim3(grid), dim3(256), 0, (hipStream_t)stream, lt, at,
                     table_words - 1, iters, every, mode, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ctr: device uint32[naddr * 32].
int dpo_calib_workgroup_atomics(uint32_t* ctr, uint32_t naddr, uint32_t iters, int grid,
                                void* stream) {
  if (!ctr || naddr < 1 || grid < 1) return -1;
  hipLaunchKernelGGL(workgroup_atomics, dim3(grid), dim3(64), 0, (hipStream_t)stream, ctr, naddr,
                     iters);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // extern "C"

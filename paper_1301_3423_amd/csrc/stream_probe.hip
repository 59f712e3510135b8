// Streaming ceiling of the device: hand-written copy, read-only and
// write-only kernels over large buffers, timed with HIP events.  A
// measurement tool for the roofline discussion of the step kernels (what
// one MI355X streams in practice, against the nominal 8 TB/s); no part of
// the lattice Boltzmann method uses it.
//
// Every kernel moves 16-byte vectors, each thread keeping U of them in
// flight per pass of a grid-stride loop; NT selects non-temporal accesses.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace {

typedef float V __attribute__((ext_vector_type(4))); // 16 bytes

template <int U, bool NT>
__global__ void __launch_bounds__(256) k_copy(const V *__restrict__ src, V *__restrict__ dst, size_t n) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x * U;
  for (size_t base = static_cast<size_t>(blockIdx.x) * blockDim.x * U + threadIdx.x; base < n; base += stride) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = base + static_cast<size_t>(u) * blockDim.x;
      if (i < n) v[u] = NT ? __builtin_nontemporal_load(src + i) : src[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = base + static_cast<size_t>(u) * blockDim.x;
      if (i < n) {
        if (NT)
          __builtin_nontemporal_store(v[u], dst + i);
        else
          dst[i] = v[u];
      }
    }
  }
}

// Sums what it reads; one float per thread is written so that the loads
// stay (sink holds gridDim.x * blockDim.x floats).
template <int U>
__global__ void __launch_bounds__(256) k_read(const V *__restrict__ src, size_t n, float *__restrict__ sink) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x * U;
  float acc = 0.f;
  for (size_t base = static_cast<size_t>(blockIdx.x) * blockDim.x * U + threadIdx.x; base < n; base += stride) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = base + static_cast<size_t>(u) * blockDim.x;
      v[u] = i < n ? src[i] : V(0.f);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc += v[u].x + v[u].y + v[u].z + v[u].w;
  }
  sink[static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x] = acc;
}

template <int U>
__global__ void __launch_bounds__(256) k_write(V *__restrict__ dst, size_t n) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x * U;
  const V w = {1.f, 2.f, 3.f, 4.f};
  for (size_t base = static_cast<size_t>(blockIdx.x) * blockDim.x * U + threadIdx.x; base < n; base += stride) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t i = base + static_cast<size_t>(u) * blockDim.x;
      if (i < n) __builtin_nontemporal_store(w, dst + i);
    }
  }
}

template <int U>
void launch(int kind, const void *src, void *dst, size_t n, float *sink, unsigned grid, hipStream_t st) {
  const dim3 b(256), g(grid);
  if (kind == 0)
    k_copy<U, false><<<g, b, 0, st>>>(static_cast<const V *>(src), static_cast<V *>(dst), n);
  else if (kind == 1)
    k_copy<U, true><<<g, b, 0, st>>>(static_cast<const V *>(src), static_cast<V *>(dst), n);
  else if (kind == 2)
    k_read<U><<<g, b, 0, st>>>(static_cast<const V *>(src), n, sink);
  else
    k_write<U><<<g, b, 0, st>>>(static_cast<V *>(dst), n);
}

} // namespace

extern "C" {

// Times `reps` launches of one streaming kernel over `bytes` bytes (a
// multiple of 16) and returns the shortest launch in milliseconds, or a
// negative value on a HIP error or bad argument.
//   kind: 0 copy src -> dst, 1 copy with non-temporal loads and stores,
//         2 read src (sums into sink), 3 write dst (non-temporal);
//   unroll: 1, 2, 4 or 8 vectors in flight per thread;
//   grid: workgroups of 256 threads (grid-stride loops cover any size);
//   src, dst: device buffers of `bytes` (src unused by kind 3, dst by 2);
//   sink: device buffer of grid * 256 floats (kind 2 only);
//   stream: the HIP stream the kernels and events run on.
// The caller owns every buffer; nothing is allocated here.
double stream_probe_ms(int kind, int unroll, unsigned grid, const void *src, void *dst, float *sink,
                       size_t bytes, int reps, hipStream_t stream) {
  if (bytes == 0 || bytes % 16 || reps < 1 || grid == 0 || kind < 0 || kind > 3) return -1.0;
  if (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8) return -1.0;
  if ((kind != 3 && !src) || (kind != 2 && !dst) || (kind == 2 && !sink)) return -1.0;
  const size_t n = bytes / 16;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -2.0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -2.0;
  }
  double best = -3.0;
  for (int r = 0; r < reps; ++r) {
    if (hipEventRecord(e0, stream) != hipSuccess) break;
    switch (unroll) {
    case 1: launch<1>(kind, src, dst, n, sink, grid, stream); break;
    case 2: launch<2>(kind, src, dst, n, sink, grid, stream); break;
    case 4: launch<4>(kind, src, dst, n, sink, grid, stream); break;
    default: launch<8>(kind, src, dst, n, sink, grid, stream); break;
    }
    if (hipGetLastError() != hipSuccess || hipEventRecord(e1, stream) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess) {
      best = -2.0;
      break;
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      best = -2.0;
      break;
    }
    if (best < 0 || ms < best) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

} // extern "C"

// Measurement kernels for the benchmark (libsqmeasure.so, loaded by bench.py
// with ctypes; not part of the generator library):
//  - a store-only kernel in exactly the launch shape of the fills' default
//    configuration: one 4 KiB chunk per workgroup, 256 lanes, one 16-byte
//    global_store_dwordx4 per lane of constant data, so each wave store
//    covers one aligned KiB.  It is the HBM write ceiling of that shape.
//  - a clock sampler: one wave that records (shader clock counter, 100 MHz
//    real-time counter) pairs at a fixed real-time spacing, run on a side
//    stream while the benchmark's step runs, so the step's mean shader clock
//    is read from the ratio of the two counters.  It stops after a fixed
//    number of samples (its run time is samples x spacing / 100 MHz).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_store_chunk(unsigned char* out, uint32_t nchunks, uint32_t v) {
  const uint32_t c = blockIdx.x;
  if (c >= nchunks) return;
  u32x4 val;
  val.x = v;
  val.y = v + 1;
  val.z = v + 2;
  val.w = v + 3;
  *(u32x4*)(out + (uint64_t)c * 4096 + threadIdx.x * 16u) = val;
}

__global__ __launch_bounds__(64) void k_clock_sampler(uint64_t* samples, uint32_t count, uint64_t spacing) {
  if (threadIdx.x != 0) return;
  uint64_t next = wall_clock64();
  for (uint32_t i = 0; i < count; ++i) {
    while (wall_clock64() < next) __builtin_amdgcn_s_sleep(8);
    samples[2 * i] = clock64();
    samples[2 * i + 1] = wall_clock64();
    next += spacing;
  }
}

}  // namespace

extern "C" {

// Writes `bytes` (a multiple of 4096, at most 2^23 chunks per launch
// segment) of constant data at `out` (1 KiB aligned); returns a hipError_t.
int sqm_store_ceiling(void* out, uint64_t bytes, uint32_t v, void* stream) {
  if (((uintptr_t)out & 1023) != 0 || (bytes & 4095) != 0) return (int)hipErrorInvalidValue;
  uint64_t chunks = bytes >> 12;
  unsigned char* p = (unsigned char*)out;
  while (chunks) {
    const uint32_t seg = (uint32_t)(chunks < (1ull << 23) ? chunks : (1ull << 23));  // grid * 256 < 2^32
    hipLaunchKernelGGL(k_store_chunk, dim3(seg), dim3(256), 0, (hipStream_t)stream, p, seg, v);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    p += (uint64_t)seg << 12;
    chunks -= seg;
  }
  return (int)hipSuccess;
}

// Launches the sampler: `count` pairs (clock64, wall_clock64) into
// `samples` (device, 16 * count bytes), one every `spacing` ticks of the
// 100 MHz real-time counter.
int sqm_clock_sampler(uint64_t* samples, uint32_t count, uint64_t spacing, void* stream) {
  if (samples == nullptr || count == 0 || spacing == 0) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_clock_sampler, dim3(1), dim3(64), 0, (hipStream_t)stream, samples, count, spacing);
  return (int)hipGetLastError();
}

}  // extern "C"

// Calibration program: the two ceilings the Squares kernels are measured
// against on this GPU.
//  1. VALU issue rate per instruction class (lane-instructions per CU per
//     clock at the nominal 2.4 GHz), from long loops of independent chains,
//     with the shader clock read from clock64()/wall_clock64().
//  2. HBM write ceiling: store-only kernels (dwordx4 per lane) in the two
//     launch shapes the fills use -- grid-stride over block*8-vector chunks,
//     and one chunk of block*U vectors per workgroup -- and hipMemsetD32,
//     each over 16 GiB.
// Every kernel writes one value per thread into a buffer sized for the grid
// (or stores inside [0, bytes)); nothing reads uninitialised memory.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

#define CK(x)                                                                             \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess) {                                                               \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);          \
      std::exit(1);                                                                       \
    }                                                                                     \
  } while (0)

constexpr int CH = 8;  // independent chains per thread

template <int OP>
__global__ void k_rate(uint64_t* out, unsigned long long* clk, int iters, uint32_t seed) {
  uint32_t x[CH], y[CH];
  uint64_t w[CH];
  for (int j = 0; j < CH; ++j) {
    x[j] = seed + threadIdx.x * 7 + j * 131 + blockIdx.x;
    y[j] = x[j] * 3 + 1;
    w[j] = ((uint64_t)x[j] << 32) | y[j];
  }
  const unsigned long long c0 = clock64(), t0 = wall_clock64();
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      if (OP == 0) asm volatile("v_add_u32_e64 %0, %0, %1" : "+v"(x[j]) : "v"(y[j]));   // 32-bit add
      if (OP == 1) w[j] = (uint64_t)(uint32_t)w[j] * (uint32_t)w[j] + w[j];              // v_mad_u64_u32
      if (OP == 2) x[j] = x[j] * y[j];                                                   // v_mul_lo_u32
      if (OP == 3) w[j] = w[j] + (uint64_t)y[j];                                         // v_lshl_add_u64
      if (OP == 4) asm volatile("v_lshl_add_u32 %0, %0, 1, %1" : "+v"(x[j]) : "v"(y[j]));
      if (OP == 5) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x[j]) : "v"(y[j]));
      if (OP == 6) asm volatile("v_add_co_u32_e32 %0, vcc, %0, %1" : "+v"(x[j]) : "v"(y[j]) : "vcc");
      if (OP == 7) asm volatile("v_lshrrev_b32_e32 %0, 3, %0" : "+v"(x[j]));
      // the conversions and float ops read the registers' bits as whatever
      // they encode; only the issue rate is measured
      if (OP == 8) asm volatile("v_cvt_f32_u32_e32 %0, %0" : "+v"(x[j]));
      if (OP == 9) asm volatile("v_mul_f32_e32 %0, %0, %1" : "+v"(x[j]) : "v"(y[j]));
      if (OP == 10) asm volatile("v_cvt_f64_u32_e32 %0, %1" : "=v"(w[j]) : "v"(x[j]));
      if (OP == 11) asm volatile("v_fma_f64 %0, %0, %0, %0" : "+v"(w[j]));
    }
  }
  const unsigned long long c1 = clock64(), t1 = wall_clock64();
  uint64_t r = 0;
  for (int j = 0; j < CH; ++j) r ^= x[j] ^ w[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = r;
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = c1 - c0;
    clk[2 * blockIdx.x + 1] = t1 - t0;
  }
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__global__ void k_store(u32x4* out, uint64_t nchunks, uint32_t v) {
  const uint32_t B = blockDim.x;
  u32x4 val = {v ^ threadIdx.x, v, v + 1, v + 2};
  for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    u32x4* p = out + c * (uint64_t)B * 8 + threadIdx.x;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      val.y += 1;
      p[u * B] = val;
    }
  }
}

// One chunk of block*U vectors per workgroup (grid = chunks).
template <int U>
__global__ void k_store_chunk(u32x4* out, uint32_t v) {
  const uint32_t B = blockDim.x;
  u32x4 val = {v ^ threadIdx.x, v, v + 1, v + 2};
  u32x4* p = out + (uint64_t)blockIdx.x * B * U + threadIdx.x;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    val.y += 1;
    p[(uint64_t)u * B] = val;
  }
}

template <typename F>
static float best_ms(F f, int reps) {
  hipEvent_t a, b;
  CK(hipEventCreate(&a));
  CK(hipEventCreate(&b));
  f();
  CK(hipDeviceSynchronize());
  float best = 1e30f;
  for (int r = 0; r < reps; ++r) {
    CK(hipEventRecord(a));
    f();
    CK(hipEventRecord(b));
    CK(hipEventSynchronize(b));
    float ms;
    CK(hipEventElapsedTime(&ms, a, b));
    if (ms < best) best = ms;
  }
  CK(hipEventDestroy(a));
  CK(hipEventDestroy(b));
  return best;
}

template <int OP>
static void rate(const char* name, int cus, uint64_t* out, unsigned long long* clk, unsigned long long* hclk) {
  const int blocks = cus * 16, threads = 256, iters = 4096;  // 16 waves per SIMD
  const float ms = best_ms([&] { k_rate<OP><<<blocks, threads>>>(out, clk, iters, 3); }, 5);
  CK(hipMemcpy(hclk, clk, sizeof(unsigned long long) * 2 * blocks, hipMemcpyDeviceToHost));
  double ratio = 0;
  for (int i = 0; i < blocks; ++i) ratio += (double)hclk[2 * i] / (double)(hclk[2 * i + 1] ? hclk[2 * i + 1] : 1);
  ratio /= blocks;
  const double lane_instr = (double)blocks * threads * iters * CH;
  const double per_cu_clk = lane_instr / (ms * 1e-3) / (cus * 2.4e9);
  std::printf("| %-16s | %8.3f | %7.1f | %5.2f |\n", name, ms, per_cu_clk, ratio * 0.1);
}

int main() {
  hipDeviceProp_t p;
  CK(hipGetDeviceProperties(&p, 0));
  const int cus = p.multiProcessorCount;
  std::printf("device %s, %d CUs, nominal clock %d MHz\n\n", p.gcnArchName, cus, p.clockRate / 1000);
  uint64_t* out;
  unsigned long long *clk, *hclk;
  CK(hipMalloc(&out, (size_t)cus * 16 * 256 * 8));
  CK(hipMalloc(&clk, (size_t)cus * 16 * 16));
  hclk = (unsigned long long*)std::malloc((size_t)cus * 16 * 16);
  std::printf("| instruction      | ms       | lane-instr/CU/clk @2.4GHz | measured shader GHz |\n|---|---|---|---|\n");
  rate<0>("v_add_u32", cus, out, clk, hclk);
  rate<4>("v_lshl_add_u32", cus, out, clk, hclk);
  rate<1>("v_mad_u64_u32", cus, out, clk, hclk);
  rate<2>("v_mul_lo_u32", cus, out, clk, hclk);
  rate<3>("64-bit add", cus, out, clk, hclk);
  rate<5>("v_mul_hi_u32", cus, out, clk, hclk);
  rate<6>("v_add_co_u32", cus, out, clk, hclk);
  rate<7>("v_lshrrev_b32", cus, out, clk, hclk);
  rate<8>("v_cvt_f32_u32", cus, out, clk, hclk);
  rate<9>("v_mul_f32", cus, out, clk, hclk);
  rate<10>("v_cvt_f64_u32", cus, out, clk, hclk);
  rate<11>("v_fma_f64", cus, out, clk, hclk);
  CK(hipFree(out));
  CK(hipFree(clk));
  std::free(hclk);

  const size_t bytes = 16ull << 30;
  void* o;
  CK(hipMalloc(&o, bytes));
  std::printf("\n| store pattern (16 GiB) | ms | GB/s |\n|---|---|---|\n");
  for (int B : {256, 1024}) {
    for (int gpc : {4, 16}) {
      const uint64_t nch = bytes / 16 / ((uint64_t)B * 8);
      const int grid = cus * gpc;
      const float ms = best_ms([&] { k_store<<<grid, B>>>((u32x4*)o, nch, 7); }, 5);
      std::printf("| dwordx4 block %4d grid %5d | %7.3f | %7.1f |\n", B, grid, ms, bytes / (ms * 1e6));
    }
  }
  // one chunk per workgroup: 16 GiB / 16 B is a multiple of every B*U here,
  // so the grid covers the buffer exactly
  for (int B : {64, 256, 1024}) {
    const uint64_t nvec = bytes / 16;
    const float m1 = best_ms([&] { k_store_chunk<1><<<(uint32_t)(nvec / B), B>>>((u32x4*)o, 7); }, 5);
    std::printf("| dwordx4 one chunk/workgroup, block %4d x 1 vector | %7.3f | %7.1f |\n", B, m1, bytes / (m1 * 1e6));
    const float m4 = best_ms([&] { k_store_chunk<4><<<(uint32_t)(nvec / B / 4), B>>>((u32x4*)o, 7); }, 5);
    std::printf("| dwordx4 one chunk/workgroup, block %4d x 4 vectors | %7.3f | %7.1f |\n", B, m4, bytes / (m4 * 1e6));
  }
  const float ms = best_ms([&] { CK(hipMemsetD32((hipDeviceptr_t)o, 5, bytes / 4)); }, 5);
  std::printf("| hipMemsetD32 | %7.3f | %7.1f |\n", ms, bytes / (ms * 1e6));
  CK(hipFree(o));
  return 0;
}

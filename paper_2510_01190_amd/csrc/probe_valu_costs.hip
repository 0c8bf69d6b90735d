// Issue cost of the vector-ALU instruction classes on this GPU: shader-clock
// cycles per wave64 instruction per SIMD, for the classes the Monte Carlo
// kernel's counters separate (a simple 32-bit operation, a 32x32->64-bit
// integer multiply-add, a transcendental).  A standalone program, not part of
// libpdiv: it gives the per-class weights of the Monte Carlo kernel's ALU
// bound (instruction counts from rocprofv3 times these costs).
//
// Eight waves per SIMD (1024 SIMDs), each running 8 independent chains of the
// instruction under test for a fixed count.  Every wave records s_memtime at
// its start and end and its hardware place (XCC, shader engine, CU, SIMD);
// per SIMD the cost is (last end - first start) / (instructions issued on it),
// and the program prints the median over SIMDs as one JSON line.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <map>
#include <vector>

namespace {

constexpr int kIters = 2000;
constexpr int kChains = 8;
constexpr int kWavesPerSimd = 8;
constexpr int kBlock = 256;

enum Op { kXor = 0, kFma = 1, kMad64 = 2, kExp = 3, kSin = 4 };

template <int OP>
__global__ __launch_bounds__(kBlock) void issue_kernel(uint64_t* __restrict__ t,
                                                       uint32_t* __restrict__ where,
                                                       uint32_t seed) {
  uint32_t a[kChains];
  float f[kChains];
#pragma unroll
  for (int i = 0; i < kChains; ++i) {
    a[i] = seed + threadIdx.x * kChains + i;
    f[i] = 1.0f + 1e-7f * static_cast<float>(a[i]);
  }
  const uint32_t b = seed * 3u + 1u;
  const float g = 0.999f;
  __syncthreads();
  const uint64_t t0 = __builtin_amdgcn_s_memtime();
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
      if constexpr (OP == kXor) asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[i]) : "v"(b));
      if constexpr (OP == kFma)
        asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(f[i]) : "v"(g), "v"(f[(i + 1) % kChains]));
      if constexpr (OP == kMad64) {
        uint64_t p, carry;
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(p), "=s"(carry) : "v"(a[i]), "v"(b));
        a[i] = static_cast<uint32_t>(p >> 32);
      }
      if constexpr (OP == kExp) asm volatile("v_exp_f32 %0, %0" : "+v"(f[i]));
      if constexpr (OP == kSin) asm volatile("v_sin_f32 %0, %0" : "+v"(f[i]));
    }
  }
  const uint64_t t1 = __builtin_amdgcn_s_memtime();
  uint32_t hw, xcc;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_HW_ID)" : "=s"(hw));
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
  uint32_t acc = 0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) acc ^= a[i] ^ __float_as_uint(f[i]);
  const int w = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  if ((threadIdx.x & 63) == 0) {
    t[2 * w] = t0;
    t[2 * w + 1] = t1;
    where[2 * w] = hw;
    where[2 * w + 1] = xcc;
  }
  if (acc == 0x9e3779b9u) t[0] = acc;  // keeps the chains live
}

// Median over SIMDs of shader-clock cycles per wave instruction, or a
// negative value on a HIP error.
template <int OP>
double cost(int n_simds) {
  const int waves = n_simds * kWavesPerSimd;
  const int blocks = waves / (kBlock / 64);
  uint64_t* t = nullptr;
  uint32_t* where = nullptr;
  if (hipMalloc(&t, sizeof(uint64_t) * 2 * waves) != hipSuccess) return -1.0;
  if (hipMalloc(&where, sizeof(uint32_t) * 2 * waves) != hipSuccess) return -1.0;
  for (int rep = 0; rep < 2; ++rep)  // the first launch warms up the clocks
    hipLaunchKernelGGL(issue_kernel<OP>, dim3(blocks), dim3(kBlock), 0, 0, t, where, 7u);
  std::vector<uint64_t> ht(2 * waves);
  std::vector<uint32_t> hw(2 * waves);
  if (hipMemcpy(ht.data(), t, sizeof(uint64_t) * 2 * waves, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(hw.data(), where, sizeof(uint32_t) * 2 * waves, hipMemcpyDeviceToHost) !=
          hipSuccess)
    return -1.0;
  (void)hipFree(t);
  (void)hipFree(where);
  struct Span {
    uint64_t lo = ~0ull, hi = 0;
    int waves = 0;
  };
  std::map<uint64_t, Span> simd;
  for (int w = 0; w < waves; ++w) {
    const uint32_t id = hw[2 * w];
    // HW_ID: SIMD bits 5:4, CU 11:8, SH 12, SE 15:13
    const uint64_t key = (uint64_t(hw[2 * w + 1]) << 32) | (id & 0xFF30u);
    Span& s = simd[key];
    s.lo = std::min(s.lo, ht[2 * w]);
    s.hi = std::max(s.hi, ht[2 * w + 1]);
    s.waves += 1;
  }
  std::vector<double> c;
  for (const auto& kv : simd)
    c.push_back(double(kv.second.hi - kv.second.lo) /
                (double(kv.second.waves) * kIters * kChains));
  std::sort(c.begin(), c.end());
  return c.empty() ? -1.0 : c[c.size() / 2];
}

}  // namespace

int main() {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, 0) != hipSuccess) return 1;
  const int n_simds = p.multiProcessorCount * 4;
  const double x = cost<kXor>(n_simds), fm = cost<kFma>(n_simds), m = cost<kMad64>(n_simds),
               e = cost<kExp>(n_simds), s = cost<kSin>(n_simds);
  if (x < 0 || fm < 0 || m < 0 || e < 0 || s < 0) {
    std::fprintf(stderr, "probe failed\n");
    return 1;
  }
  std::printf(
      "{\"simds\": %d, \"waves_per_simd\": %d, \"cycles_per_wave_instruction_per_simd\": "
      "{\"v_xor_b32\": %.3f, \"v_fmac_f32\": %.3f, \"v_mad_u64_u32\": %.3f, \"v_exp_f32\": %.3f, "
      "\"v_sin_f32\": %.3f}}\n",
      n_simds, kWavesPerSimd, x, fm, m, e, s);
  return 0;
}

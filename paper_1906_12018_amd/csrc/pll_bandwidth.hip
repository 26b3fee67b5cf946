// Streaming-read reference kernel: the HBM read rate a plain, fully
// coalesced read of a large buffer reaches on this device.  It is the
// "achievable" bandwidth that the query kernel's rate is compared with (the
// query only reads labels and writes 4 bytes per pair).  Not part of the
// labeling method.
//
// Every lane reads 16-byte words with kUnroll independent loads in flight and
// folds them into an XOR so the loads cannot be dropped; each workgroup adds
// one atomic XOR of its folded value to the sink.
#include <hip/hip_runtime.h>

#include "pll_bench.h"
#include "pll_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kUnroll = 8;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(kBlock) k_stream_read(const u32x4* __restrict__ src, uint64_t words,
                                                        unsigned long long* __restrict__ sink) {
    const uint64_t total = (uint64_t)gridDim.x * kBlock;
    uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x;
    uint32_t acc = 0;
    // full rounds: kUnroll loads per lane, each a whole grid's width apart
    for (; i + (kUnroll - 1) * total < words; i += kUnroll * total) {
        u32x4 x[kUnroll];
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) x[k] = __builtin_nontemporal_load(src + i + k * total);
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) acc ^= x[k].x ^ x[k].y ^ x[k].z ^ x[k].w;
    }
    for (; i < words; i += total) {
        const u32x4 x = __builtin_nontemporal_load(src + i);
        acc ^= x.x ^ x.y ^ x.z ^ x.w;
    }
    for (int s = 32; s >= 1; s >>= 1) acc ^= (uint32_t)__shfl_xor((int)acc, s);
    __shared__ uint32_t s_acc[kBlock / 64];
    if ((threadIdx.x & 63) == 0) s_acc[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0;
        for (int w = 0; w < kBlock / 64; ++w) a ^= s_acc[w];
        atomicXor(sink, (unsigned long long)a);
    }
}

}  // namespace

extern "C" int pll_bench_stream_read(const void* d_buf, uint64_t bytes, uint64_t* d_sink, uint32_t workgroups,
                                     hipStream_t stream) {
    if (!d_buf || !d_sink || (bytes & 15) || (reinterpret_cast<uintptr_t>(d_buf) & 15)) return PLL_EINVAL;
    if (bytes == 0) return PLL_OK;
    if (workgroups == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_stream_read, kBlock, 0) != hipSuccess)
            return PLL_EDEVICE;
        workgroups = (uint32_t)(cus * (per_cu > 0 ? per_cu : 1));
    }
    k_stream_read<<<workgroups, kBlock, 0, stream>>>(static_cast<const u32x4*>(d_buf), bytes / 16,
                                                     reinterpret_cast<unsigned long long*>(d_sink));
    return hipGetLastError() == hipSuccess ? PLL_OK : PLL_EDEVICE;
}

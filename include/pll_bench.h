/*
 * pll_bench.h -- measurement helpers of libpll (not part of the labeling
 * method; used to put the kernels' rates beside what the device reaches).
 */
#ifndef PLL_BENCH_H_
#define PLL_BENCH_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Streaming read of `bytes` of device memory at d_buf (both multiples of 16;
 * PLL_EINVAL otherwise): every 16-byte word is read once, fully coalesced,
 * and the XOR of all words is XORed into d_sink[0] (uint64, device) so the
 * reads cannot be elided.  `workgroups` sets the grid (256 threads each);
 * 0 = as many as fit on the device at once.  Asynchronous on `stream`; time
 * it with events on that stream.  The caller owns both buffers; a buffer far
 * larger than the last-level cache (256 MB on MI355X) measures HBM.  This is
 * the achievable read bandwidth the query kernel's rate is compared with.
 */
int pll_bench_stream_read(const void* d_buf, uint64_t bytes, uint64_t* d_sink, uint32_t workgroups,
                          hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PLL_BENCH_H_ */

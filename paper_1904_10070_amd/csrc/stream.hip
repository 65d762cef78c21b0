// stream.hip -- HBM streaming reference kernels (include/tlb_stream.h): the copy, 2-read/1-write
// and read-only rates that bound the stage kernel of tlb.hip on this GPU.
//
// One dwordx4 per lane and access, nontemporal.  The launch shapes are the fastest of a sweep on
// 2 GiB buffers (persistent grid-stride grids of 4-32 workgroups per compute unit with 1, 2 or 4
// chunks per lane and round, against one-shot grids; cached against nontemporal accesses).

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "tlb.h"
#include "tlb_internal.h"
#include "tlb_stream.h"

namespace {

constexpr int STREAM_THREADS = 256;
constexpr int READ_BLOCKS_PER_CU = 8;
constexpr int MAX_READ_BLOCKS = 8192;

typedef float v4f __attribute__((ext_vector_type(4)));
__device__ __forceinline__ v4f ld(const v4f* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st(v4f* p, v4f v) { __builtin_nontemporal_store(v, p); }

// copy (MODE 0) and add (MODE 1): one chunk per lane and one workgroup per 256 chunks, so that
// the grid is many short workgroups walking the buffers in address order (measured faster
// than a persistent grid-stride loop for both, by 5-30 %)
template <int MODE>
__global__ __launch_bounds__(STREAM_THREADS) void tlb_stream_kernel(const v4f* __restrict__ x,
                                                                   const v4f* __restrict__ y,
                                                                   v4f* __restrict__ z,
                                                                   long long n) {
  const long long i = (long long)blockIdx.x * STREAM_THREADS + threadIdx.x;
  if (i >= n) return;
  v4f a = ld(x + i);
  if constexpr (MODE == 1) a += ld(y + i);
  st(z + i, a);
}

// read (MODE 2): a grid-stride loop over a resident grid (8 workgroups per compute unit), the
// sum kept per lane; one 16-byte partial per workgroup goes to z so that no load is dead
__global__ __launch_bounds__(STREAM_THREADS) void tlb_stream_read_kernel(
    const v4f* __restrict__ x, v4f* __restrict__ z, long long n) {
  const long long stride = (long long)gridDim.x * STREAM_THREADS;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (long long i = (long long)blockIdx.x * STREAM_THREADS + threadIdx.x; i < n; i += stride)
    acc += ld(x + i);
  __shared__ v4f part[STREAM_THREADS / 64];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    acc.x += __shfl_xor(acc.x, d, 64);
    acc.y += __shfl_xor(acc.y, d, 64);
    acc.z += __shfl_xor(acc.z, d, 64);
    acc.w += __shfl_xor(acc.w, d, 64);
  }
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    v4f s = part[0];
    for (int w = 1; w < STREAM_THREADS / 64; ++w) s += part[w];
    z[blockIdx.x] = s;
  }
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

extern "C" int32_t tlb_hbm_stream(int32_t mode, const void* x, const void* y, void* z,
                                  int64_t n16, void* hip_stream) {
  if (mode < 0 || mode > 2) return tlbi_fail(TLB_EINVAL, "unknown stream mode");
  if (n16 < 1) return tlbi_fail(TLB_EINVAL, "n16 must be >= 1");
  if (!x || !z || (mode == 1 && !y)) return tlbi_fail(TLB_EINVAL, "a buffer is NULL");
  if (!aligned16(x) || !aligned16(z) || (mode == 1 && !aligned16(y)))
    return tlbi_fail(TLB_EINVAL, "buffers must be 16-byte aligned");
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return tlbi_fail(TLB_EHIP, std::string("device query: ") + hipGetErrorString(e));
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const v4f* xx = static_cast<const v4f*>(x);
  const v4f* yy = static_cast<const v4f*>(y);
  v4f* zz = static_cast<v4f*>(z);
  const long long blocks = (n16 + STREAM_THREADS - 1) / STREAM_THREADS;
  if (mode == 2) {
    long long rb = (long long)cus * READ_BLOCKS_PER_CU;
    if (rb > blocks) rb = blocks;
    if (rb > MAX_READ_BLOCKS) rb = MAX_READ_BLOCKS;
    hipLaunchKernelGGL(tlb_stream_read_kernel, dim3((unsigned)rb), dim3(STREAM_THREADS), 0, s, xx,
                       zz, (long long)n16);
  } else {
    if (blocks > 0x7FFFFFFFLL) return tlbi_fail(TLB_EINVAL, "n16 too large for one launch");
    if (mode == 0)
      hipLaunchKernelGGL(tlb_stream_kernel<0>, dim3((unsigned)blocks), dim3(STREAM_THREADS), 0, s,
                         xx, yy, zz, (long long)n16);
    else
      hipLaunchKernelGGL(tlb_stream_kernel<1>, dim3((unsigned)blocks), dim3(STREAM_THREADS), 0, s,
                         xx, yy, zz, (long long)n16);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return tlbi_fail(TLB_EHIP, std::string("stream launch: ") + hipGetErrorString(e));
  return TLB_OK;
}

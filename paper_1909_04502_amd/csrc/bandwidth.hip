// bandwidth.hip -- copy kernels that measure the memory ceiling the step kernels are held to.
//
// The step kernels read Q population planes at a site and write Q planes back, one thread per site
// and one element per plane.  "site" copies Q planes with exactly that pattern and no arithmetic
// (all loads of a thread issued before its stores, as in the fused update), so its bandwidth is what
// the population layout allows; "flat" copies the same bytes as 16-byte vectors over a grid that
// fills the chip, the plain streaming ceiling of the part.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/rlbm.h"

namespace {

template <bool NT, typename S>
__device__ __forceinline__ void put(S *p, S v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <int Q, typename S, bool NT>
__global__ void __launch_bounds__(256) k_copy_site(const S *__restrict__ src, S *__restrict__ dst, int64_t sites) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= sites) return;
  S v[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) v[i] = src[(int64_t)i * sites + s];
#pragma unroll
  for (int i = 0; i < Q; ++i) put<NT>(dst + (int64_t)i * sites + s, v[i]);
}

// each thread moves kVec 16-byte vectors, kVec * blockDim apart within its block's chunk
constexpr int kVec = 4;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ void __launch_bounds__(256) k_copy_flat(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * blockDim.x * kVec + threadIdx.x;
  u32x4 v[kVec];
#pragma unroll
  for (int k = 0; k < kVec; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i < n) v[k] = src[i];
  }
#pragma unroll
  for (int k = 0; k < kVec; ++k) {
    const int64_t i = base + (int64_t)k * blockDim.x;
    if (i < n) put<NT>(dst + i, v[k]);
  }
}

template <int Q, typename S>
hipError_t launch_site(const void *src, void *dst, int64_t sites, int nt, hipStream_t stream) {
  const dim3 grid((unsigned)((sites + 255) / 256)), block(256);
  if (nt)
    hipLaunchKernelGGL((k_copy_site<Q, S, true>), grid, block, 0, stream, (const S *)src, (S *)dst, sites);
  else
    hipLaunchKernelGGL((k_copy_site<Q, S, false>), grid, block, 0, stream, (const S *)src, (S *)dst, sites);
  return hipGetLastError();
}

}  // namespace

extern "C" rlbm_status rlbm_copy_planes(const void *src, void *dst, int64_t sites, int32_t planes,
                                        int32_t elem_bytes, int32_t mode, int32_t nontemporal, hipStream_t stream) {
  if (!src || !dst || sites < 1 || (elem_bytes != 4 && elem_bytes != 8) || (nontemporal != 0 && nontemporal != 1))
    return RLBM_ERR_INVALID_ARG;
  const int64_t bytes = sites * planes * (int64_t)elem_bytes;
  const char *ps = (const char *)src, *pd = (const char *)dst;
  if (ps < pd + bytes && pd < ps + bytes) return RLBM_ERR_INVALID_ARG;
  hipError_t he = hipSuccess;
  if (mode == 0) {
    if (planes == 32) he = elem_bytes == 8 ? launch_site<32, double>(src, dst, sites, nontemporal, stream)
                                           : launch_site<32, float>(src, dst, sites, nontemporal, stream);
    else if (planes == 104) he = elem_bytes == 8 ? launch_site<104, double>(src, dst, sites, nontemporal, stream)
                                                 : launch_site<104, float>(src, dst, sites, nontemporal, stream);
    else return RLBM_ERR_UNSUPPORTED;
  } else if (mode == 1) {
    if (bytes % 16 != 0 || ((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return RLBM_ERR_INVALID_ARG;
    const int64_t n = bytes / 16;
    const dim3 grid((unsigned)((n + 256 * kVec - 1) / (256 * kVec))), block(256);
    if (nontemporal)
      hipLaunchKernelGGL((k_copy_flat<true>), grid, block, 0, stream, (const u32x4 *)src, (u32x4 *)dst, n);
    else
      hipLaunchKernelGGL((k_copy_flat<false>), grid, block, 0, stream, (const u32x4 *)src, (u32x4 *)dst, n);
    he = hipGetLastError();
  } else {
    return RLBM_ERR_INVALID_ARG;
  }
  return he == hipSuccess ? RLBM_OK : RLBM_ERR_DEVICE;
}

// Memory-bandwidth reference with the access pattern of the collide-stream
// step: q population arrays copied element by element, each thread reading
// its element of every array and then writing all of them, with the same
// streaming hints.  No arithmetic and no neighbour shifts: the rate it
// reaches is what the step's loads and stores can reach on this device.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "lattice_kernels.hpp"
#include "lbm.h"
#include "lbm_internal.hpp"

namespace lbm {

template <class T, int Q, bool NT>
__global__ __launch_bounds__(256) void k_stream_copy(const T* __restrict__ src, T* __restrict__ dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    T v[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) v[k] = ld<T, NT>(src + (int64_t)k * n + i);
#pragma unroll
    for (int k = 0; k < Q; ++k) st<T, NT>(dst + (int64_t)k * n + i, v[k]);
}

template <class T>
static void stream_copy_t(const void* src, void* dst, int64_t n, int q, bool nt, hipStream_t st)
{
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    const T* a = (const T*)src;
    T* b = (T*)dst;
    if (q == 19) {
        if (nt) hipLaunchKernelGGL((k_stream_copy<T, 19, true>), grid, block, 0, st, a, b, n);
        else hipLaunchKernelGGL((k_stream_copy<T, 19, false>), grid, block, 0, st, a, b, n);
    } else {
        if (nt) hipLaunchKernelGGL((k_stream_copy<T, 27, true>), grid, block, 0, st, a, b, n);
        else hipLaunchKernelGGL((k_stream_copy<T, 27, false>), grid, block, 0, st, a, b, n);
    }
}

} // namespace lbm

extern "C" {

int lbm_stream_copy(const void* src, void* dst, int64_t n, int32_t q, int32_t elem_bytes, int32_t nt, void* stream)
{
    char msg[160];
    if (!src || !dst || n < 0 || (q != 19 && q != 27) || (elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8)) {
        std::snprintf(msg, sizeof msg, "lbm_stream_copy: bad arguments (n %lld, q %d, elem_bytes %d)", (long long)n,
                      (int)q, (int)elem_bytes);
        lbm_internal_set_error(msg);
        return LBM_EINVAL;
    }
    if ((n + 255) / 256 > 0x7fffffffLL) {
        lbm_internal_set_error("lbm_stream_copy: n exceeds the launch grid");
        return LBM_EINVAL;
    }
    if (n == 0) return LBM_OK;
    const hipStream_t st = (hipStream_t)stream;
    switch (elem_bytes) {
    case 2: lbm::stream_copy_t<uint16_t>(src, dst, n, q, nt != 0, st); break;
    case 4: lbm::stream_copy_t<uint32_t>(src, dst, n, q, nt != 0, st); break;
    default: lbm::stream_copy_t<uint64_t>(src, dst, n, q, nt != 0, st); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        std::snprintf(msg, sizeof msg, "lbm_stream_copy: %s", hipGetErrorString(e));
        lbm_internal_set_error(msg);
        return LBM_EDEVICE;
    }
    return LBM_OK;
}

} // extern "C"

// Memory-bandwidth reference with the access pattern of the collide-stream
// step: q population arrays copied element by element, each thread reading
// its element of every array and then writing all of them, with the same
// streaming hints.  No arithmetic and no neighbour shifts: the rate it
// reaches is what the step's loads and stores can reach on this device.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

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

// Wider accesses: each thread copies W consecutive bytes of every array
// (W = 8 or 16, a multiple of the element size); the arrays are nb bytes
// long, nb a multiple of W.
template <int W> struct Chunk;
template <> struct Chunk<8> { using T = uint64_t; };
template <> struct Chunk<16> { using T = __attribute__((ext_vector_type(4))) uint32_t; };

template <int W, int Q, bool NT>
__global__ __launch_bounds__(256) void k_stream_copy_wide(const char* __restrict__ src, char* __restrict__ dst,
                                                          int64_t nb)
{
    using T = typename Chunk<W>::T;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= nb / W) return;
    T v[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        const T* p = reinterpret_cast<const T*>(src + k * nb) + c;
        v[k] = NT ? __builtin_nontemporal_load(p) : *p;
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
        T* p = reinterpret_cast<T*>(dst + k * nb) + c;
        if (NT)
            __builtin_nontemporal_store(v[k], p);
        else
            *p = v[k];
    }
}

// The step kernels' cap on resident wavefronts per SIMD (by LDS allocation;
// LBM_WAVES_PER_SIMD, default five for 4- and 8-byte elements, none for
// 2-byte ones), applied to the reference too: dynamic LDS per work-group.
static unsigned copy_lds(int elem_bytes)
{
    const char* env = std::getenv("LBM_WAVES_PER_SIMD");
    const int waves = env ? std::atoi(env) : (elem_bytes >= 4 ? 5 : 0);
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess || lds <= 0)
        lds = 163840;
    return occ_pad(waves, lds, 0, dim3(256));
}

template <class T>
static void stream_copy_t(const void* src, void* dst, int64_t n, int q, bool nt, hipStream_t st)
{
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    const unsigned pad = copy_lds((int)sizeof(T));
    const T* a = (const T*)src;
    T* b = (T*)dst;
    if (q == 19) {
        if (nt) hipLaunchKernelGGL((k_stream_copy<T, 19, true>), grid, block, pad, st, a, b, n);
        else hipLaunchKernelGGL((k_stream_copy<T, 19, false>), grid, block, pad, st, a, b, n);
    } else {
        if (nt) hipLaunchKernelGGL((k_stream_copy<T, 27, true>), grid, block, pad, st, a, b, n);
        else hipLaunchKernelGGL((k_stream_copy<T, 27, false>), grid, block, pad, st, a, b, n);
    }
}

template <int W>
static void stream_copy_w(const void* src, void* dst, int64_t nb, int q, bool nt, int elem_bytes, hipStream_t st)
{
    const dim3 grid((unsigned)((nb / W + 255) / 256)), block(256);
    const unsigned pad = copy_lds(elem_bytes);
    const char* a = (const char*)src;
    char* b = (char*)dst;
    if (q == 19) {
        if (nt) hipLaunchKernelGGL((k_stream_copy_wide<W, 19, true>), grid, block, pad, st, a, b, nb);
        else hipLaunchKernelGGL((k_stream_copy_wide<W, 19, false>), grid, block, pad, st, a, b, nb);
    } else {
        if (nt) hipLaunchKernelGGL((k_stream_copy_wide<W, 27, true>), grid, block, pad, st, a, b, nb);
        else hipLaunchKernelGGL((k_stream_copy_wide<W, 27, false>), grid, block, pad, st, a, b, nb);
    }
}

} // namespace lbm

extern "C" {

int lbm_stream_copy(const void* src, void* dst, int64_t n, int32_t q, int32_t elem_bytes, int32_t lane_bytes,
                    int32_t nt, void* stream)
{
    char msg[200];
    if (lane_bytes == 0) lane_bytes = elem_bytes;
    const bool lanes_ok = lane_bytes == elem_bytes || ((lane_bytes == 8 || lane_bytes == 16) && lane_bytes > elem_bytes);
    if (!src || !dst || n < 0 || (q != 19 && q != 27) || (elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8) ||
        !lanes_ok || (n * elem_bytes) % lane_bytes != 0) {
        std::snprintf(msg, sizeof msg, "lbm_stream_copy: bad arguments (n %lld, q %d, elem_bytes %d, lane_bytes %d)",
                      (long long)n, (int)q, (int)elem_bytes, (int)lane_bytes);
        lbm_internal_set_error(msg);
        return LBM_EINVAL;
    }
    if ((n * elem_bytes / lane_bytes + 255) / 256 > 0x7fffffffLL) {
        lbm_internal_set_error("lbm_stream_copy: n exceeds the launch grid");
        return LBM_EINVAL;
    }
    if (n == 0) return LBM_OK;
    const hipStream_t st = (hipStream_t)stream;
    if (lane_bytes == elem_bytes) {
        switch (elem_bytes) {
        case 2: lbm::stream_copy_t<uint16_t>(src, dst, n, q, nt != 0, st); break;
        case 4: lbm::stream_copy_t<uint32_t>(src, dst, n, q, nt != 0, st); break;
        default: lbm::stream_copy_t<uint64_t>(src, dst, n, q, nt != 0, st); break;
        }
    } else if (lane_bytes == 8) {
        lbm::stream_copy_w<8>(src, dst, n * elem_bytes, q, nt != 0, elem_bytes, st);
    } else {
        lbm::stream_copy_w<16>(src, dst, n * elem_bytes, q, nt != 0, elem_bytes, st);
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

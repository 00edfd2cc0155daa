// Final, deterministic reduction of per-block FP64 diagnostic partials.
#include "lbm_internal.hpp"

namespace lbm {

namespace {
constexpr int NDIAG = NDIAG_OUT;
__device__ inline double combine(int k, double a, double b) { return k == 5 ? fmax(a, b) : (k == 7 ? fmin(a, b) : a + b); }
} // namespace

// One block: thread t folds partials t, t+256, ... in order, then a fixed tree;
// the first nout totals are written.
__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ partials, int nblocks,
                                                         double* __restrict__ out, int nout)
{
    __shared__ double lds[NDIAG][256];
    const int t = threadIdx.x;
    double v[NDIAG] = {0, 0, 0, 0, 0, 0, 0, 1e300};
    for (int b = t; b < nblocks; b += 256) {
        const double* p = partials + (int64_t)b * NDIAG;
        for (int k = 0; k < NDIAG; ++k) v[k] = combine(k, v[k], p[k]);
    }
    for (int k = 0; k < NDIAG; ++k) lds[k][t] = v[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int k = 0; k < NDIAG; ++k) lds[k][t] = combine(k, lds[k][t], lds[k][t + w]);
        __syncthreads();
    }
    if (t == 0)
        for (int k = 0; k < nout; ++k) out[k] = lds[k][0];
}

void launch_reduce(const double* partials, int nblocks, double* out, hipStream_t st, int nout)
{
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, st, partials, nblocks, out, nout);
}

} // namespace lbm

// Host side of the C ABI declared in include/lbm.h.
#include "lbm.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <algorithm>
#include <vector>

#include "d3q19_cm.hpp"
#include "handle.hpp"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                                 \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            return fail(e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "%s: %s (%s:%d)", #expr, \
                        hipGetErrorString(e_), __FILE__, __LINE__);                                   \
    } while (0)

int elem_bytes(int precision) { return precision == LBM_FP64 ? 8 : (precision == LBM_FP32 ? 4 : 2); }

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

} // namespace

void lbm_internal_set_error(const char* msg)
{
    std::snprintf(g_err, sizeof g_err, "%s", msg);
}

int lbm_fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}


namespace {

int pattern_of(const lbm_handle* h)
{
    if (h->p.streaming == LBM_AB) return 0;
    return (h->steps & 1) ? 2 : 1;
}

int validate(const lbm_params* p)
{
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (p->abi_version != LBM_ABI_VERSION)
        return fail(LBM_EINVAL, "abi_version %u != %d", p->abi_version, LBM_ABI_VERSION);
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(LBM_EINVAL, "lattice size must be positive");
    if ((int64_t)p->nx * p->ny * p->nz > 0x7fffffffLL) return fail(LBM_EINVAL, "more than 2^31-1 nodes");
    if (p->nz > 65535) return fail(LBM_EINVAL, "nz > 65535");
    if (p->q != 19 && p->q != 27) return fail(LBM_EINVAL, "q must be 19 or 27 (got %d)", p->q);
    if (p->precision < LBM_FP64 || p->precision > LBM_BF16_SHIFTED) return fail(LBM_EINVAL, "bad precision");
    if (p->streaming != LBM_AB && p->streaming != LBM_AA) return fail(LBM_EINVAL, "bad streaming");
    auto rate_ok = [](double w) { return std::isfinite(w) && w > 0.0 && w < 2.0; };
    if (!rate_ok(p->omega)) return fail(LBM_EINVAL, "omega must be in (0,2) (got %g)", p->omega);
    if (!rate_ok(p->omega_bulk)) return fail(LBM_EINVAL, "omega_bulk must be in (0,2)");
    for (int j = 0; j < 9; ++j)
        if (!(std::isfinite(p->omega_hi[j]) && p->omega_hi[j] > 0.0 && p->omega_hi[j] <= 2.0))
            return fail(LBM_EINVAL, "omega_hi[%d] must be in (0,2]", j);
    if (!(std::isfinite(p->rho0) && p->rho0 > 0.0)) return fail(LBM_EINVAL, "rho0 must be positive");
    if (p->force_mode < LBM_FORCE_NONE || p->force_mode > LBM_FORCE_KOLMOGOROV) return fail(LBM_EINVAL, "bad force_mode");
    if (p->force_mode == LBM_FORCE_FIELD && !p->force_field) return fail(LBM_EINVAL, "force_field is NULL");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(p->force[d])) return fail(LBM_EINVAL, "force must be finite");
    if (!std::isfinite(p->kolmogorov_amp)) return fail(LBM_EINVAL, "kolmogorov_amp must be finite");
    if (p->walls_y != 0 && p->walls_y != 1) return fail(LBM_EINVAL, "walls_y must be 0 or 1");
    if (p->walls_y && p->ny < 2) return fail(LBM_EINVAL, "walls need ny >= 2");
    if (p->check_every < 0) return fail(LBM_EINVAL, "check_every must be >= 0");
    if (p->block_x < 0 || p->block_y < 0) return fail(LBM_EINVAL, "negative block shape");
    if (p->cache_policy < 0 || p->cache_policy > 2) return fail(LBM_EINVAL, "cache_policy must be 0, 1 or 2");
    if (p->q == 27) {
        if (p->precision != LBM_FP64 && p->precision != LBM_FP32)
            return fail(LBM_EUNSUPPORTED, "D3Q27 supports FP64 and FP32 storage");
        bool paper_rates = p->omega_bulk == 1.0;
        for (int j = 0; j < 9; ++j) paper_rates = paper_rates && p->omega_hi[j] == 1.0;
        if (!paper_rates)
            return fail(LBM_EUNSUPPORTED, "D3Q27 relaxes every non-shear moment at rate 1 (omega_bulk/omega_hi)");
    }
    const int bx = p->block_x ? p->block_x : 64, by = p->block_y ? p->block_y : 1;
    if (bx * by > 256 || (bx * by) % 64 != 0)
        return fail(LBM_EINVAL, "block_x*block_y must be a multiple of 64 and at most 256");
    if (p->moments != LBM_CENTRAL_MOMENTS && p->moments != LBM_RAW_MOMENTS) return fail(LBM_EINVAL, "bad moments");
    if (p->moments == LBM_RAW_MOMENTS && p->coupled != LBM_COUPLED_NONE)
        return fail(LBM_EUNSUPPORTED, "raw moments: no coupled lattice");
    if (p->coupled < LBM_COUPLED_NONE || p->coupled > LBM_COUPLED_COLOUR) return fail(LBM_EINVAL, "bad coupled");
    if (p->rounding != LBM_ROUND_NEAREST && p->rounding != LBM_ROUND_STOCHASTIC) return fail(LBM_EINVAL, "bad rounding");
    if (p->rounding == LBM_ROUND_STOCHASTIC &&
        (p->precision != LBM_BF16_SHIFTED || p->q != 19 || p->moments != LBM_CENTRAL_MOMENTS ||
         p->coupled != LBM_COUPLED_NONE))
        return fail(LBM_EUNSUPPORTED, "stochastic rounding: D3Q19 central moments with BF16 storage, no coupled lattice");
    if (p->coupled != LBM_COUPLED_NONE) return coupled_validate(p);
    return LBM_OK;
}

int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Default work-group shape: 256 threads covering whole x-rows where possible;
// narrow lattices pack several rows per block.
void default_block(const lbm_params* p, int& bx, int& by)
{
    if (p->block_x && p->block_y) {
        bx = p->block_x;
        by = p->block_y;
        return;
    }
    // one block per x-row (up to 256 nodes): measured fastest at 256^3.  A
    // row shorter than 256 nodes whose length is not a power of two: whole
    // rows per work-group when some number of them fills whole wavefronts
    // (48 x 4, 96 x 2, 192 x 1: no idle lane, and the rows can be staged);
    // rows longer than 256 nodes: row_width
    const int nx = p->nx;
    if (nx < 256 && (nx & (nx - 1)) != 0)
        for (int k = 256 / nx; k >= 1; --k)
            if (nx * k % 64 == 0) {
                bx = nx;
                by = k;
                return;
            }
    bx = nx <= 256 ? next_pow2(nx) : lbm::row_width(nx);
    if (bx < 8) bx = 8;
    by = 256 / bx;
    const int ny2 = next_pow2(p->ny);
    while (by > 1 && by / 2 >= ny2 && bx * (by / 2) >= 64) by /= 2;
}

// Row staging of the x-moving populations through LDS: possible for a
// periodic lattice with work-groups spanning whole rows, in the A-B step and
// the AA odd step (the AA even step is local).  On by default wherever it is
// possible: with the scalar-base addressing it is the tuner's choice at 256^3
// for every storage type, A-B and AA, and it keeps HBM traffic at the
// algorithmic bytes (direct x-shifted accesses fetched 16-38 % more); the
// tuner may choose either; LBM_ROW_STAGING=0 turns it off, =1 on wherever it
// is possible (both override the default and the tuner).
void set_row_stage(lbm_handle* h)
{
    const char* env = std::getenv("LBM_ROW_STAGING");
    const bool allowed = !(env && env[0] == '0') && (h->p.streaming == LBM_AB || h->p.streaming == LBM_AA) &&
                         !h->walls && (int)h->step_block.x == h->g.nx;
    const bool want = (env && env[0] == '1') || h->row_stage_pref < 0 || h->row_stage_pref == 1;
    h->g.row_stage = allowed && want;
    // a 512-wide step work-group exists only for the staged kernels: without
    // staging the step falls back to 256-thread work-groups over the rows,
    // with an x width that divides the row where one does (no idle lanes)
    if (h->step_block.x > 256 && !h->g.row_stage) {
        const int nx = h->g.nx, wx = lbm::row_width(nx);
        h->step_block = dim3(wx, 256 / wx, 1);
        h->step_grid = dim3((nx + wx - 1) / wx, (h->g.ny + 256 / wx - 1) / (256 / wx), h->g.nz);
    }
}

// Can one work-group of nx threads span each row (257..1024 nodes) with
// staging?  Periodic A-B / AA, the 3-D grid (no XCD remap), and the staged
// rows of the x-moving populations (kernels for rows up to 512 or up to 1024)
// within 64 KB of LDS.
bool wide_rows_possible(const lbm_handle* h)
{
    const int qx = h->p.q == 27 ? 18 : 10;
    const int w = h->g.nx <= 512 ? 512 : 1024;
    return h->g.nx > 256 && h->g.nx <= 1024 && !h->walls && h->g.xcd_chunk == 1 &&
           (h->p.streaming == LBM_AB || h->p.streaming == LBM_AA) &&
           (int64_t)qx * w * elem_bytes(h->p.precision) <= 65536;
}

int64_t pad_stride(int64_t N, int eb)
{
    // Separate the starts of consecutive population arrays by a non-power-of-two
    // number of 256-byte blocks so the streams of one step spread over channels.
    // 68 x 256 B for 4- and 8-byte elements, 102 x 256 B for 2-byte ones
    // (256^3, alternating runs on one machine: FP16 A-B 0.724 -> 0.737 of
    // 8 TB/s, BF16 A-B 0.725 -> 0.731, AA within noise; FP32 A-B with
    // 102 x 256 B: 0.732 against 0.740)
    const char* env = std::getenv("LBM_PAD_BYTES");
    int64_t pad_bytes = env ? std::atoll(env) : (eb == 2 ? 26112 : 17408);
    int64_t base = round_up(N * eb, 4096);
    return (base + pad_bytes) / eb;
}

int run_check(lbm_handle* h)
{
    lbm::launch_moments(h->p.q, h->kprec, pattern_of(h), h->walls, h->buf[h->cur], h->g, h->ph, nullptr, nullptr,
                        h->partials, h->grid, h->block, h->stream);
    lbm::launch_reduce(h->partials, h->nblocks, h->diag_dev, h->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h->diag_host, h->diag_dev, lbm::NDIAG_OUT * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

} // namespace

extern "C" {

void lbm_params_default(lbm_params* p)
{
    std::memset(p, 0, sizeof *p);
    p->abi_version = LBM_ABI_VERSION;
    p->nx = p->ny = p->nz = 32;
    p->q = 19;
    p->precision = LBM_FP32;
    p->streaming = LBM_AB;
    p->omega = 1.0;
    p->omega_bulk = 1.0;
    for (int j = 0; j < 9; ++j) p->omega_hi[j] = 1.0;
    p->rho0 = 1.0;
    p->force_mode = LBM_FORCE_NONE;
}

int lbm_abi_version(void) { return LBM_ABI_VERSION; }

const char* lbm_last_error(void) { return g_err; }

int lbm_create(const lbm_params* p, void* stream, lbm_handle** out)
{
    g_err[0] = 0;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(p);
    if (rc) return rc;
    lbm_handle* h = new lbm_handle();
    h->p = *p;
    h->kprec = p->rounding == LBM_ROUND_STOCHASTIC ? lbm::PREC_BF16SR : p->precision;
    h->stream = (hipStream_t)stream;
    auto cleanup = [&](int code) {
        lbm_destroy(h);
        return code;
    };
    if (hipGetDevice(&h->device) != hipSuccess) return cleanup(fail(LBM_EDEVICE, "no HIP device"));
    const int eb = elem_bytes(p->precision);
    h->g.nx = p->nx;
    h->g.ny = p->ny;
    h->g.nz = p->nz;
    h->g.nxy = p->nx * p->ny;
    h->g.N = p->nx * p->ny * p->nz;
    h->g.stride = pad_stride(h->g.N, eb);
    // 32-bit element offsets while every population array is below 4 GiB;
    // LBM_OFF32=0 keeps 64-bit addressing (the path of larger lattices)
    {
        const char* env = std::getenv("LBM_OFF32");
        h->g.off32 = h->g.stride * eb < ((int64_t)1 << 32) && !(env && env[0] == '0');
    }
    // AA even step with 16-bit storage: loads without the streaming hint up
    // to 2^25 nodes (measured faster there, slower beyond); LBM_AA_EVEN_CACHED
    // =0/1 forces either
    {
        const char* env = std::getenv("LBM_AA_EVEN_CACHED");
        const bool want = env ? env[0] == '1' : h->g.N <= (1 << 25);
        h->g.even_cached = eb == 2 && want;
    }
    // step kernels with 4- and 8-byte storage: at most five resident
    // wavefronts per SIMD (by LDS allocation).  At 256^3, A-B, one machine:
    // FP32 0.737 -> 0.769 of 8 TB/s (seven waves -> five; four the same,
    // three 0.762), raw moments 0.723 -> 0.745, FP64 0.707 -> 0.722 (six
    // waves -> five); 16-bit storage keeps every wave it can hold (eight:
    // FP16 0.734, with five 0.67).  LBM_WAVES_PER_SIMD=n sets the cap (0:
    // none).
    {
        const char* env = std::getenv("LBM_WAVES_PER_SIMD");
        h->g.occ_waves = env ? std::atoi(env) : (eb >= 4 ? 5 : 0);
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, h->device) == hipSuccess &&
            lds > 0)
            h->g.lds_per_cu = lds;
    }
    h->walls = p->walls_y != 0;
    // default: streaming hints for A-B with 4- and 8-byte storage and for
    // every staged step (set below), ordinary accesses otherwise -- the
    // tuner's choices at 256^3
    if (p->cache_policy == 0)
        h->nt = p->streaming == LBM_AB && eb >= 4;
    else
        h->nt = p->cache_policy == 1;
    h->general = p->omega_bulk != 1.0;
    for (int j = 0; j < 9; ++j) h->general = h->general || p->omega_hi[j] != 1.0;

    h->ph.omega = p->omega;
    h->ph.omega_bulk = p->omega_bulk;
    for (int j = 0; j < 9; ++j) h->ph.omega_hi[j] = p->omega_hi[j];
    h->ph.rho0 = p->rho0;
    h->ph.force_mode = lbm::FORCE_NONE;
    for (int d = 0; d < 3; ++d) h->ph.force[d] = p->force[d];
    h->ph.force_field = nullptr;
    h->ph.row_table = nullptr;

    int bx, by;
    default_block(p, bx, by);
    h->block = dim3(bx, by, 1);
    h->grid = dim3((p->nx + bx - 1) / bx, (p->ny + by - 1) / by, p->nz);
    h->nblocks = h->grid.x * h->grid.y * h->grid.z;
    // step kernels: LBM_XCD_CHUNK=c > 1 launches one 1-D grid of the same
    // blocks permuted so that each XCD sweeps runs of c consecutive rows.
    // Measured at 256^3 (A-B, c = 2..64 and one contiguous range per XCD):
    // FP32 within +-0.5 %, FP16 shifted 12-17 % slower, so the default keeps
    // the 3-D grid and the hardware's round-robin order.
    {
        const char* env = std::getenv("LBM_XCD_CHUNK");
        const int chunk = env ? std::atoi(env) : 1;
        const bool remap = chunk > 1 && h->nblocks % (8 * chunk) == 0;
        h->g.xcd_chunk = remap ? chunk : 1;
        h->step_grid = remap ? dim3(h->nblocks, 1, 1) : h->grid;
        h->step_block = h->block;
        set_row_stage(h);
        // rows of 257..1024 nodes: one work-group of nx threads per row,
        // staged (unless LBM_ROW_STAGING=0).  FP16 A-B against direct reads
        // on 256-thread work-groups: 0.685 / 0.49 of 8 TB/s at 320^3, 0.68 /
        // 0.51 at 384^3, 0.70 / 0.62 at 512^3, 0.66 / 0.65 at 1024 x 128^2
        if (!remap && wide_rows_possible(h)) {
            const char* rs = std::getenv("LBM_ROW_STAGING");
            const bool want = !(rs && rs[0] == '0');
            if (want) {
                h->step_block = dim3(h->g.nx, 1, 1);
                h->step_grid = dim3(1, h->g.ny, h->g.nz);
                set_row_stage(h);
            }
        }
        if (p->cache_policy == 0 && h->g.row_stage) h->nt = true;
    }

    const int64_t pop_bytes = (int64_t)p->q * h->g.stride * eb;
    const int nbuf = p->streaming == LBM_AB ? 2 : 1;
    for (int b = 0; b < nbuf; ++b) {
        hipError_t e = hipMalloc(&h->buf[b], pop_bytes);
        if (e != hipSuccess)
            return cleanup(fail(LBM_ENOMEM, "population buffer of %lld bytes: %s", (long long)pop_bytes, hipGetErrorString(e)));
        h->bytes += pop_bytes;
    }
    if (hipMalloc((void**)&h->partials, (int64_t)h->nblocks * lbm::NDIAG_OUT * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&h->diag_dev, lbm::NDIAG_OUT * sizeof(double)) != hipSuccess ||
        hipHostMalloc((void**)&h->diag_host, lbm::NDIAG_OUT * sizeof(double), hipHostMallocDefault) != hipSuccess)
        return cleanup(fail(LBM_ENOMEM, "diagnostic buffers"));
    h->bytes += (int64_t)(h->nblocks + 1) * lbm::NDIAG_OUT * sizeof(double);

    switch (p->force_mode) {
    case LBM_FORCE_UNIFORM: h->ph.force_mode = lbm::FORCE_UNIFORM; break;
    case LBM_FORCE_FIELD:
        h->ph.force_mode = lbm::FORCE_FIELD;
        h->ph.force_field = p->force_field;
        break;
    case LBM_FORCE_KOLMOGOROV: {
        h->ph.force_mode = lbm::FORCE_ROW_TABLE;
        double* tab = (double*)std::malloc(sizeof(double) * p->ny);
        const double two_pi = 6.283185307179586476925286766559;
        for (int y = 0; y < p->ny; ++y) tab[y] = p->kolmogorov_amp * std::sin(two_pi * y / p->ny);
        hipError_t e = hipMalloc((void**)&h->row_table, sizeof(double) * p->ny);
        if (e == hipSuccess) e = hipMemcpy(h->row_table, tab, sizeof(double) * p->ny, hipMemcpyHostToDevice);
        std::free(tab);
        if (e != hipSuccess) return cleanup(fail(LBM_EDEVICE, "force table: %s", hipGetErrorString(e)));
        h->ph.row_table = h->row_table;
        h->bytes += sizeof(double) * p->ny;
        break;
    }
    default: break;
    }
    if (p->coupled != LBM_COUPLED_NONE) {
        const int crc = coupled_create(h);
        if (crc) return cleanup(crc);
    }
    *out = h;
    return LBM_OK;
}

int lbm_destroy(lbm_handle* h)
{
    if (!h) return LBM_OK;
    if (h->stream || h->buf[0]) hipStreamSynchronize(h->stream);
    if (h->cp) coupled_destroy(h);
    if (h->fb_partials) hipFree(h->fb_partials);
    for (int b = 0; b < 2; ++b)
        if (h->buf[b]) hipFree(h->buf[b]);
    if (h->row_table) hipFree(h->row_table);
    if (h->partials) hipFree(h->partials);
    if (h->diag_dev) hipFree(h->diag_dev);
    if (h->diag_host) hipHostFree(h->diag_host);
    delete h;
    return LBM_OK;
}

int lbm_init(lbm_handle* h, const double* rho, const double* u, int on_device)
{
    if (!h || !rho || !u) return fail(LBM_EINVAL, "NULL argument");
    if (h->cp && h->p.coupled != LBM_COUPLED_SHAN_CHEN)
        return fail(LBM_EINVAL, "a coupled lattice starts from its own init call (lbm_init_phase)");
    const int64_t N = h->g.N;
    const double* drho = rho;
    const double* du = u;
    double* staging = nullptr;
    if (!on_device) {
        HIP_TRY(hipMalloc((void**)&staging, sizeof(double) * 4 * N));
        HIP_TRY(hipMemcpyAsync(staging, rho, sizeof(double) * N, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipMemcpyAsync(staging + N, u, sizeof(double) * 3 * N, hipMemcpyHostToDevice, h->stream));
        drho = staging;
        du = staging + N;
    }
    h->steps = 0;
    h->cur = 0;
    lbm::launch_init(h->p.q, h->kprec, pattern_of(h), h->walls, h->buf[h->cur], h->g, h->p.rho0, drho, du, h->grid,
                     h->block, h->stream);
    hipError_t e = hipGetLastError();
    if (staging) {
        hipStreamSynchronize(h->stream);
        hipFree(staging);
    }
    if (e != hipSuccess) return fail(LBM_EDEVICE, "init kernel: %s", hipGetErrorString(e));
    return LBM_OK;
}

int lbm_step(lbm_handle* h, int64_t nsteps)
{
    if (!h) return fail(LBM_EINVAL, "NULL handle");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
    for (int64_t s = 0; s < nsteps; ++s) {
        const int pat = pattern_of(h);
        const int src = h->cur;
        const int dst = h->p.streaming == LBM_AB ? 1 - h->cur : h->cur;
        if (h->cp) {
            const int crc = coupled_step(h);
            if (crc) return crc;
            h->cur = dst;
            h->steps++;
            if (h->p.check_every > 0 && h->steps % h->p.check_every == 0) {
                double d[6];
                const int mrc = coupled_moments(h, nullptr, nullptr, d, 1);
                if (mrc) return mrc;
                if (!(h->diag_host[6] == 0.0 && std::isfinite(d[0]) && h->diag_host[7] > 0.0))
                    return fail(LBM_EUNSTABLE, "unstable at step %lld: %g bad nodes", (long long)h->steps,
                                h->diag_host[6]);
            }
            continue;
        }
        if (h->mlp)
            lbm::launch_step_mlp(h->p.precision, pat, h->walls, h->nt, h->buf[src], h->buf[dst], h->g, h->ph,
                                 h->mlp->packed, h->fb_partials, h->grid, h->block, h->stream);
        else
        {
            // stochastic rounding: a new key per step (seed and step count hashed)
            if (h->kprec == lbm::PREC_BF16SR) h->ph.sr_key = lbm::hash32(h->p.seed ^ lbm::hash32((uint32_t)h->steps));
            lbm::launch_step(h->p.q, h->p.moments == LBM_RAW_MOMENTS, h->kprec, pat, h->walls, h->general, h->nt,
                             h->buf[src], h->buf[dst], h->g, h->ph, h->step_grid, h->step_block, h->stream);
        }
        h->cur = dst;
        h->steps++;
        if (h->p.check_every > 0 && h->steps % h->p.check_every == 0) {
            int rc = run_check(h);
            if (rc) return rc;
            const double* d = h->diag_host;
            if (!(d[6] == 0.0 && std::isfinite(d[0]) && d[7] > 0.0))
                return fail(LBM_EUNSTABLE, "unstable at step %lld: %g bad nodes, sum rho = %g, min rho = %g",
                            (long long)h->steps, d[6], d[0], d[7]);
        }
    }
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

int lbm_moments(lbm_handle* h, double* rho, double* u, double* diag, int on_device)
{
    if (!h) return fail(LBM_EINVAL, "NULL handle");
    if (h->cp) return coupled_moments(h, rho, u, diag, on_device);
    const int64_t N = h->g.N;
    double* drho = rho;
    double* du = u;
    double* staging = nullptr;
    if (!on_device && (rho || u)) {
        HIP_TRY(hipMalloc((void**)&staging, sizeof(double) * 4 * N));
        drho = rho ? staging : nullptr;
        du = u ? staging + N : nullptr;
    }
    lbm::launch_moments(h->p.q, h->kprec, pattern_of(h), h->walls, h->buf[h->cur], h->g, h->ph, drho, du, h->partials,
                        h->grid, h->block, h->stream);
    if (diag) lbm::launch_reduce(h->partials, h->nblocks, h->diag_dev, h->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && staging) {
        if (rho) e = hipMemcpyAsync(rho, staging, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess && u) e = hipMemcpyAsync(u, staging + N, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, h->stream);
    }
    if (e == hipSuccess && diag)
        e = hipMemcpyAsync(h->diag_host, h->diag_dev, lbm::NDIAG_OUT * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && (diag || staging)) e = hipStreamSynchronize(h->stream);
    if (staging) hipFree(staging);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "moments: %s", hipGetErrorString(e));
    if (diag)
        for (int k = 0; k < 6; ++k) diag[k] = h->diag_host[k];
    return LBM_OK;
}

int lbm_get_populations(lbm_handle* h, double* f, int on_device)
{
    if (!h || !f) return fail(LBM_EINVAL, "NULL argument");
    const int64_t bytes = sizeof(double) * h->p.q * (int64_t)h->g.N;
    double* dst = f;
    if (!on_device) HIP_TRY(hipMalloc((void**)&dst, bytes));
    lbm::launch_get_pops(h->p.q, h->kprec, pattern_of(h), h->walls, h->buf[h->cur], h->g, h->p.rho0, dst, h->grid,
                         h->block, h->stream);
    hipError_t e = hipGetLastError();
    if (!on_device) {
        if (e == hipSuccess) e = hipMemcpyAsync(f, dst, bytes, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        hipFree(dst);
    }
    if (e != hipSuccess) return fail(LBM_EDEVICE, "get_populations: %s", hipGetErrorString(e));
    return LBM_OK;
}

int lbm_set_populations(lbm_handle* h, const double* f, int on_device)
{
    if (!h || !f) return fail(LBM_EINVAL, "NULL argument");
    const int64_t bytes = sizeof(double) * h->p.q * (int64_t)h->g.N;
    const double* src = f;
    double* staging = nullptr;
    if (!on_device) {
        HIP_TRY(hipMalloc((void**)&staging, bytes));
        HIP_TRY(hipMemcpyAsync(staging, f, bytes, hipMemcpyHostToDevice, h->stream));
        src = staging;
    }
    lbm::launch_set_pops(h->p.q, h->kprec, pattern_of(h), h->walls, h->buf[h->cur], h->g, h->p.rho0, src, h->grid,
                         h->block, h->stream);
    hipError_t e = hipGetLastError();
    if (staging) {
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        hipFree(staging);
    }
    if (e != hipSuccess) return fail(LBM_EDEVICE, "set_populations: %s", hipGetErrorString(e));
    return LBM_OK;
}

int64_t lbm_step_count(const lbm_handle* h) { return h ? h->steps : -1; }

int32_t lbm_step_variant(const lbm_handle* h)
{
    if (!h) return -1;
    return h->g.row_stage ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Autotuner of the plain step: work-group shape x cache policy
// ---------------------------------------------------------------------------
namespace {

struct TuneEntry {
    std::string arch;
    int nx, ny, nz, q, moments, precision, streaming, walls, general;
    int bx, by, nt, rs;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune_cache; // process-wide: (GPU arch, lattice, variant) -> launch

void apply_launch(lbm_handle* h, int bx, int by, bool nt, int rs)
{
    h->step_block = dim3(bx, by, 1);
    h->step_grid = dim3((h->g.nx + bx - 1) / bx, (h->g.ny + by - 1) / by, h->g.nz);
    h->g.xcd_chunk = 1;
    h->nt = nt;
    h->row_stage_pref = rs;
    set_row_stage(h);
}

} // namespace

int lbm_tune(lbm_handle* h, int32_t trial_steps, int32_t* block_x, int32_t* block_y, int32_t* cache_policy,
             int32_t* row_stage)
{
    if (!h || trial_steps < 0) return fail(LBM_EINVAL, "bad arguments");
    if (h->cp || h->mlp) return fail(LBM_EUNSUPPORTED, "the tuner sets up the plain step (no coupled lattice or network)");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, h->device));
    TuneEntry key{prop.gcnArchName, h->g.nx, h->g.ny, h->g.nz, h->p.q, h->p.moments, h->kprec,
                  h->p.streaming, h->walls ? 1 : 0, h->general ? 1 : 0, 0, 0, 0, 0};
    auto same = [&](const TuneEntry& e) {
        return e.arch == key.arch && e.nx == key.nx && e.ny == key.ny && e.nz == key.nz && e.q == key.q &&
               e.moments == key.moments &&
               e.precision == key.precision && e.streaming == key.streaming && e.walls == key.walls &&
               e.general == key.general;
    };
    bool cached = false;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        for (const TuneEntry& e : g_tune_cache)
            if (same(e)) {
                key = e;
                cached = true;
            }
    }
    if (!cached) {
        const int steps = trial_steps + (trial_steps & 1);
        const int shapes[][2] = {{1024, 1}, {256, 1}, {128, 2}, {64, 4}, {128, 1}, {64, 2}, {64, 1}};
        const int nx2 = next_pow2(h->g.nx), ny2 = next_pow2(h->g.ny);
        const bool wide_ok = wide_rows_possible(h);
        struct Cand {
            int bx, by, nt, rs;
            float ms;
        };
        std::vector<Cand> cands;
        for (const auto& sh : shapes) {
            // the wide entry: one work-group of nx threads per row (257..1024), staged only
            if (sh[0] > 256 && !wide_ok) continue;
            // skip shapes that would leave most of a work-group idle
            if (sh[0] <= 256 && ((sh[0] > 64 && sh[0] > nx2) || (sh[1] > 1 && sh[1] > ny2))) continue;
            const int bx = sh[0] > 256 ? h->g.nx : sh[0];
            for (int c = 0; c < 4; ++c) {
                const int nt = c & 1 ? 0 : 1, rs = c >> 1 ? 0 : 1;
                if (bx > 256 && rs == 0) continue;
                apply_launch(h, bx, sh[1], nt != 0, rs);
                if (rs == 1 && !h->g.row_stage) continue; // staging not possible with this shape
                cands.push_back({bx, sh[1], nt, h->g.row_stage ? 1 : 0, 1e30f});
            }
        }

        hipEvent_t a, b;
        HIP_TRY(hipEventCreate(&a));
        HIP_TRY(hipEventCreate(&b));
        // three interleaved rounds, each candidate's fastest round counts:
        // one slow sample (a clock or neighbour transient) does not decide
        for (int round = 0; round < 3; ++round)
            for (Cand& c : cands) {
                apply_launch(h, c.bx, c.by, c.nt != 0, c.rs);
                int rc = lbm_step(h, 2);
                if (rc) return rc;
                HIP_TRY(hipEventRecord(a, h->stream));
                rc = lbm_step(h, steps);
                if (rc) return rc;
                HIP_TRY(hipEventRecord(b, h->stream));
                HIP_TRY(hipEventSynchronize(b));
                float ms = 0.0f;
                HIP_TRY(hipEventElapsedTime(&ms, a, b));
                c.ms = std::min(c.ms, ms);
            }
        float best = 1e30f;
        for (const Cand& c : cands)
            if (c.ms < best) {
                best = c.ms;
                key.bx = c.bx;
                key.by = c.by;
                key.nt = c.nt;
                key.rs = c.rs;
            }
        hipEventDestroy(a);
        hipEventDestroy(b);
        if (best == 1e30f) return fail(LBM_EINVAL, "no candidate work-group shape fits the lattice");
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache.push_back(key);
    }
    apply_launch(h, key.bx, key.by, key.nt != 0, key.rs);
    if (block_x) *block_x = key.bx;
    if (block_y) *block_y = key.by;
    if (cache_policy) *cache_policy = key.nt ? 1 : 2;
    if (row_stage) *row_stage = h->g.row_stage;
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// Learned rates
// ---------------------------------------------------------------------------
int lbm_mlp_destroy(lbm_mlp* m)
{
    if (!m) return LBM_OK;
    hipStreamSynchronize(m->stream);
    void* bufs[] = {m->theta, m->m1, m->m2, m->grad, m->inv_scale, m->packed, m->inv_sigma, m->gbuf, m->traj,
                    m->grad_parts, m->loss_parts, m->loss_dev, m->red_tmp, m->isig_steps, m->loss_steps,
                    m->energies, m->energy_parts};
    for (void* b : bufs)
        if (b) hipFree(b);
    if (m->loss_host) hipHostFree(m->loss_host);
    if (m->loss_steps_host) hipHostFree(m->loss_steps_host);
    delete m;
    return LBM_OK;
}

static int mlp_repack(lbm_mlp* m)
{
    lbm::launch_mlp_pack(m->theta, m->inv_scale, m->packed, m->stream);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

int lbm_mlp_create(const float* params, const float* scales, void* stream, lbm_mlp** out)
{
    g_err[0] = 0;
    if (!out || !scales) return fail(LBM_EINVAL, "NULL argument");
    *out = nullptr;
    for (int j = 0; j < 11; ++j)
        if (!(std::isfinite(scales[j]) && scales[j] > 0.0f)) return fail(LBM_EINVAL, "scales must be positive");
    if (params)
        for (int p = 0; p < LBM_MLP_NPARAM; ++p)
            if (!std::isfinite(params[p])) return fail(LBM_EINVAL, "non-finite parameter %d", p);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(LBM_EDEVICE, "no HIP device");
    lbm_mlp* m = new lbm_mlp();
    m->stream = (hipStream_t)stream;
    const size_t pb = sizeof(float) * LBM_MLP_NPARAM;
    if (hipMalloc((void**)&m->theta, pb) != hipSuccess || hipMalloc((void**)&m->m1, pb) != hipSuccess ||
        hipMalloc((void**)&m->m2, pb) != hipSuccess ||
        hipMalloc((void**)&m->grad, sizeof(double) * LBM_MLP_NPARAM) != hipSuccess ||
        hipMalloc((void**)&m->inv_scale, sizeof(float) * 16) != hipSuccess ||
        hipMalloc(&m->packed, lbm::mlp_packed_bytes()) != hipSuccess ||
        hipMalloc((void**)&m->inv_sigma, sizeof(float) * 10) != hipSuccess ||
        hipMalloc((void**)&m->loss_dev, sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&m->red_tmp, lbm::reduce_grad_tmp_bytes()) != hipSuccess ||
        hipHostMalloc((void**)&m->loss_host, sizeof(double), hipHostMallocDefault) != hipSuccess) {
        lbm_mlp_destroy(m);
        return fail(LBM_ENOMEM, "network buffers");
    }
    float inv[16] = {0};
    for (int j = 0; j < 11; ++j) inv[j] = 1.0f / scales[j];
    hipError_t e = hipMemcpyAsync(m->inv_scale, inv, sizeof inv, hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) e = params ? hipMemcpyAsync(m->theta, params, pb, hipMemcpyHostToDevice, m->stream)
                                    : hipMemsetAsync(m->theta, 0, pb, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->m1, 0, pb, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->m2, 0, pb, m->stream);
    if (e == hipSuccess) e = hipMemsetAsync(m->grad, 0, sizeof(double) * LBM_MLP_NPARAM, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) {
        lbm_mlp_destroy(m);
        return fail(LBM_EDEVICE, "network upload: %s", hipGetErrorString(e));
    }
    int rc = mlp_repack(m);
    if (rc) {
        lbm_mlp_destroy(m);
        return rc;
    }
    *out = m;
    return LBM_OK;
}

int lbm_mlp_set_params(lbm_mlp* m, const float* params)
{
    if (!m || !params) return fail(LBM_EINVAL, "NULL argument");
    const size_t pb = sizeof(float) * LBM_MLP_NPARAM;
    HIP_TRY(hipMemcpyAsync(m->theta, params, pb, hipMemcpyHostToDevice, m->stream));
    HIP_TRY(hipMemsetAsync(m->m1, 0, pb, m->stream));
    HIP_TRY(hipMemsetAsync(m->m2, 0, pb, m->stream));
    m->adam_t = 0;
    int rc = mlp_repack(m);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(m->stream));
    return LBM_OK;
}

int lbm_mlp_get_params(const lbm_mlp* m, float* params)
{
    if (!m || !params) return fail(LBM_EINVAL, "NULL argument");
    HIP_TRY(hipMemcpyAsync(params, m->theta, sizeof(float) * LBM_MLP_NPARAM, hipMemcpyDeviceToHost, m->stream));
    HIP_TRY(hipStreamSynchronize(m->stream));
    return LBM_OK;
}

int lbm_mlp_set_scales(lbm_mlp* m, const float* scales)
{
    if (!m || !scales) return fail(LBM_EINVAL, "NULL argument");
    float inv[16] = {0};
    for (int j = 0; j < 11; ++j) {
        if (!(std::isfinite(scales[j]) && scales[j] > 0.0f)) return fail(LBM_EINVAL, "scales must be positive");
        inv[j] = 1.0f / scales[j];
    }
    HIP_TRY(hipMemcpyAsync(m->inv_scale, inv, sizeof inv, hipMemcpyHostToDevice, m->stream));
    int rc = mlp_repack(m);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(m->stream));
    return LBM_OK;
}

int lbm_set_mlp(lbm_handle* h, const lbm_mlp* m)
{
    if (!h) return fail(LBM_EINVAL, "NULL handle");
    if (m) {
        if (h->cp) return fail(LBM_EUNSUPPORTED, "learned rates apply to the single-phase lattice");
        if (h->p.q != 19) return fail(LBM_EUNSUPPORTED, "learned rates need the D3Q19 lattice");
        if (h->p.moments != LBM_CENTRAL_MOMENTS)
            return fail(LBM_EUNSUPPORTED, "learned rates act on central moments");
        if (h->p.precision == LBM_FP64) return fail(LBM_EUNSUPPORTED, "learned rates run with FP32 collision");
        if (h->p.rounding != LBM_ROUND_NEAREST) return fail(LBM_EUNSUPPORTED, "learned rates store to nearest");
        if (!h->fb_partials) {
            HIP_TRY(hipMalloc((void**)&h->fb_partials, sizeof(uint32_t) * h->nblocks));
            h->bytes += sizeof(uint32_t) * h->nblocks;
        }
        HIP_TRY(hipMemsetAsync(h->fb_partials, 0, sizeof(uint32_t) * h->nblocks, h->stream));
        // the network's uploads are ordered on its own stream
        HIP_TRY(hipStreamSynchronize(m->stream));
    }
    h->mlp = m;
    return LBM_OK;
}

int64_t lbm_fallback_count(lbm_handle* h)
{
    if (!h || !h->fb_partials) return 0;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(LBM_EDEVICE, "sync");
    uint32_t* host = (uint32_t*)std::malloc(sizeof(uint32_t) * h->nblocks);
    if (!host) return fail(LBM_ENOMEM, "host buffer");
    int64_t total = -1;
    if (hipMemcpy(host, h->fb_partials, sizeof(uint32_t) * h->nblocks, hipMemcpyDeviceToHost) == hipSuccess) {
        total = 0;
        for (int b = 0; b < h->nblocks; ++b) total += host[b];
    }
    std::free(host);
    return total < 0 ? fail(LBM_EDEVICE, "copy") : total;
}

int lbm_mlp_zero_grad(lbm_mlp* m)
{
    if (!m) return fail(LBM_EINVAL, "NULL argument");
    HIP_TRY(hipMemsetAsync(m->grad, 0, sizeof(double) * LBM_MLP_NPARAM, m->stream));
    return LBM_OK;
}

static int grow(void** p, int64_t& have, int64_t need, size_t elem)
{
    if (have >= need) return LBM_OK;
    if (*p) hipFree(*p);
    *p = nullptr;
    have = 0;
    if (hipMalloc(p, elem * need) != hipSuccess) return fail(LBM_ENOMEM, "training scratch");
    have = need;
    return LBM_OK;
}

// Shared checks of the training entry points; fills the inverse moment scales
// 1 / (sigma_k sqrt(steps)).
static int training_checks(lbm_mlp* m, lbm_handle* h, const double sigma[10], int steps, float isig[10])
{
    if (h->mlp != m) return fail(LBM_EINVAL, "the network must be attached to the handle (lbm_set_mlp)");
    if (h->p.q != 19 || h->p.precision != LBM_FP32 || h->p.streaming != LBM_AB || h->walls ||
        h->p.force_mode != LBM_FORCE_NONE || h->p.moments != LBM_CENTRAL_MOMENTS)
        return fail(LBM_EUNSUPPORTED, "training needs a periodic, force-free D3Q19 FP32 A-B lattice");
    for (int k = 0; k < 10; ++k) {
        if (!(std::isfinite(sigma[k]) && sigma[k] > 0.0)) return fail(LBM_EINVAL, "sigma must be positive");
        isig[k] = (float)(1.0 / (sigma[k] * std::sqrt((double)steps)));
    }
    return LBM_OK;
}

int lbm_mlp_accumulate_grad(lbm_mlp* m, lbm_handle* h, const float* target, const double sigma[10], double* loss)
{
    if (!m || !h || !target || !sigma) return fail(LBM_EINVAL, "NULL argument");
    float isig[10];
    int rc = training_checks(m, h, sigma, 1, isig);
    if (rc) return rc;
    const lbm::Geom& g = h->g;
    const int nwb = ((g.nx + 63) / 64) * g.ny * g.nz; // backward: one wavefront per block
    rc = grow((void**)&m->gbuf, m->gbuf_elems, (int64_t)2 * 19 * g.N, sizeof(float));
    if (!rc) rc = grow((void**)&m->grad_parts, m->grad_parts_n, (int64_t)nwb * LBM_MLP_NPARAM, sizeof(float));
    if (!rc) rc = grow((void**)&m->loss_parts, m->loss_parts_n, h->nblocks, sizeof(double));
    if (rc) return rc;
    // the network and the lattice may use different streams: order m's work first
    HIP_TRY(hipStreamSynchronize(m->stream));
    HIP_TRY(hipMemcpyAsync(m->inv_sigma, isig, sizeof isig, hipMemcpyHostToDevice, h->stream));
    void* state = h->buf[h->cur];
    void* post = h->buf[1 - h->cur];
    lbm::launch_step_mlp(LBM_FP32, 0, false, false, state, post, g, h->ph, m->packed, h->fb_partials, h->grid, h->block,
                         h->stream);
    lbm::launch_train_loss((const float*)post, g, (float)h->p.rho0, target, m->inv_sigma, m->gbuf, m->loss_parts,
                           false, nullptr, 0.0f, h->grid, h->block, h->stream);
    lbm::launch_train_backward((const float*)state, m->gbuf, g, h->ph, m->packed, m->grad_parts, nullptr, false,
                               h->stream);
    lbm::launch_reduce_grad(m->grad_parts, nwb, m->grad, m->red_tmp, h->stream);
    lbm::launch_sum_partials(m->loss_parts, h->nblocks, m->loss_dev, h->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(m->loss_host, m->loss_dev, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (loss) *loss = *m->loss_host;
    return LBM_OK;
}

int lbm_mlp_accumulate_rollout_grad(lbm_mlp* m, lbm_handle* h, const float* targets, int32_t steps,
                                    const double sigma[10], const double* step_weight, float* dstate,
                                    double* step_loss, double* loss)
{
    if (!m || !h || !targets || !sigma) return fail(LBM_EINVAL, "NULL argument");
    if (steps < 1 || steps > LBM_MLP_MAX_ROLLOUT)
        return fail(LBM_EINVAL, "steps must be in [1, %d]", LBM_MLP_MAX_ROLLOUT);
    float isig[10];
    int rc = training_checks(m, h, sigma, 1, isig);
    if (rc) return rc;
    // step k's loss enters as (w_k / steps) loss_k: its inverse scales carry sqrt(w_k / steps)
    std::vector<float> isk((size_t)steps * 10);
    std::vector<double> wk((size_t)steps, 1.0);
    for (int k = 0; k < steps; ++k) {
        if (step_weight) {
            if (!(std::isfinite(step_weight[k]) && step_weight[k] > 0.0))
                return fail(LBM_EINVAL, "step weights must be positive");
            wk[k] = step_weight[k];
        }
        const double f = std::sqrt(wk[k] / steps);
        for (int j = 0; j < 10; ++j) isk[(size_t)k * 10 + j] = (float)(f / sigma[j]);
    }
    const lbm::Geom& g = h->g;
    const int64_t state_elems = (int64_t)19 * g.stride;
    const int nwb = ((g.nx + 63) / 64) * g.ny * g.nz;
    rc = grow((void**)&m->gbuf, m->gbuf_elems, (int64_t)2 * 19 * g.N, sizeof(float));
    if (!rc) rc = grow((void**)&m->traj, m->traj_elems, (int64_t)steps * state_elems, sizeof(float));
    if (!rc) rc = grow((void**)&m->grad_parts, m->grad_parts_n, (int64_t)nwb * LBM_MLP_NPARAM, sizeof(float));
    if (!rc) rc = grow((void**)&m->loss_parts, m->loss_parts_n, (int64_t)steps * h->nblocks, sizeof(double));
    if (!rc) rc = grow((void**)&m->isig_steps, m->isig_steps_n, (int64_t)steps * 10, sizeof(float));
    const bool energy = m->energy_weight > 0.0;
    if (!rc && energy) rc = grow((void**)&m->energies, m->energies_n, (int64_t)2 * steps, sizeof(double));
    if (!rc && energy) rc = grow((void**)&m->energy_parts, m->energy_parts_n, (int64_t)2 * h->nblocks, sizeof(double));
    if (!rc && m->loss_steps_n < LBM_MLP_MAX_ROLLOUT) {
        // both buffers or neither: a partial allocation is released, so a
        // later call starts from nothing again
        double *dev = nullptr, *host = nullptr;
        if (hipMalloc((void**)&dev, sizeof(double) * LBM_MLP_MAX_ROLLOUT) != hipSuccess ||
            hipHostMalloc((void**)&host, sizeof(double) * LBM_MLP_MAX_ROLLOUT, hipHostMallocDefault) != hipSuccess) {
            if (dev) hipFree(dev);
            return fail(LBM_ENOMEM, "rollout loss buffers");
        }
        m->loss_steps = dev;
        m->loss_steps_host = host;
        m->loss_steps_n = LBM_MLP_MAX_ROLLOUT;
    }
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(m->stream));
    HIP_TRY(hipMemcpyAsync(m->isig_steps, isk.data(), sizeof(float) * isk.size(), hipMemcpyHostToDevice, h->stream));
    // forward: P_0 = h's state, P_k = m->traj + (k - 1) * state_elems
    auto P = [&](int k) -> float* {
        return k == 0 ? (float*)h->buf[h->cur] : m->traj + (int64_t)(k - 1) * state_elems;
    };
    for (int k = 0; k < steps; ++k)
        lbm::launch_step_mlp(LBM_FP32, 0, false, false, P(k), P(k + 1), g, h->ph, m->packed, h->fb_partials, h->grid,
                             h->block, h->stream);
    // kinetic energies of every state and target (energy term)
    if (energy)
        for (int k = 1; k <= steps; ++k) {
            lbm::launch_train_energy(P(k), g, (float)h->p.rho0, targets + (int64_t)(k - 1) * 10 * g.N, m->energy_parts,
                                     h->grid, h->block, h->stream);
            lbm::launch_sum_partials(m->energy_parts, h->nblocks, m->energies + 2 * (k - 1), h->stream);
            lbm::launch_sum_partials(m->energy_parts + h->nblocks, h->nblocks, m->energies + 2 * (k - 1) + 1, h->stream);
        }
    const float ew = (float)(m->energy_weight / steps);
    // backward: A holds dL/df(t0 + k + 1); the step from P_k turns it into
    // dL/df(t0 + k) (in B, or in dstate for k = 0), to which the loss after k
    // steps adds its own gradient
    float* A = m->gbuf;
    float* B = m->gbuf + (int64_t)19 * g.N;
    auto loss_at = [&](int k, float* adj, bool acc) { // loss after k steps (k = 1..steps)
        lbm::launch_train_loss(P(k), g, (float)h->p.rho0, targets + (int64_t)(k - 1) * 10 * g.N,
                               m->isig_steps + (int64_t)(k - 1) * 10, adj,
                               m->loss_parts + (int64_t)(k - 1) * h->nblocks, acc,
                               energy ? m->energies + 2 * (k - 1) : nullptr, ew, h->grid, h->block, h->stream);
    };
    loss_at(steps, A, false);
    for (int k = steps - 1; k >= 0; --k) {
        float* out = k > 0 ? B : dstate;
        // the partials of all steps add up in place; one reduction at the end
        lbm::launch_train_backward(P(k), A, g, h->ph, m->packed, m->grad_parts, out, k < steps - 1, h->stream);
        if (k > 0) {
            loss_at(k, B, true);
            std::swap(A, B);
        }
    }
    lbm::launch_reduce_grad(m->grad_parts, nwb, m->grad, m->red_tmp, h->stream);
    for (int k = 0; k < steps; ++k)
        lbm::launch_sum_partials(m->loss_parts + (int64_t)k * h->nblocks, h->nblocks, m->loss_steps + k, h->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(m->loss_steps_host, m->loss_steps, sizeof(double) * steps, hipMemcpyDeviceToHost, h->stream));
    std::vector<double> en(energy ? 2 * (size_t)steps : 0);
    if (energy)
        HIP_TRY(hipMemcpyAsync(en.data(), m->energies, sizeof(double) * en.size(), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    double total = 0.0;
    for (int k = 0; k < steps; ++k) {
        total += m->loss_steps_host[k];
        if (step_loss) step_loss[k] = m->loss_steps_host[k] * steps / wk[k];
        if (energy) {
            const double r = (en[2 * k] - en[2 * k + 1]) / en[2 * k + 1];
            total += m->energy_weight / steps * r * r;
        }
    }
    if (loss) *loss = total;
    return LBM_OK;
}

int lbm_mlp_set_energy_weight(lbm_mlp* m, double w)
{
    if (!m) return fail(LBM_EINVAL, "NULL argument");
    if (!(std::isfinite(w) && w >= 0.0)) return fail(LBM_EINVAL, "the energy weight must be finite and >= 0");
    m->energy_weight = w;
    return LBM_OK;
}

int lbm_mlp_get_grad(const lbm_mlp* m, double* grad)
{
    if (!m || !grad) return fail(LBM_EINVAL, "NULL argument");
    HIP_TRY(hipMemcpyAsync(grad, m->grad, sizeof(double) * LBM_MLP_NPARAM, hipMemcpyDeviceToHost, m->stream));
    HIP_TRY(hipStreamSynchronize(m->stream));
    return LBM_OK;
}

int lbm_mlp_adam_step(lbm_mlp* m, double lr, double beta1, double beta2, double eps)
{
    if (!m) return fail(LBM_EINVAL, "NULL argument");
    if (!(lr > 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0))
        return fail(LBM_EINVAL, "bad Adam hyper-parameters");
    m->adam_t++;
    const double c1 = 1.0 - std::pow(beta1, (double)m->adam_t), c2 = 1.0 - std::pow(beta2, (double)m->adam_t);
    lbm::launch_adam(m->theta, m->m1, m->m2, m->grad, (float)lr, (float)beta1, (float)beta2, (float)eps, (float)c1,
                     (float)c2, m->stream);
    int rc = mlp_repack(m);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(m->stream));
    return LBM_OK;
}

int lbm_feature_rms(lbm_handle* h, double rms[11])
{
    if (!h || !rms) return fail(LBM_EINVAL, "NULL argument");
    if (h->p.q != 19 || h->p.precision == LBM_FP64 || h->p.moments != LBM_CENTRAL_MOMENTS)
        return fail(LBM_EUNSUPPORTED, "central-moment D3Q19 with FP32/16-bit storage");
    double* part = nullptr;
    double* out = nullptr;
    HIP_TRY(hipMalloc((void**)&part, sizeof(double) * 11 * (h->nblocks + 1)));
    out = part + 11 * (int64_t)h->nblocks;
    lbm::launch_feature_sumsq(h->p.precision, pattern_of(h), h->walls, h->buf[h->cur], h->g, h->ph, part, out,
                              h->nblocks, h->grid, h->block, h->stream);
    double host[11];
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(host, out, sizeof host, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    hipFree(part);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "feature_rms: %s", hipGetErrorString(e));
    for (int k = 0; k < 11; ++k) rms[k] = std::sqrt(host[k] / (double)h->g.N);
    return LBM_OK;
}

int lbm_project_q27(const double* f27, int64_t n, double* f19, float* moments, void* stream)
{
    if (!f27 || n <= 0) return fail(LBM_EINVAL, "bad arguments");
    lbm::launch_project_q27(f27, n, f19, moments, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}


int64_t lbm_device_bytes(const lbm_handle* h) { return h ? h->bytes : -1; }

} // extern "C"

// ---------------------------------------------------------------------------
// lbm_moments_noalloc: the per-work-group partial totals of the moments kernel
// live in a fixed device array instead of the handle's allocation, so the
// call allocates nothing.  In host code `scratch` names a host-side stand-in:
// its device address is looked up once per device (hipGetSymbolAddress, with
// that device current) and only that address is handed to kernels.
// ---------------------------------------------------------------------------
namespace {

constexpr int NOALLOC_MAX_PARTIALS = 16384; // work-groups whose partials fit: 16384 x 8 doubles = 1 MiB
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) double scratch[NOALLOC_MAX_PARTIALS * lbm::NDIAG_OUT];

std::mutex g_scratch_mu;
double* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

int scratch_address(int dev, double** out)
{
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(LBM_EUNSUPPORTED, "device %d beyond %d", dev, NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int cur = -1;
        HIP_TRY(hipGetDevice(&cur));
        if (cur != dev) HIP_TRY(hipSetDevice(dev));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) HIP_TRY(hipSetDevice(cur));
        if (e != hipSuccess || !ptr) return fail(LBM_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_dev[dev] = (double*)ptr;
    }
    *out = g_scratch_dev[dev];
    return LBM_OK;
}

} // namespace

extern "C" int lbm_moments_noalloc(lbm_handle* h, double* rho, double* u, double* diag)
{
    if (!h) return fail(LBM_EINVAL, "NULL handle");
    if (h->cp) return fail(LBM_EUNSUPPORTED, "lbm_moments_noalloc: not for coupled lattices (use lbm_moments)");
    // one work-group per (x-block, y-block) and per group of z planes: as many
    // plane groups as the fixed partials array holds
    const int64_t plane_groups = (int64_t)h->grid.x * h->grid.y;
    if (plane_groups > NOALLOC_MAX_PARTIALS)
        return fail(LBM_EINVAL, "lbm_moments_noalloc: %lld work-groups per z plane (nx %d, ny %d) exceed the %d the fixed "
                    "scratch holds; use lbm_moments", (long long)plane_groups, h->g.nx, h->g.ny, NOALLOC_MAX_PARTIALS);
    double* part = nullptr;
    const int rc = scratch_address(h->device, &part);
    if (rc) return rc;
    const int64_t gz = std::min<int64_t>(h->grid.z, NOALLOC_MAX_PARTIALS / plane_groups);
    const dim3 grid(h->grid.x, h->grid.y, (unsigned)gz);
    lbm::launch_moments(h->p.q, h->kprec, pattern_of(h), h->walls, h->buf[h->cur], h->g, h->ph, rho, u, part, grid,
                        h->block, h->stream);
    if (diag) lbm::launch_reduce(part, (int)(plane_groups * gz), diag, h->stream, 6);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

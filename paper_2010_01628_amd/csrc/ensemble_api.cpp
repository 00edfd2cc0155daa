// Host side of the ensemble entry points of include/lbm.h: one allocation for
// every box, a (box, tile) work list, one persistent launch per step, the
// step loop captured in a HIP graph and replayed.
#include "lbm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lbm_internal.hpp"

namespace {

thread_local char e_err[512] = "";

int efail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(e_err, sizeof e_err, fmt, ap);
    va_end(ap);
    lbm_internal_set_error(e_err);
    return code;
}

#define EHIP(expr)                                                                                                  \
    do {                                                                                                            \
        hipError_t e_ = (expr);                                                                                     \
        if (e_ != hipSuccess)                                                                                       \
            return efail(e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int TILE = 256;

} // namespace

struct lbm_ensemble {
    hipStream_t stream = nullptr;
    bool own_stream = false; // created here when the caller passed NULL (the null stream cannot be captured)
    int q = 19, precision = LBM_FP32, nboxes = 0, ntiles = 0;
    int64_t nodes = 0, elems = 0;
    int eb = 4;
    bool off32 = true; // every box's population arrays below 4 GiB (and LBM_OFF32 != 0)
    std::vector<int> L;
    std::vector<double> omega;
    std::vector<int64_t> off, stride;
    std::vector<int> tile0, tiles;
    void* buf[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t steps = 0;
    void* boxes_dev = nullptr;
    int* tile_box_dev = nullptr;
    int* tile_count_dev = nullptr;
    double* tile_out = nullptr;
    double* box_out = nullptr;
    const lbm_mlp* mlp = nullptr;
    uint32_t* fb = nullptr;  // fallback counts, one per work-group of the largest grid
    int64_t fb_len = 0;
    int grid = 0;
    // captured step loop: `graph_steps` steps starting from buffer parity 0
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_steps = 0;
    const void* graph_net = nullptr; // network weights the captured launches read (NULL: plain rates)
    // plain step: at most occ_waves resident wavefronts per SIMD (by LDS
    // allocation; 0: no cap), as for the single lattice
    int occ_waves = 5, lds_per_cu = 163840;
};

namespace {

void launch_one(lbm_ensemble* e)
{
    const int src = e->cur, dst = 1 - e->cur;
    lbm::launch_ens_step(e->q, e->precision == LBM_FP64 ? 0 : 1, e->mlp != nullptr, e->off32, e->buf[src], e->buf[dst],
                         e->boxes_dev, e->tile_box_dev, e->ntiles, 1.0f, e->mlp ? e->mlp->packed : nullptr, e->fb,
                         e->grid, TILE, e->occ_waves, e->lds_per_cu, e->stream);
    e->cur = dst;
}

void drop_graph(lbm_ensemble* e)
{
    if (e->exec) hipGraphExecDestroy(e->exec);
    if (e->graph) hipGraphDestroy(e->graph);
    e->exec = nullptr;
    e->graph = nullptr;
}

int build_graph(lbm_ensemble* e, int nsteps)
{
    drop_graph(e);
    const int saved = e->cur;
    EHIP(hipStreamBeginCapture(e->stream, hipStreamCaptureModeThreadLocal));
    for (int s = 0; s < nsteps; ++s) launch_one(e);
    hipError_t err = hipStreamEndCapture(e->stream, &e->graph);
    e->cur = saved;
    if (err != hipSuccess) return efail(LBM_EDEVICE, "graph capture: %s", hipGetErrorString(err));
    EHIP(hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0));
    e->graph_steps = nsteps;
    e->graph_net = e->mlp ? e->mlp->packed : nullptr;
    return LBM_OK;
}

} // namespace

extern "C" {

int lbm_ensemble_create(const lbm_box* boxes, int32_t nboxes, int32_t q, int32_t precision, void* stream,
                        lbm_ensemble** out)
{
    if (!out || !boxes || nboxes <= 0) return efail(LBM_EINVAL, "bad arguments");
    *out = nullptr;
    if (q != 19 && q != 27) return efail(LBM_EINVAL, "q must be 19 or 27");
    if (precision != LBM_FP32 && precision != LBM_FP64) return efail(LBM_EUNSUPPORTED, "ensembles store FP32 or FP64");
    for (int b = 0; b < nboxes; ++b) {
        if (boxes[b].n < 2 || boxes[b].n > 1024) return efail(LBM_EINVAL, "box %d: side must be in [2, 1024]", b);
        if (!(boxes[b].omega > 0.0 && boxes[b].omega < 2.0)) return efail(LBM_EINVAL, "box %d: omega in (0,2)", b);
    }
    lbm_ensemble* e = new lbm_ensemble();
    e->stream = (hipStream_t)stream;
    if (!e->stream) {
        if (hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) != hipSuccess) {
            delete e;
            return efail(LBM_EDEVICE, "stream creation");
        }
        e->own_stream = true;
    }
    e->q = q;
    e->precision = precision;
    e->nboxes = nboxes;
    e->eb = precision == LBM_FP64 ? 8 : 4;
    int64_t elems = 0;
    int tiles = 0;
    for (int b = 0; b < nboxes; ++b) {
        const int L = boxes[b].n;
        const int64_t N = (int64_t)L * L * L;
        // pad each population array to a multiple of 256 elements plus 68*256 B
        const int64_t stride = ((N + 255) / 256) * 256 + 17408 / e->eb;
        e->L.push_back(L);
        e->omega.push_back(boxes[b].omega);
        e->off.push_back(elems);
        e->stride.push_back(stride);
        if (stride * e->eb >= ((int64_t)1 << 32)) e->off32 = false;
        e->tile0.push_back(tiles);
        const int nt = (int)((N + TILE - 1) / TILE);
        e->tiles.push_back(nt);
        tiles += nt;
        elems += (int64_t)q * stride;
        e->nodes += N;
    }
    e->ntiles = tiles;
    e->elems = elems;
    {
        const char* env = std::getenv("LBM_OFF32");
        if (env && env[0] == '0') e->off32 = false;
    }
    auto cleanup = [&](int code) {
        lbm_ensemble_destroy(e);
        return code;
    };
    std::vector<char> desc(lbm::ens_box_desc_bytes() * nboxes);
    std::vector<int> tile_box(tiles);
    for (int b = 0; b < nboxes; ++b) {
        lbm::ens_fill_box_desc(desc.data() + b * lbm::ens_box_desc_bytes(), e->L[b], e->tile0[b], e->off[b],
                               e->stride[b], e->omega[b]);
        for (int t = 0; t < e->tiles[b]; ++t) tile_box[e->tile0[b] + t] = b;
    }
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return cleanup(efail(LBM_EDEVICE, "no HIP device"));
    // five wavefronts per SIMD for the plain step: 64-box workload, one
    // machine, D3Q19 5.42 -> 5.58 TB/s, D3Q27 5.16 -> 5.27 (four: the same
    // for D3Q19, six: 5.51); LBM_WAVES_PER_SIMD=n sets the cap (0: none)
    {
        const char* env = std::getenv("LBM_WAVES_PER_SIMD");
        if (env) e->occ_waves = std::atoi(env);
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess && lds > 0)
            e->lds_per_cu = lds;
    }
    // default: one work-group per tile (the tuner's choice on MI355X for the
    // 64-box workload); lbm_ensemble_tune also tries 2..64 persistent
    // work-groups per CU
    e->grid = tiles;
    for (int k = 0; k < 2; ++k)
        if (hipMalloc(&e->buf[k], elems * e->eb) != hipSuccess) return cleanup(efail(LBM_ENOMEM, "population buffers"));
    if (hipMalloc(&e->boxes_dev, desc.size()) != hipSuccess ||
        hipMalloc((void**)&e->tile_box_dev, sizeof(int) * tiles) != hipSuccess ||
        hipMalloc((void**)&e->tile_count_dev, sizeof(int) * nboxes) != hipSuccess ||
        hipMalloc((void**)&e->tile_out, sizeof(double) * 2 * tiles) != hipSuccess ||
        hipMalloc((void**)&e->box_out, sizeof(double) * 2 * nboxes) != hipSuccess ||
        hipMalloc((void**)&e->fb, sizeof(uint32_t) * (size_t)(e->fb_len = std::max<int64_t>((int64_t)ncu * 64, tiles))) !=
            hipSuccess)
        return cleanup(efail(LBM_ENOMEM, "ensemble tables"));
    hipError_t err = hipMemcpy(e->boxes_dev, desc.data(), desc.size(), hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(e->tile_box_dev, tile_box.data(), sizeof(int) * tiles, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemcpy(e->tile_count_dev, e->tiles.data(), sizeof(int) * nboxes, hipMemcpyHostToDevice);
    if (err == hipSuccess) err = hipMemset(e->buf[0], 0, elems * e->eb);
    if (err == hipSuccess) err = hipMemset(e->buf[1], 0, elems * e->eb);
    if (err == hipSuccess) err = hipMemset(e->fb, 0, sizeof(uint32_t) * (size_t)e->fb_len);
    // the set-up above ran on the null stream; the ensemble's stream may not
    // be ordered with it
    if (err == hipSuccess) err = hipDeviceSynchronize();
    if (err != hipSuccess) return cleanup(efail(LBM_EDEVICE, "ensemble upload: %s", hipGetErrorString(err)));
    *out = e;
    return LBM_OK;
}

int lbm_ensemble_destroy(lbm_ensemble* e)
{
    if (!e) return LBM_OK;
    hipStreamSynchronize(e->stream);
    drop_graph(e);
    void* bufs[] = {e->buf[0], e->buf[1], e->boxes_dev, e->tile_box_dev, e->tile_count_dev, e->tile_out, e->box_out, e->fb};
    for (void* b : bufs)
        if (b) hipFree(b);
    if (e->own_stream) hipStreamDestroy(e->stream);
    delete e;
    return LBM_OK;
}

static lbm::Geom box_geom(const lbm_ensemble* e, int b)
{
    lbm::Geom g;
    g.nx = g.ny = g.nz = e->L[b];
    g.nxy = e->L[b] * e->L[b];
    g.N = e->L[b] * e->L[b] * e->L[b];
    g.stride = e->stride[b];
    return g;
}

static void box_launch_shape(const lbm_ensemble* e, int b, dim3& grid, dim3& block)
{
    const int L = e->L[b];
    int bx = 8;
    while (bx < L && bx < 256) bx <<= 1;
    int by = 256 / bx;
    grid = dim3((L + bx - 1) / bx, (L + by - 1) / by, L);
    block = dim3(bx, by, 1);
}

int lbm_ensemble_init(lbm_ensemble* e, int32_t box, const double* rho, const double* u, int on_device)
{
    if (!e || !rho || !u || box < 0 || box >= e->nboxes) return efail(LBM_EINVAL, "bad arguments");
    const lbm::Geom g = box_geom(e, box);
    const double* dr = rho;
    const double* du = u;
    double* staging = nullptr;
    if (!on_device) {
        EHIP(hipMalloc((void**)&staging, sizeof(double) * 4 * g.N));
        EHIP(hipMemcpyAsync(staging, rho, sizeof(double) * g.N, hipMemcpyHostToDevice, e->stream));
        EHIP(hipMemcpyAsync(staging + g.N, u, sizeof(double) * 3 * g.N, hipMemcpyHostToDevice, e->stream));
        dr = staging;
        du = staging + g.N;
    }
    dim3 grid, block;
    box_launch_shape(e, box, grid, block);
    char* base = (char*)e->buf[e->cur] + e->off[box] * e->eb;
    lbm::launch_init(e->q, e->precision == LBM_FP64 ? 0 : 1, 0, false, base, g, 1.0, dr, du, grid, block, e->stream);
    hipError_t err = hipGetLastError();
    if (staging) {
        hipStreamSynchronize(e->stream);
        hipFree(staging);
    }
    if (err != hipSuccess) return efail(LBM_EDEVICE, "init: %s", hipGetErrorString(err));
    return LBM_OK;
}

int lbm_ensemble_get_populations(lbm_ensemble* e, int32_t box, double* f, int on_device)
{
    if (!e || !f || box < 0 || box >= e->nboxes) return efail(LBM_EINVAL, "bad arguments");
    const lbm::Geom g = box_geom(e, box);
    const int64_t bytes = sizeof(double) * e->q * (int64_t)g.N;
    double* dst = f;
    if (!on_device) EHIP(hipMalloc((void**)&dst, bytes));
    dim3 grid, block;
    box_launch_shape(e, box, grid, block);
    const char* base = (const char*)e->buf[e->cur] + e->off[box] * e->eb;
    lbm::launch_get_pops(e->q, e->precision == LBM_FP64 ? 0 : 1, 0, false, base, g, 1.0, dst, grid, block, e->stream);
    hipError_t err = hipGetLastError();
    if (!on_device) {
        if (err == hipSuccess) err = hipMemcpyAsync(f, dst, bytes, hipMemcpyDeviceToHost, e->stream);
        if (err == hipSuccess) err = hipStreamSynchronize(e->stream);
        hipFree(dst);
    }
    if (err != hipSuccess) return efail(LBM_EDEVICE, "get_populations: %s", hipGetErrorString(err));
    return LBM_OK;
}

int lbm_ensemble_set_mlp(lbm_ensemble* e, const lbm_mlp* m)
{
    if (!e) return efail(LBM_EINVAL, "NULL ensemble");
    if (m && (e->q != 19 || e->precision != LBM_FP32))
        return efail(LBM_EUNSUPPORTED, "learned rates need a D3Q19 FP32 ensemble");
    if (m) EHIP(hipStreamSynchronize(m->stream));
    // a captured step loop has the previous network's weight pointer baked
    // into its launches: replaying it would read that network (possibly freed)
    if (m != e->mlp) drop_graph(e);
    e->mlp = m;
    return LBM_OK;
}

int lbm_ensemble_step(lbm_ensemble* e, int64_t nsteps)
{
    if (!e || nsteps < 0) return efail(LBM_EINVAL, "bad arguments");
    const char* env = std::getenv("LBM_ENSEMBLE_GRAPH_STEPS");
    // even (rounded down): a replay then leaves the buffer parity unchanged,
    // which the replay loop below relies on (e->cur is not advanced by it)
    int chunk = env ? std::atoi(env) : 16;
    chunk &= ~1;
    int64_t left = nsteps;
    // single steps until the parity is even, so the graph always starts from buffer 0
    while (left > 0 && (e->cur != 0 || chunk < 2 || left < chunk)) {
        launch_one(e);
        e->steps++;
        left--;
    }
    if (left >= chunk && chunk >= 2) {
        if (!e->exec || e->graph_steps != chunk || e->graph_net != (e->mlp ? e->mlp->packed : nullptr)) {
            int rc = build_graph(e, chunk);
            if (rc) return rc;
        }
        while (left >= chunk) {
            EHIP(hipGraphLaunch(e->exec, e->stream));
            e->steps += chunk;
            left -= chunk;
        }
    }
    while (left > 0) {
        launch_one(e);
        e->steps++;
        left--;
    }
    EHIP(hipGetLastError());
    return LBM_OK;
}

int lbm_ensemble_energy(lbm_ensemble* e, double* ke, double* mass)
{
    if (!e || (!ke && !mass)) return efail(LBM_EINVAL, "bad arguments");
    lbm::launch_ens_energy(e->q, e->precision == LBM_FP64 ? 0 : 1, e->buf[e->cur], e->boxes_dev, e->tile_box_dev,
                           e->ntiles, e->nboxes, e->tile_count_dev, 1.0, e->tile_out, e->box_out, e->grid, e->stream);
    EHIP(hipGetLastError());
    std::vector<double> host(2 * e->nboxes);
    EHIP(hipMemcpyAsync(host.data(), e->box_out, sizeof(double) * 2 * e->nboxes, hipMemcpyDeviceToHost, e->stream));
    EHIP(hipStreamSynchronize(e->stream));
    for (int b = 0; b < e->nboxes; ++b) {
        if (ke) ke[b] = host[2 * b];
        if (mass) mass[b] = host[2 * b + 1];
    }
    return LBM_OK;
}

int64_t lbm_ensemble_nodes(const lbm_ensemble* e) { return e ? e->nodes : -1; }
int64_t lbm_ensemble_step_count(const lbm_ensemble* e) { return e ? e->steps : -1; }

int64_t lbm_ensemble_fallback_count(lbm_ensemble* e)
{
    if (!e) return efail(LBM_EINVAL, "NULL ensemble");
    if (hipStreamSynchronize(e->stream) != hipSuccess) return efail(LBM_EDEVICE, "sync");
    std::vector<uint32_t> host(e->fb_len);
    if (hipMemcpy(host.data(), e->fb, sizeof(uint32_t) * e->fb_len, hipMemcpyDeviceToHost) != hipSuccess)
        return efail(LBM_EDEVICE, "copy");
    int64_t t = 0;
    for (uint32_t v : host) t += v;
    return t;
}

int lbm_ensemble_tune(lbm_ensemble* e, int32_t trial_steps, int32_t* grid_out)
{
    if (!e || trial_steps < 2) return efail(LBM_EINVAL, "bad arguments");
    int dev = 0, ncu = 0;
    EHIP(hipGetDevice(&dev));
    EHIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // Candidates: workgroups per CU.  Timing runs real steps on the current
    // state, then the buffers return to the same parity (even step counts).
    // (0: one work-group per tile, i.e. no persistence)
    const int mult[] = {2, 4, 8, 16, 32, 64, 0};
    hipEvent_t a, b;
    EHIP(hipEventCreate(&a));
    EHIP(hipEventCreate(&b));
    float best_ms = 1e30f;
    int best = e->grid;
    const int steps = trial_steps + (trial_steps & 1);
    for (int m : mult) {
        int g = m ? ncu * m : e->ntiles;
        if (g > e->ntiles) g = e->ntiles;
        e->grid = g;
        launch_one(e);
        launch_one(e); // warm-up, parity unchanged
        EHIP(hipEventRecord(a, e->stream));
        for (int s = 0; s < steps; ++s) launch_one(e);
        EHIP(hipEventRecord(b, e->stream));
        EHIP(hipEventSynchronize(b));
        float ms = 0.0f;
        EHIP(hipEventElapsedTime(&ms, a, b));
        e->steps += steps + 2;
        if (ms < best_ms) {
            best_ms = ms;
            best = g;
        }
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    e->grid = best;
    drop_graph(e); // captured with another grid
    if (grid_out) *grid_out = best;
    return LBM_OK;
}

} // extern "C"

// Host side of the coupled lattices of include/lbm.h (two-phase phase field,
// magnetic field).
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "coupled.hpp"
#include "handle.hpp"

namespace {

#define CHIP(expr)                                                                                        \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess)                                                                             \
            return lbm_fail(e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "%s: %s", #expr,        \
                            hipGetErrorString(e_));                                                       \
    } while (0)

int eb_of(int precision) { return precision == LBM_FP64 ? 8 : 4; }

// Copy a host array to a fresh device buffer (or use the device pointer).
struct Staged {
    const double* ptr = nullptr;
    double* owned = nullptr;
    ~Staged()
    {
        if (owned) hipFree(owned);
    }
};

int stage_in(const double* src, int64_t n, int on_device, hipStream_t st, Staged& out)
{
    if (!src) return LBM_OK;
    if (on_device) {
        out.ptr = src;
        return LBM_OK;
    }
    CHIP(hipMalloc((void**)&out.owned, sizeof(double) * n));
    CHIP(hipMemcpyAsync(out.owned, src, sizeof(double) * n, hipMemcpyHostToDevice, st));
    out.ptr = out.owned;
    return LBM_OK;
}

} // namespace

static int magnetic_validate(const lbm_params* p)
{
    if (p->q != 19) return lbm_fail(LBM_EUNSUPPORTED, "the magnetic coupling runs on D3Q19");
    if (p->precision != LBM_FP64 && p->precision != LBM_FP32)
        return lbm_fail(LBM_EUNSUPPORTED, "the magnetic coupling stores FP64 or FP32");
    if (p->streaming != LBM_AB) return lbm_fail(LBM_EUNSUPPORTED, "the magnetic coupling streams A-B");
    bool paper = p->omega_bulk == 1.0;
    for (int j = 0; j < 9; ++j) paper = paper && p->omega_hi[j] == 1.0;
    if (!paper) return lbm_fail(LBM_EUNSUPPORTED, "the magnetic coupling uses the paper's bulk and higher-order rates");
    const lbm_magnetic_params& m = p->magnetic;
    if (!(std::isfinite(m.eta) && m.eta > 0.0)) return lbm_fail(LBM_EINVAL, "eta must be positive");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(m.b_wall[a])) return lbm_fail(LBM_EINVAL, "b_wall must be finite");
    return LBM_OK;
}

static int shan_chen_validate(const lbm_params* p)
{
    if (p->q != 19) return lbm_fail(LBM_EUNSUPPORTED, "the Shan-Chen lattice is D3Q19");
    if (p->precision != LBM_FP64 && p->precision != LBM_FP32)
        return lbm_fail(LBM_EUNSUPPORTED, "the Shan-Chen lattice stores FP64 or FP32");
    if (p->streaming != LBM_AB) return lbm_fail(LBM_EUNSUPPORTED, "the Shan-Chen lattice streams A-B");
    if (p->walls_y) return lbm_fail(LBM_EUNSUPPORTED, "the Shan-Chen lattice is periodic");
    if (p->force_mode != LBM_FORCE_NONE && p->force_mode != LBM_FORCE_UNIFORM)
        return lbm_fail(LBM_EUNSUPPORTED, "the Shan-Chen lattice adds only a uniform external force");
    if (!std::isfinite(p->shan_chen.G)) return lbm_fail(LBM_EINVAL, "G must be finite");
    return LBM_OK;
}

static int colour_validate(const lbm_params* p)
{
    if (p->q != 19) return lbm_fail(LBM_EUNSUPPORTED, "the colour-gradient lattice is D3Q19");
    if (p->precision != LBM_FP64 && p->precision != LBM_FP32)
        return lbm_fail(LBM_EUNSUPPORTED, "the colour-gradient lattice stores FP64 or FP32");
    if (p->streaming != LBM_AB) return lbm_fail(LBM_EUNSUPPORTED, "the colour-gradient lattice streams A-B");
    if (p->force_mode != LBM_FORCE_NONE)
        return lbm_fail(LBM_EUNSUPPORTED, "the colour-gradient lattice takes its body force from colour.gravity");
    bool paper = p->omega_bulk == 1.0;
    for (int j = 0; j < 9; ++j) paper = paper && p->omega_hi[j] == 1.0;
    if (!paper) return lbm_fail(LBM_EUNSUPPORTED, "the colour-gradient lattice uses the paper's bulk and higher-order rates");
    const lbm_colour_params& c = p->colour;
    auto frac = [](double a) { return std::isfinite(a) && a >= 0.0 && a < 1.0; };
    if (!frac(c.alpha_red) || !frac(c.alpha_blue)) return lbm_fail(LBM_EINVAL, "alpha must be in [0, 1)");
    if (!(std::isfinite(c.A) && c.A >= 0.0)) return lbm_fail(LBM_EINVAL, "A must be >= 0");
    if (!(std::isfinite(c.beta) && c.beta >= 0.0 && c.beta <= 1.0)) return lbm_fail(LBM_EINVAL, "beta must be in [0, 1]");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(c.gravity[a])) return lbm_fail(LBM_EINVAL, "gravity must be finite");
    if (!std::isfinite(c.rho_ref)) return lbm_fail(LBM_EINVAL, "rho_ref must be finite");
    return LBM_OK;
}

int coupled_validate(const lbm_params* p)
{
    if (p->coupled == LBM_COUPLED_MAGNETIC) return magnetic_validate(p);
    if (p->coupled == LBM_COUPLED_COLOUR) return colour_validate(p);
    if (p->coupled == LBM_COUPLED_SHAN_CHEN) return shan_chen_validate(p);
    const lbm_phase_params& q = p->phase;
    if (p->q != 19) return lbm_fail(LBM_EUNSUPPORTED, "the two-phase lattice is D3Q19");
    if (p->precision != LBM_FP64 && p->precision != LBM_FP32)
        return lbm_fail(LBM_EUNSUPPORTED, "the two-phase lattice stores FP64 or FP32");
    if (p->streaming != LBM_AB) return lbm_fail(LBM_EUNSUPPORTED, "the two-phase lattice streams A-B");
    if (p->walls_y) return lbm_fail(LBM_EUNSUPPORTED, "the two-phase lattice is periodic");
    if (p->force_mode != LBM_FORCE_NONE) return lbm_fail(LBM_EUNSUPPORTED, "the two-phase lattice takes no external force");
    bool paper = p->omega_bulk == 1.0;
    for (int j = 0; j < 9; ++j) paper = paper && p->omega_hi[j] == 1.0;
    if (!paper) return lbm_fail(LBM_EUNSUPPORTED, "the two-phase lattice uses the paper's bulk and higher-order rates");
    if (p->rho0 != 1.0) return lbm_fail(LBM_EINVAL, "the two-phase lattice stores deviations from rho0 = 1");
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!pos(q.rho_light) || !pos(q.rho_heavy)) return lbm_fail(LBM_EINVAL, "phase densities must be positive");
    if (!(std::isfinite(q.sigma) && q.sigma >= 0.0)) return lbm_fail(LBM_EINVAL, "sigma must be >= 0");
    if (!pos(q.width)) return lbm_fail(LBM_EINVAL, "interface width must be positive");
    if (!pos(q.mobility)) return lbm_fail(LBM_EINVAL, "mobility must be positive");
    return LBM_OK;
}

int coupled_create(lbm_handle* h)
{
    const lbm_params& p = h->p;
    lbm_coupled* c = new lbm_coupled();
    h->cp = c;
    const int eb = eb_of(p.precision);
    if (p.coupled == LBM_COUPLED_SHAN_CHEN) {
        c->q = 0;
        c->sc_G = p.shan_chen.G;
        CHIP(hipMalloc(&c->scratch, (int64_t)h->g.N * eb));
        h->bytes += (int64_t)h->g.N * eb;
        return LBM_OK;
    }
    c->q = p.coupled == LBM_COUPLED_MAGNETIC ? 21 : (p.coupled == LBM_COUPLED_COLOUR ? 19 : 7);
    const int64_t bytes = (int64_t)c->q * h->g.stride * eb;
    for (int b = 0; b < 2; ++b) {
        CHIP(hipMalloc(&c->buf[b], bytes));
        h->bytes += bytes;
    }
    if (p.coupled == LBM_COUPLED_COLOUR) {
        CHIP(hipMalloc(&c->scratch, (int64_t)h->g.N * eb));
        h->bytes += (int64_t)h->g.N * eb;
        const lbm_colour_params& q = p.colour;
        c->cc.omega = p.omega;
        c->cc.alpha_r = q.alpha_red;
        c->cc.alpha_b = q.alpha_blue;
        c->cc.A = q.A;
        c->cc.beta = q.beta;
        for (int a = 0; a < 3; ++a) c->cc.g[a] = q.gravity[a];
        c->cc.rho_ref = q.rho_ref;
        h->p.rho0 = 0.0; // both colours are stored whole
        h->ph.rho0 = 0.0;
        return LBM_OK;
    }
    if (p.coupled == LBM_COUPLED_MAGNETIC) {
        c->mc.omega_m = 1.0 / (p.magnetic.eta / 0.25 + 0.5);
        for (int a = 0; a < 3; ++a) c->mc.b_wall[a] = p.magnetic.b_wall[a];
        return LBM_OK;
    }
    CHIP(hipMalloc(&c->scratch, (int64_t)h->g.N * eb));
    h->bytes += (int64_t)h->g.N * eb;
    const lbm_phase_params& q = p.phase;
    c->pc.rho_l = q.rho_light;
    c->pc.drho = q.rho_heavy - q.rho_light;
    c->pc.beta = 12.0 * q.sigma / q.width;
    c->pc.kappa = 1.5 * q.sigma * q.width;
    c->pc.four_over_w = 4.0 / q.width;
    c->pc.omega = p.omega;
    c->pc.omega_phi = 1.0 / (q.mobility / 0.25 + 0.5);
    return LBM_OK;
}

void coupled_destroy(lbm_handle* h)
{
    lbm_coupled* c = h->cp;
    if (!c) return;
    for (int b = 0; b < 2; ++b)
        if (c->buf[b]) hipFree(c->buf[b]);
    if (c->scratch) hipFree(c->scratch);
    delete c;
    h->cp = nullptr;
}

// Launch shape of the two-phase, Shan-Chen and colour-gradient step kernels
// (not the magnetic lattice, which keeps the 3-D grid): a 1-D grid of
// 256-wide work-groups over all nodes, so that no lane idles when nx is not a
// multiple of the work-group width (192^3: a quarter of a 256-wide row
// block, 100^3: 28 % of a 128-wide one); LBM_COUPLED_FLAT=0 keeps the 3-D
// grid of the other kernels.
static void flat_launch(const lbm_handle* h, lbm::Geom& g, dim3& grid, dim3& block)
{
    const char* env = std::getenv("LBM_COUPLED_FLAT");
    g = h->g;
    grid = h->grid;
    block = h->block;
    if (env && env[0] == '0') return;
    g.flat = 1;
    grid = dim3((unsigned)((h->g.N + 255) / 256), 1, 1);
    block = dim3(256, 1, 1);
}

int coupled_step(lbm_handle* h)
{
    lbm_coupled* c = h->cp;
    const int src = h->cur, dst = 1 - h->cur;
    lbm::Geom fg;
    dim3 fgrid, fblock;
    flat_launch(h, fg, fgrid, fblock);
    // the two-phase step on whole-row work-groups with the x-moving
    // populations staged through LDS (rows of up to 256 nodes, periodic);
    // LBM_ROW_STAGING=0 keeps the density launch's grid.  (Staging the
    // Shan-Chen step measured 2 % slower at 100^3: rows of 100 nodes leave a
    // fifth of the lanes idle.)
    lbm::Geom rg = h->g;
    dim3 rgrid(0, 0, 0), rblock(0, 0, 0);
    {
        const char* env = std::getenv("LBM_ROW_STAGING");
        if (h->g.nx <= 256 && !h->walls && !(env && env[0] == '0')) {
            const int by = std::max(1, 256 / h->g.nx);
            rg.flat = 0;
            rblock = dim3(h->g.nx, by, 1);
            rgrid = dim3(1, (h->g.ny + by - 1) / by, h->g.nz);
        }
    }
    if (h->p.coupled == LBM_COUPLED_COLOUR) {
        lbm::launch_cg_step(h->p.precision, h->walls, h->nt, h->buf[src], h->buf[dst], c->buf[src], c->buf[dst],
                            c->scratch, fg, c->cc, fgrid, fblock, h->stream);
        CHIP(hipGetLastError());
        return LBM_OK;
    }
    if (h->p.coupled == LBM_COUPLED_SHAN_CHEN) {
        lbm::launch_sc_step(h->p.precision, h->general, h->nt, h->buf[src], h->buf[dst], c->scratch, fg, h->ph, c->sc_G,
                            fgrid, fblock, h->stream);
        CHIP(hipGetLastError());
        return LBM_OK;
    }
    if (h->p.coupled == LBM_COUPLED_MAGNETIC) {
        lbm::launch_mhd_step(h->p.precision, h->walls, h->nt, h->buf[src], h->buf[dst], c->buf[src], c->buf[dst], h->g,
                             h->ph, c->mc, h->grid, h->block, h->stream);
        CHIP(hipGetLastError());
        return LBM_OK;
    }
    lbm::launch_phase_step(h->p.precision, h->nt, h->buf[src], h->buf[dst], c->buf[src], c->buf[dst], c->scratch, fg,
                           c->pc, fgrid, fblock, rg, rgrid, rblock, h->stream);
    CHIP(hipGetLastError());
    return LBM_OK;
}

int coupled_moments(lbm_handle* h, double* rho, double* u, double* diag, int on_device)
{
    lbm_coupled* c = h->cp;
    const int64_t N = h->g.N;
    double* drho = rho;
    double* du = u;
    double* staging = nullptr;
    if (!on_device && (rho || u)) {
        CHIP(hipMalloc((void**)&staging, sizeof(double) * 4 * N));
        drho = rho ? staging : nullptr;
        du = u ? staging + N : nullptr;
    }
    if (h->p.coupled == LBM_COUPLED_COLOUR)
        lbm::launch_cg_fields(h->p.precision, h->walls, h->buf[h->cur], c->buf[h->cur], h->g, c->cc, drho, du, nullptr,
                              nullptr, h->partials, h->grid, h->block, h->stream);
    else if (h->p.coupled == LBM_COUPLED_SHAN_CHEN)
        lbm::launch_sc_fields(h->p.precision, h->buf[h->cur], c->scratch, h->g, h->ph, c->sc_G, drho, du, h->partials,
                              h->grid, h->block, h->stream);
    else if (h->p.coupled == LBM_COUPLED_MAGNETIC)
        lbm::launch_mhd_fields(h->p.precision, h->walls, h->buf[h->cur], c->buf[h->cur], h->g, h->ph, c->mc, drho, du,
                               nullptr, nullptr, h->partials, h->grid, h->block, h->stream);
    else
        lbm::launch_phase_fields(h->p.precision, h->buf[h->cur], c->buf[h->cur], c->scratch, h->g, c->pc, nullptr,
                                 nullptr, drho, du, h->partials, h->grid, h->block, h->stream);
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
    if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "coupled moments: %s", hipGetErrorString(e));
    if (diag)
        for (int k = 0; k < 6; ++k) diag[k] = h->diag_host[k];
    return LBM_OK;
}

extern "C" {

int lbm_init_phase(lbm_handle* h, const double* phi, const double* p, const double* u, int on_device)
{
    if (!h || !phi || !p || !u) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (!h->cp || h->p.coupled != LBM_COUPLED_PHASE) return lbm_fail(LBM_EINVAL, "not a two-phase lattice");
    const int64_t N = h->g.N;
    Staged sphi, sp, su;
    int rc = stage_in(phi, N, on_device, h->stream, sphi);
    if (!rc) rc = stage_in(p, N, on_device, h->stream, sp);
    if (!rc) rc = stage_in(u, 3 * N, on_device, h->stream, su);
    if (rc) return rc;
    h->steps = 0;
    h->cur = 0;
    lbm::launch_phase_init(h->p.precision, h->buf[0], h->cp->buf[0], h->g, h->cp->pc, sphi.ptr, sp.ptr, su.ptr, h->grid,
                           h->block, h->stream);
    CHIP(hipGetLastError());
    if (!on_device) CHIP(hipStreamSynchronize(h->stream)); // staging buffers are freed on return
    return LBM_OK;
}

int lbm_phase_fields(lbm_handle* h, double* phi, double* p, int on_device)
{
    if (!h) return lbm_fail(LBM_EINVAL, "NULL handle");
    if (!h->cp || h->p.coupled != LBM_COUPLED_PHASE) return lbm_fail(LBM_EINVAL, "not a two-phase lattice");
    const int64_t N = h->g.N;
    double* dphi = phi;
    double* dp = p;
    double* staging = nullptr;
    if (!on_device && (phi || p)) {
        CHIP(hipMalloc((void**)&staging, sizeof(double) * 2 * N));
        dphi = phi ? staging : nullptr;
        dp = p ? staging + N : nullptr;
    }
    lbm::launch_phase_fields(h->p.precision, h->buf[h->cur], h->cp->buf[h->cur], h->cp->scratch, h->g, h->cp->pc, dphi,
                             dp, nullptr, nullptr, h->partials, h->grid, h->block, h->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && staging) {
        if (phi) e = hipMemcpyAsync(phi, staging, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess && p) e = hipMemcpyAsync(p, staging + N, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
    if (staging) hipFree(staging);
    if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "phase fields: %s", hipGetErrorString(e));
    return LBM_OK;
}

int lbm_get_coupled_populations(lbm_handle* h, double* out, int on_device)
{
    if (!h || !out) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (!h->cp || h->cp->q == 0) return lbm_fail(LBM_EINVAL, "no coupled populations");
    const int64_t bytes = sizeof(double) * h->cp->q * (int64_t)h->g.N;
    double* dst = out;
    if (!on_device) CHIP(hipMalloc((void**)&dst, bytes));
    if (h->p.coupled == LBM_COUPLED_COLOUR)
        lbm::launch_get_pops(19, h->p.precision, 0, h->walls, h->cp->buf[h->cur], h->g, 0.0, dst, h->grid, h->block,
                             h->stream);
    else if (h->p.coupled == LBM_COUPLED_MAGNETIC)
        lbm::launch_mhd_get_g(h->p.precision, h->walls, h->cp->buf[h->cur], h->g, h->cp->mc, dst, h->grid, h->block,
                              h->stream);
    else
        lbm::launch_phase_get_h(h->p.precision, h->cp->buf[h->cur], h->g, dst, h->grid, h->block, h->stream);
    hipError_t e = hipGetLastError();
    if (!on_device) {
        if (e == hipSuccess) e = hipMemcpyAsync(out, dst, bytes, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        hipFree(dst);
    }
    if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "get_coupled_populations: %s", hipGetErrorString(e));
    return LBM_OK;
}

int lbm_set_coupled_populations(lbm_handle* h, const double* in, int on_device)
{
    if (!h || !in) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (!h->cp || h->cp->q == 0) return lbm_fail(LBM_EINVAL, "no coupled populations");
    Staged s;
    int rc = stage_in(in, (int64_t)h->cp->q * h->g.N, on_device, h->stream, s);
    if (rc) return rc;
    if (h->p.coupled == LBM_COUPLED_COLOUR)
        lbm::launch_set_pops(19, h->p.precision, 0, h->walls, h->cp->buf[h->cur], h->g, 0.0, s.ptr, h->grid, h->block,
                             h->stream);
    else if (h->p.coupled == LBM_COUPLED_MAGNETIC)
        lbm::launch_mhd_set_g(h->p.precision, h->walls, h->cp->buf[h->cur], h->g, h->cp->mc, s.ptr, h->grid, h->block,
                              h->stream);
    else
        lbm::launch_phase_set_h(h->p.precision, h->cp->buf[h->cur], h->g, s.ptr, h->grid, h->block, h->stream);
    CHIP(hipGetLastError());
    if (!on_device) CHIP(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_init_colour(lbm_handle* h, const double* rho_red, const double* rho_blue, const double* u, int on_device)
{
    if (!h || !rho_red || !rho_blue || !u) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (!h->cp || h->p.coupled != LBM_COUPLED_COLOUR) return lbm_fail(LBM_EINVAL, "not a colour-gradient lattice");
    const int64_t N = h->g.N;
    Staged sr, sb, su;
    int rc = stage_in(rho_red, N, on_device, h->stream, sr);
    if (!rc) rc = stage_in(rho_blue, N, on_device, h->stream, sb);
    if (!rc) rc = stage_in(u, 3 * N, on_device, h->stream, su);
    if (rc) return rc;
    h->steps = 0;
    h->cur = 0;
    lbm::launch_cg_init(h->p.precision, h->walls, h->buf[0], h->cp->buf[0], h->g, h->cp->cc, sr.ptr, sb.ptr, su.ptr,
                        h->grid, h->block, h->stream);
    CHIP(hipGetLastError());
    if (!on_device) CHIP(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_colour_fields(lbm_handle* h, double* rho_red, double* rho_blue, int on_device)
{
    if (!h) return lbm_fail(LBM_EINVAL, "NULL handle");
    if (!h->cp || h->p.coupled != LBM_COUPLED_COLOUR) return lbm_fail(LBM_EINVAL, "not a colour-gradient lattice");
    const int64_t N = h->g.N;
    double* dr = rho_red;
    double* db = rho_blue;
    double* staging = nullptr;
    if (!on_device && (rho_red || rho_blue)) {
        CHIP(hipMalloc((void**)&staging, sizeof(double) * 2 * N));
        dr = rho_red ? staging : nullptr;
        db = rho_blue ? staging + N : nullptr;
    }
    lbm::launch_cg_fields(h->p.precision, h->walls, h->buf[h->cur], h->cp->buf[h->cur], h->g, h->cp->cc, nullptr,
                          nullptr, dr, db, h->partials, h->grid, h->block, h->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && staging) {
        if (rho_red) e = hipMemcpyAsync(rho_red, staging, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess && rho_blue)
            e = hipMemcpyAsync(rho_blue, staging + N, sizeof(double) * N, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
    if (staging) hipFree(staging);
    if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "colour fields: %s", hipGetErrorString(e));
    return LBM_OK;
}

int lbm_init_magnetic(lbm_handle* h, const double* rho, const double* u, const double* b, int on_device)
{
    if (!h || !rho || !u || !b) return lbm_fail(LBM_EINVAL, "NULL argument");
    if (!h->cp || h->p.coupled != LBM_COUPLED_MAGNETIC) return lbm_fail(LBM_EINVAL, "not a magnetic lattice");
    const int64_t N = h->g.N;
    Staged sr, su, sb;
    int rc = stage_in(rho, N, on_device, h->stream, sr);
    if (!rc) rc = stage_in(u, 3 * N, on_device, h->stream, su);
    if (!rc) rc = stage_in(b, 3 * N, on_device, h->stream, sb);
    if (rc) return rc;
    h->steps = 0;
    h->cur = 0;
    lbm::launch_mhd_init(h->p.precision, h->walls, h->buf[0], h->cp->buf[0], h->g, h->p.rho0, h->cp->mc, sr.ptr, su.ptr,
                         sb.ptr, h->grid, h->block, h->stream);
    CHIP(hipGetLastError());
    if (!on_device) CHIP(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_magnetic_fields(lbm_handle* h, double* b, double* j, int on_device)
{
    if (!h) return lbm_fail(LBM_EINVAL, "NULL handle");
    if (!h->cp || h->p.coupled != LBM_COUPLED_MAGNETIC) return lbm_fail(LBM_EINVAL, "not a magnetic lattice");
    const int64_t N = h->g.N;
    double* db = b;
    double* dj = j;
    double* staging = nullptr;
    if (!on_device && (b || j)) {
        CHIP(hipMalloc((void**)&staging, sizeof(double) * 6 * N));
        db = b ? staging : nullptr;
        dj = j ? staging + 3 * N : nullptr;
    }
    lbm::launch_mhd_fields(h->p.precision, h->walls, h->buf[h->cur], h->cp->buf[h->cur], h->g, h->ph, h->cp->mc, nullptr,
                           nullptr, db, dj, h->partials, h->grid, h->block, h->stream);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && staging) {
        if (b) e = hipMemcpyAsync(b, staging, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess && j) e = hipMemcpyAsync(j, staging + 3 * N, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
    if (staging) hipFree(staging);
    if (e != hipSuccess) return lbm_fail(LBM_EDEVICE, "magnetic fields: %s", hipGetErrorString(e));
    return LBM_OK;
}

} // extern "C"

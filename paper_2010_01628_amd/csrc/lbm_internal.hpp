// Internal interface between the host API (lbm_api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// kernel storage types; PREC_BF16SR: BF16 with stochastic rounding (plain
// D3Q19 central-moment steps only)
enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_FP16 = 2, PREC_BF16 = 3, PREC_BF16SR = 4 };
enum { FORCE_NONE = 0, FORCE_UNIFORM = 1, FORCE_FIELD = 2, FORCE_ROW_TABLE = 3 };

struct Geom {
    int nx, ny, nz, nxy;
    int N;          // nodes
    int64_t stride; // elements between consecutive population arrays (>= N)
    int xcd_chunk = 1; // 1-D step grids: rows per XCD run (1 = launch order)
    int row_stage = 0; // periodic A-B / AA odd step with whole-row work-groups: x-moving populations via LDS
    int flat = 0;      // kernels that use thread_node(): 1-D grid over all nodes in index order
    int off32 = 0;     // every population array is below 4 GiB (32-bit element byte offsets)
    int even_cached = 0; // AA even step with 16-bit storage: population loads without the streaming hint
    int occ_waves = 0;   // step kernels: cap on resident wavefronts per SIMD (0: none), by LDS allocation
    int lds_per_cu = 163840; // bytes of LDS per compute unit
};

// x width of a 256-thread work-group over rows longer than 256 nodes that no
// single work-group spans: the widest of 256, 128, 64 and 32 that divides the
// row (no lane idles at the row's end), else 256
inline int row_width(int nx)
{
    return nx % 256 == 0 ? 256 : nx % 128 == 0 ? 128 : nx % 64 == 0 ? 64 : nx % 32 == 0 ? 32 : 256;
}

struct Phys {
    double omega, omega_bulk, omega_hi[9];
    double rho0;
    int force_mode;
    double force[3];
    const double* force_field; // device, double[3N]
    const double* row_table;   // device, double[ny]: F_x per y row
    uint32_t sr_key;           // stochastic rounding: key of the current step
};

#define LBM_DECLARE_LAUNCHERS(SUFFIX)                                                                              \
    void launch_step_##SUFFIX(int precision, int pattern, bool walls, bool general, bool nt, const void* src,        \
                              void* dst, const Geom& g, const Phys& ph, dim3 grid, dim3 block, hipStream_t st);     \
    void launch_init_##SUFFIX(int precision, int pattern, bool walls, void* buf, const Geom& g, double rho0,         \
                              const double* rho, const double* u, dim3 grid, dim3 block, hipStream_t st);           \
    void launch_set_pops_##SUFFIX(int precision, int pattern, bool walls, void* buf, const Geom& g, double rho0,     \
                                  const double* f, dim3 grid, dim3 block, hipStream_t st);                          \
    void launch_get_pops_##SUFFIX(int precision, int pattern, bool walls, const void* buf, const Geom& g,           \
                                  double rho0, double* f, dim3 grid, dim3 block, hipStream_t st);                   \
    void launch_moments_##SUFFIX(int precision, int pattern, bool walls, const void* buf, const Geom& g,            \
                                 const Phys& ph, double* rho, double* u, double* partials, dim3 grid, dim3 block,   \
                                 hipStream_t st);
LBM_DECLARE_LAUNCHERS(q19)
LBM_DECLARE_LAUNCHERS(q27)
#undef LBM_DECLARE_LAUNCHERS

void launch_step_q19rm(int precision, int pattern, bool walls, bool general, bool nt, const void* src, void* dst,
                       const Geom& g, const Phys& ph, dim3 grid, dim3 block, hipStream_t st);

void launch_step_q27rm(int precision, int pattern, bool walls, bool nt, const void* src, void* dst, const Geom& g,
                       const Phys& ph, dim3 grid, dim3 block, hipStream_t st);

// Dispatch on the lattice (q = 19 or 27) and the moment space.
inline void launch_step(int q, bool raw, int precision, int pattern, bool walls, bool general, bool nt,
                        const void* src, void* dst, const Geom& g, const Phys& ph, dim3 grid, dim3 block,
                        hipStream_t st)
{
    if (q == 27 && raw) launch_step_q27rm(precision, pattern, walls, nt, src, dst, g, ph, grid, block, st);
    else if (q == 27) launch_step_q27(precision, pattern, walls, general, nt, src, dst, g, ph, grid, block, st);
    else if (raw) launch_step_q19rm(precision, pattern, walls, general, nt, src, dst, g, ph, grid, block, st);
    else launch_step_q19(precision, pattern, walls, general, nt, src, dst, g, ph, grid, block, st);
}
inline void launch_init(int q, int precision, int pattern, bool walls, void* buf, const Geom& g, double rho0,
                        const double* rho, const double* u, dim3 grid, dim3 block, hipStream_t st)
{
    if (q == 27) launch_init_q27(precision, pattern, walls, buf, g, rho0, rho, u, grid, block, st);
    else launch_init_q19(precision, pattern, walls, buf, g, rho0, rho, u, grid, block, st);
}
inline void launch_set_pops(int q, int precision, int pattern, bool walls, void* buf, const Geom& g, double rho0,
                            const double* f, dim3 grid, dim3 block, hipStream_t st)
{
    if (q == 27) launch_set_pops_q27(precision, pattern, walls, buf, g, rho0, f, grid, block, st);
    else launch_set_pops_q19(precision, pattern, walls, buf, g, rho0, f, grid, block, st);
}
inline void launch_get_pops(int q, int precision, int pattern, bool walls, const void* buf, const Geom& g, double rho0,
                            double* f, dim3 grid, dim3 block, hipStream_t st)
{
    if (q == 27) launch_get_pops_q27(precision, pattern, walls, buf, g, rho0, f, grid, block, st);
    else launch_get_pops_q19(precision, pattern, walls, buf, g, rho0, f, grid, block, st);
}
inline void launch_moments(int q, int precision, int pattern, bool walls, const void* buf, const Geom& g,
                           const Phys& ph, double* rho, double* u, double* partials, dim3 grid, dim3 block,
                           hipStream_t st)
{
    if (q == 27) launch_moments_q27(precision, pattern, walls, buf, g, ph, rho, u, partials, grid, block, st);
    else launch_moments_q19(precision, pattern, walls, buf, g, ph, rho, u, partials, grid, block, st);
}
// nout: totals written to out (at most NDIAG_OUT)
void launch_reduce(const double* partials, int nblocks, double* out, hipStream_t st, int nout = 8);

// learned rates (mlp.hip)
constexpr int MLP_PARAMS = 1737;
void launch_step_mlp(int precision, int pattern, bool walls, bool nt, const void* src, void* dst, const Geom& g,
                     const Phys& ph, const void* net, uint32_t* fb_partials, dim3 grid, dim3 block, hipStream_t st);
// energy (device, [E, E_target]) or nullptr: adds the energy term ew ((E - E_t) / E_t)^2
void launch_train_loss(const float* post, const Geom& g, float rho0, const float* target, const float* inv_sigma,
                       float* gbuf, double* loss_partials, bool accumulate, const double* energy, float ew, dim3 grid,
                       dim3 block, hipStream_t st);
// per-block partial kinetic energies of post (pulled) and of the target moments: partials[b], partials[nblocks + b]
void launch_train_energy(const float* post, const Geom& g, float rho0, const float* target, double* partials,
                         dim3 grid, dim3 block, hipStream_t st);
// gout != nullptr: also write dL/df(t) (rollout back-propagation);
// accumulate: add to grad_partials instead of overwriting them
void launch_train_backward(const float* state, const float* gbuf, const Geom& g, const Phys& ph, const void* net,
                           float* grad_partials, float* gout, bool accumulate, hipStream_t st);
// tmp: reduce_grad_tmp_bytes() of device scratch
size_t reduce_grad_tmp_bytes();
void launch_reduce_grad(const float* partials, int nparts, double* grad, double* tmp, hipStream_t st);
void launch_sum_partials(const double* partials, int n, double* out, hipStream_t st);
void launch_adam(float* theta, float* m1, float* m2, const double* grad, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t st);
void launch_mlp_pack(const float* theta, const float* inv_scale, void* packed, hipStream_t st);
void launch_project_q27(const double* f27, int64_t N, double* f19, float* mom, hipStream_t st);
size_t mlp_packed_bytes();
void launch_feature_sumsq(int precision, int pattern, bool walls, const void* buf, const Geom& g, const Phys& ph,
                          double* partials, double* out, int nblocks, dim3 grid, dim3 block, hipStream_t st);

constexpr int NDIAG_OUT = 8;

} // namespace lbm

// Sets the message returned by lbm_last_error() on this thread.
void lbm_internal_set_error(const char* msg);

// The learned-rate network object behind the opaque lbm_mlp of lbm.h.
struct lbm_mlp {
    hipStream_t stream = nullptr;
    float* theta = nullptr;     // FP32 master parameters (device)
    float* m1 = nullptr;        // Adam moments
    float* m2 = nullptr;
    double* grad = nullptr;     // accumulated gradient (FP64)
    float* inv_scale = nullptr; // 16 floats
    void* packed = nullptr;     // bf16 network for the kernels
    float* inv_sigma = nullptr; // 10 floats
    int64_t adam_t = 0;
    // training scratch, grown on demand
    float* gbuf = nullptr; // two adjoint buffers of 19 N floats (rollouts alternate them)
    int64_t gbuf_elems = 0;
    float* traj = nullptr; // rollout states after steps 1..s (19 x stride floats each)
    int64_t traj_elems = 0;
    float* grad_parts = nullptr;
    int64_t grad_parts_n = 0;
    double* loss_parts = nullptr;
    int64_t loss_parts_n = 0;
    double* loss_dev = nullptr;
    double* loss_host = nullptr;
    double* red_tmp = nullptr; // gradient reduction slices
    float* isig_steps = nullptr; // rollouts: 10 inverse moment scales per step
    int64_t isig_steps_n = 0;
    double* loss_steps = nullptr; // rollouts: loss of each step (device, and its host copy)
    int64_t loss_steps_n = 0;
    double* loss_steps_host = nullptr;
    double energy_weight = 0.0; // rollouts: weight of the kinetic-energy term
    double* energies = nullptr; // rollouts: [E, E_target] per step (device)
    int64_t energies_n = 0;
    double* energy_parts = nullptr; // per-block partial energies of one step
    int64_t energy_parts_n = 0;
};


// ensemble (ensemble.hip)
namespace lbm {
// off32: every box's population arrays are below 4 GiB (32-bit element offsets)
void launch_ens_step(int q, int precision, bool mlp, bool off32, const void* src, void* dst, const void* boxes,
                     const int* tile_box, int ntiles, float rho0, const void* net, uint32_t* fb, int grid, int block,
                     int occ_waves, int lds_per_cu, hipStream_t st);
void launch_ens_energy(int q, int precision, const void* buf, const void* boxes, const int* tile_box, int ntiles,
                       int nboxes, const int* tile_count, double rho0, double* tile_out, double* box_out, int grid,
                       hipStream_t st);
size_t ens_box_desc_bytes();
void ens_fill_box_desc(void* out, int L, int tile0, int64_t off, int64_t stride, double omega);
} // namespace lbm

// Internal interface between the host API (lbm_api.cpp) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_FP16 = 2, PREC_BF16 = 3 };
enum { FORCE_NONE = 0, FORCE_UNIFORM = 1, FORCE_FIELD = 2, FORCE_ROW_TABLE = 3 };

struct Geom {
    int nx, ny, nz, nxy;
    int N;          // nodes
    int64_t stride; // elements between consecutive population arrays (>= N)
};

struct Phys {
    double omega, omega_bulk, omega_hi[9];
    double rho0;
    int force_mode;
    double force[3];
    const double* force_field; // device, double[3N]
    const double* row_table;   // device, double[ny]: F_x per y row
};

void launch_step(int precision, int pattern, bool walls, bool general, bool nt, const void* src, void* dst,
                 const Geom& g, const Phys& ph, dim3 grid, dim3 block, hipStream_t st);
void launch_init(int precision, int pattern, bool walls, void* buf, const Geom& g, double rho0, const double* rho,
                 const double* u, dim3 grid, dim3 block, hipStream_t st);
void launch_set_pops(int precision, int pattern, bool walls, void* buf, const Geom& g, double rho0, const double* f,
                     dim3 grid, dim3 block, hipStream_t st);
void launch_get_pops(int precision, int pattern, bool walls, const void* buf, const Geom& g, double rho0, double* f,
                     dim3 grid, dim3 block, hipStream_t st);
void launch_moments(int precision, int pattern, bool walls, const void* buf, const Geom& g, const Phys& ph, double* rho,
                    double* u, double* partials, dim3 grid, dim3 block, hipStream_t st);
void launch_reduce(const double* partials, int nblocks, double* out, hipStream_t st);

constexpr int NDIAG_OUT = 8;

} // namespace lbm

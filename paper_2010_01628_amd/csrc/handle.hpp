// The lattice handle behind the opaque lbm_handle of include/lbm.h, shared by
// the host-side sources of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"
#include "lbm_internal.hpp"
#include "coupled.hpp"

// State of a coupled lattice (lbm_params.coupled != LBM_COUPLED_NONE).
struct lbm_coupled {
    void* buf[2] = {nullptr, nullptr}; // its populations (A-B), same stride as the flow lattice
    int q = 0;                         // populations per node (7 phase, 21 magnetic, 0 Shan-Chen)
    void* scratch = nullptr;           // phase field phi or pseudo-potential psi (collision arithmetic type)
    double sc_G = 0.0;                 // Shan-Chen interaction strength
    lbm::CgConst cc{};                 // colour-gradient constants (buf: blue colour)
    lbm::PhaseConst pc{};
    lbm::MhdConst mc{};
};

struct lbm_handle {
    lbm_params p;
    int kprec = 0;                     // kernel storage type (lbm::PREC_*; BF16SR for stochastic rounding)
    int device = 0;
    hipStream_t stream = nullptr;
    lbm::Geom g{};
    lbm::Phys ph{};
    void* buf[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t steps = 0;
    double* row_table = nullptr;
    double* partials = nullptr;
    double* diag_dev = nullptr;
    double* diag_host = nullptr;
    dim3 grid, block;
    dim3 step_grid, step_block;        // launch shape of the plain step kernel (tunable)
    int row_stage_pref = -1;           // -1: default (staged wherever possible), 0/1: tuner's choice
    bool walls = false, general = false, nt = true;
    int64_t bytes = 0;
    int nblocks = 0;
    const lbm_mlp* mlp = nullptr;
    uint32_t* fb_partials = nullptr; // per-block fallback counts of the learned step
    lbm_coupled* cp = nullptr;         // coupled lattice, if any
};

// Coupled-lattice parts of the entry points (coupled_api.cpp).
int coupled_validate(const lbm_params* p);
int coupled_create(lbm_handle* h);
void coupled_destroy(lbm_handle* h);
int coupled_step(lbm_handle* h);
int coupled_moments(lbm_handle* h, double* rho, double* u, double* diag, int on_device);
// error reporting of lbm_api.cpp (message for lbm_last_error)
int lbm_fail(int code, const char* fmt, ...);

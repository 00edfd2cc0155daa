/*
 * lbm.h -- C ABI of liblbm.so, an MI355X (gfx950) implementation of the D3Q19
 * central-moment (CM) multiple-relaxation-time lattice Boltzmann method of
 * A. De Rosis & C. Coreixas, "Multiphysics flow simulations using D3Q19
 * lattice Boltzmann methods based on central moments" (arXiv 2010.01628).
 *
 * What one step computes (Sec. II.B, eqs. "lbe", "posColl0", "system",
 * "streaming_f"): at every node, rho = sum_i f_i and the force-shifted
 * velocity u = (sum_i f_i c_i + F/2)/rho; the CMs k = T(u) f; the relaxation
 * k* = (I - K) k + K k_eq + (I - K/2) R with the Galilean-invariant k_eq and
 * the forcing CMs R of App. B; f* = T(u)^-1 k*; then streaming
 * f_i(x + c_i, t+1) = f*_i(x, t).  Velocities and their order are those of
 * Sec. II.A (opposite(i) = i +- 9).
 *
 * Conventions shared by every entry point:
 *   - Node index n = x + nx*(y + ny*z).  Per-node fields are structure of
 *     arrays: a scalar field is double[N]; a vector field is double[3*N] with
 *     component d at [d*N + n].  Population arrays are double[19*N] with
 *     population i at [i*N + n].
 *   - Pointers marked "host or device" are device pointers when on_device is
 *     non-zero (they must then be device memory of the handle's GPU), host
 *     pointers otherwise.  The caller owns every pointer it passes; the library
 *     never frees or retains caller memory past the call.
 *   - Every call is ordered on the HIP stream given to lbm_create.  Calls that
 *     write host memory synchronize that stream before returning; calls that
 *     read or write only device memory do not.
 *   - Errors: a negative lbm_status is returned and lbm_last_error() gives a
 *     message (thread-local).  Nothing is printed.  A handle on which a call
 *     failed with LBM_EDEVICE should be destroyed.
 *   - One handle must not be used from two threads at once.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 7

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,       /* bad argument or parameter */
    LBM_ENOMEM = -2,       /* device allocation failed */
    LBM_EDEVICE = -3,      /* HIP runtime error */
    LBM_EUNSTABLE = -4,    /* a stability check found a non-finite or non-positive density */
    LBM_EUNSUPPORTED = -5  /* valid request the library does not implement */
} lbm_status;

/* Storage precision of the populations.  Collision arithmetic is FP64 for
 * LBM_FP64 and FP32 otherwise.  Populations are stored as deviations
 * s_i = f_i - w_i rho0 from the rest equilibrium at the reference density. */
typedef enum {
    LBM_FP64 = 0,
    LBM_FP32 = 1,
    LBM_FP16_SHIFTED = 2,
    LBM_BF16_SHIFTED = 3
} lbm_precision;

/* Streaming pattern: two buffers (pull from the neighbours into the other
 * buffer) or one buffer updated in place (AA pattern, even/odd steps). */
typedef enum { LBM_AB = 0, LBM_AA = 1 } lbm_streaming;

/* Rounding of the stored populations.  Nearest (even) everywhere by default.
 * Stochastic (BF16 storage of the plain D3Q19 central-moment lattice only):
 * each post-collision population rounds up to the next BF16 value with
 * probability equal to the fraction of the BF16 step it lies above the lower
 * one, so rounding errors average out instead of repeating at neighbouring
 * nodes of a smooth field.  The random bits are counter-based: a 32-bit hash
 * of (seed, step count, node, population), so runs repeat bit for bit, and
 * A-B and AA agree bit for bit.  Not a method of the paper: a storage option. */
typedef enum { LBM_ROUND_NEAREST = 0, LBM_ROUND_STOCHASTIC = 1 } lbm_rounding;

typedef enum {
    LBM_FORCE_NONE = 0,
    LBM_FORCE_UNIFORM = 1,    /* F = force[0..2] at every node */
    LBM_FORCE_FIELD = 2,      /* F read from force_field (device, double[3*N]) */
    LBM_FORCE_KOLMOGOROV = 3  /* F_x = kolmogorov_amp * sin(2 pi y / ny), F_y = F_z = 0 */
} lbm_force_mode;

/* Moment space of the collision.  Central moments (Sec. II.B) are the
 * paper's method; raw moments are its N = I special case, the classical
 * raw-moment MRT written in the same basis (App. C): k = M f, the raw
 * equilibrium moments printed there, the raw moments of the forcing term of
 * App. B (eq. RMQ19), the same K, f* = M^-1 k*.  With K = I both give the
 * same populations.  For D3Q27 (timed in App. D, not written out) the raw
 * moments of the same equilibrium and forcing term are used. */
typedef enum { LBM_CENTRAL_MOMENTS = 0, LBM_RAW_MOMENTS = 1 } lbm_moment_space;

/* Lattice coupled to the flow (Sec. III multiphysics cases). */
typedef enum {
    LBM_COUPLED_NONE = 0,
    LBM_COUPLED_PHASE = 1,    /* two-phase flow with a conservative phase field (see below) */
    LBM_COUPLED_MAGNETIC = 2, /* magnetohydrodynamics with a vector magnetic lattice (see below) */
    LBM_COUPLED_SHAN_CHEN = 3, /* Shan-Chen pseudo-potential two-phase flow (see below) */
    LBM_COUPLED_COLOUR = 4    /* colour-gradient two-phase flow (see below) */
} lbm_coupling;

/* Two-phase flow (not in the paper, whose multiphase models are Shan-Chen and
 * the colour gradient): conservative Allen-Cahn phase field phi in [0, 1]
 * (P.-H. Chiu & Y.-T. Lin, J. Comput. Phys. 230, 2011) carried by a D3Q7
 * lattice in the form of A. Fakhari et al. (Phys. Rev. E 96, 2017), coupled
 * to pressure-based D3Q19 flow populations (zeroth moment p/cs^2, first
 * moment rho u; X. He, S. Chen & R. Zhang, J. Comput. Phys. 152, 1999;
 * H. Liang et al., Phys. Rev. E 97, 2018) collided with the CM scheme of
 * Sec. II.B.  rho = rho_light + phi (rho_heavy - rho_light); surface tension
 * F = mu grad(phi), mu = 4 beta phi (phi - 1)(phi - 1/2) - kappa lap(phi),
 * beta = 12 sigma / width, kappa = 3 sigma width / 2. */
typedef struct {
    double rho_light;         /* density where phi = 0, > 0 */
    double rho_heavy;         /* density where phi = 1, > 0 */
    double sigma;             /* surface tension, >= 0 */
    double width;             /* interface width W (lattice units), > 0 */
    double mobility;          /* M > 0; phase relaxation rate 1 / (4 M + 1/2) */
} lbm_phase_params;

/* Magnetohydrodynamics (Sec. III, Hartmann flow; the paper cites the magnetic
 * lattice without writing it out): induction equation on a D3Q7 vector
 * lattice in the form of P. J. Dellar (J. Comput. Phys. 179, 2002),
 * g_eq_{i,a} = w_i (b_a + c_i.(u b_a - b u_a) / cs^2), cs^2 = 1/4, one
 * relaxation rate 1 / (4 eta + 1/2); current j = curl b from the magnetic
 * non-equilibrium; the Lorentz force j x b (mu0 = 1) joins the external
 * force in the flow collision.  With walls_y, magnetic populations are
 * anti-bounced back so that b = b_wall on the walls. */
typedef struct {
    double eta;               /* magnetic diffusivity, > 0 */
    double b_wall[3];         /* field imposed at the y walls (walls_y = 1) */
} lbm_magnetic_params;

/* Shan-Chen two-phase flow (static-bubble case of Sec. III): pseudo-potential
 * psi = 1 - exp(-rho) and interaction force
 * F(x) = -G psi(x) sum_i w_i c_i psi(x + c_i) (X. Shan & H. Chen, Phys. Rev. E
 * 47, 1993) from the density of the step's populations; any uniform force
 * (force_mode LBM_FORCE_UNIFORM) adds to it; the sum enters the collision as
 * F.  Bulk pressure p = rho/3 + G psi^2 / 6.  No extra populations: one more
 * field (psi) and one more launch per step. */
typedef struct {
    double G;                 /* interaction strength (the paper: -5); finite */
} lbm_shan_chen_params;

/* Colour-gradient two-phase flow (App. E; the Rayleigh-Taylor case of
 * Sec. III): red and blue populations f^r, f^b; the total f collides with the
 * scheme of Sec. II.B towards h_eq = f_eq(rho, u) + rho (phi_i(alpha) - w_i),
 * phi_i = alpha, (1 - alpha)/12, (1 - alpha)/24 by |c_i|^2,
 * alpha = (rho_r alpha_r + rho_b alpha_b)/rho; the perturbation
 * (A/2)|grad phi| [w_i (c_i.grad phi)^2/|grad phi|^2 - B_i] adds interfacial
 * tension sigma = (2/9) A / omega; the recolouring
 * f^r,b = (rho_r,b / rho) f -/+ beta (rho_r rho_b / rho^2) cos(theta_i) rho phi_i(alpha)
 * separates the colours (phi = (rho_r - rho_b)/rho, grad phi from the isotropic
 * stencil, mirrored at the y walls); body force F = (rho - rho_ref) gravity.
 * Both colours are stored whole (rho0 is not used). */
typedef struct {
    double alpha_red;         /* rest fraction of red, in [0, 1); stable densities
                                 rho_r0 (1 - alpha_red) = rho_b0 (1 - alpha_blue) */
    double alpha_blue;        /* rest fraction of blue (the paper: 1/3) */
    double A;                 /* perturbation amplitude A_r + A_b >= 0 */
    double beta;              /* recolouring parameter in [0, 1] (the paper: 0.7) */
    double gravity[3];        /* g; F = (rho - rho_ref) g */
    double rho_ref;
} lbm_colour_params;

typedef struct {
    uint32_t abi_version;     /* must be LBM_ABI_VERSION */
    int32_t nx, ny, nz;       /* lattice nodes; periodic in x and z, and in y unless walls_y */
    int32_t q;                /* 19, or 27 for the D3Q27 CM lattice of App. D (FP64/FP32 storage,
                                 omega on the deviatoric moments, 1 elsewhere) */
    int32_t precision;        /* lbm_precision */
    int32_t streaming;        /* lbm_streaming */
    double omega;             /* shear rate of k5..k9, 1/(nu/cs^2 + 1/2), in (0, 2) (Sec. II.B) */
    double omega_bulk;        /* rate of k4; the paper's choice is 1 */
    double omega_hi[9];       /* rates of k10..k18; the paper's choice is 1 */
    double rho0;              /* reference density of the stored deviations (usually 1) */
    int32_t force_mode;       /* lbm_force_mode */
    double force[3];          /* LBM_FORCE_UNIFORM */
    double kolmogorov_amp;    /* LBM_FORCE_KOLMOGOROV */
    const double *force_field;/* LBM_FORCE_FIELD: device pointer, double[3*N], must stay valid
                                 while steps run */
    int32_t walls_y;          /* 1: stationary no-slip walls half a link outside y = 0 and
                                 y = ny - 1 (halfway bounce-back) */
    int32_t check_every;      /* > 0: every that many steps lbm_step checks that the density
                                 is finite and positive everywhere (FP64 reduction) */
    int32_t block_x, block_y; /* work-group shape of the step kernels (product a multiple of 64,
                                 at most 256); 0 = library default: whole x rows of up to 256
                                 nodes per work-group, one work-group of nx threads per row
                                 of 257..1024 nodes (where the staging rows fit in 64 KB of
                                 LDS; not for A-B with 16-bit storage, which keeps 256-wide
                                 direct work-groups there), the x-moving populations staged
                                 through LDS on periodic lattices */
    int32_t cache_policy;     /* population loads/stores: 0 = library default (non-temporal
                                 for staged steps and for A-B with 4- and 8-byte storage,
                                 cached otherwise), 1 = non-temporal (streaming) hints,
                                 2 = ordinary cached accesses */
    int32_t coupled;          /* lbm_coupling */
    lbm_phase_params phase;   /* LBM_COUPLED_PHASE: q = 19, FP64 or FP32, A-B, periodic, no
                                 external force, the paper's bulk and higher-order rates,
                                 rho0 = 1 */
    lbm_magnetic_params magnetic; /* LBM_COUPLED_MAGNETIC: q = 19, FP64 or FP32, A-B, the paper's
                                 bulk and higher-order rates; any external force mode */
    int32_t moments;          /* lbm_moment_space; LBM_RAW_MOMENTS: no coupled lattice and no
                                 network (lbm_set_mlp); with q = 27 the D3Q27 rates and forcing
                                 of the CM lattice, in raw moments */
    lbm_shan_chen_params shan_chen; /* LBM_COUPLED_SHAN_CHEN: q = 19, FP64 or FP32, A-B, periodic,
                                 force mode NONE or UNIFORM; any rates; initialised with
                                 lbm_init (f = f_eq(rho, u)) */
    lbm_colour_params colour; /* LBM_COUPLED_COLOUR: q = 19, FP64 or FP32, A-B, walls_y allowed,
                                 force mode NONE (gravity is in here), the paper's bulk and
                                 higher-order rates; initialised with lbm_init_colour; the
                                 populations of lbm_get/set_populations are red, those of
                                 lbm_get/set_coupled_populations blue */
    int32_t rounding;         /* lbm_rounding; LBM_ROUND_STOCHASTIC needs q = 19, central moments,
                                 LBM_BF16_SHIFTED, no coupled lattice and no network
                                 (LBM_EUNSUPPORTED otherwise) */
    uint32_t seed;            /* key of the stochastic rounding's random bits */
} lbm_params;

typedef struct lbm_handle lbm_handle;

/* Environment variables read by lbm_create (testing and measurement; none is
 * needed in normal use):
 *   LBM_OFF32=0         64-bit population addresses even where every array is
 *                       below 4 GiB (the path of larger lattices);
 *   LBM_ROW_STAGING=0/1 no staging of the x-moving populations / staging
 *                       wherever it is possible, overriding the default and
 *                       lbm_tune;
 *   LBM_XCD_CHUNK=c     a 1-D step grid in which each XCD sweeps runs of c
 *                       consecutive rows;
 *   LBM_COUPLED_FLAT=0  the 3-D grid of row work-groups instead of the flat
 *                       1-D grid for the two-phase, Shan-Chen and
 *                       colour-gradient step kernels;
 *   LBM_AA_EVEN_CACHED=0/1  with 16-bit storage, the AA even step's loads
 *                       with / without the streaming hint (default: without
 *                       up to 2^25 nodes).
 *   LBM_WAVES_PER_SIMD=n cap on the step kernels' resident wavefronts per
 *                       SIMD, set through their LDS allocation (default: 5
 *                       for 4- and 8-byte storage, none for 2-byte; 0: none).
 * None of them changes results: every path is tested bit for bit against the
 * default one. */

/* Fill *p with defaults: 32^3, q = 19, FP32, A-B, omega = 1, all other rates
 * 1, rho0 = 1, no force, periodic, no checks. */
void lbm_params_default(lbm_params *p);

/* Create a lattice on the current HIP device.  stream: a hipStream_t (NULL =
 * the default stream) on which all later calls of this handle are ordered.
 * Allocates the population buffer(s): 19*N elements each (two for LBM_AB).
 * Returns LBM_EINVAL for bad parameters, LBM_ENOMEM if the device is full. */
int lbm_create(const lbm_params *p, void *stream, lbm_handle **out);

/* Initialise at equilibrium from macroscopic fields (Sec. III: populations
 * start at the equilibrium of the initial fields, eq. EqQ19RM):
 * f_i(x, 0) = f_i^eq(rho(x), u(x)).  rho: double[N], u: double[3*N] (host or
 * device).  Resets the step counter to 0. */
int lbm_init(lbm_handle *h, const double *rho, const double *u, int on_device);

/* Advance nsteps >= 0 time steps.  Returns LBM_EUNSTABLE at the first failed
 * stability check (state left readable, step counter at the failed check). */
int lbm_step(lbm_handle *h, int64_t nsteps);

/* Macroscopic fields at the current time: rho = sum_i f_i (double[N]) and the
 * force-shifted u = (sum_i f_i c_i + F/2)/rho (double[3*N]); either may be
 * NULL.  diag (host, may be NULL) receives FP64 totals
 * [sum rho, sum rho u_x, sum rho u_y, sum rho u_z, 1/2 sum rho |u|^2,
 *  max |u|] over all nodes. */
int lbm_moments(lbm_handle *h, double *rho, double *u, double *diag, int on_device);

/* lbm_moments for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same fields and totals, computed by the same kernels, with the
 * per-work-group partial totals in a fixed 1 MiB device array of the library
 * (one per GPU, held until the process ends) instead of handle memory.
 * rho (double[N]), u (double[3*N]) and diag (double[6], the totals of
 * lbm_moments in the same order) are DEVICE pointers, each may be NULL.
 * Asynchronous: ordered on the handle's stream, no synchronization, no
 * allocation, no host copy.  The totals equal lbm_moments' up to the order of
 * the FP64 summation (the partials group several z planes per work-group).
 * Every call on one GPU uses that GPU's single array: calls that overlap in
 * time on one GPU (handles on different streams) race; order them.
 * Errors: LBM_EINVAL for a NULL handle or a lattice with more than 16384
 * step work-groups per z plane (the array's capacity; lbm_moments has no
 * such limit), LBM_EUNSUPPORTED for coupled lattices, LBM_EDEVICE if the
 * array's address cannot be found or a launch fails. */
int lbm_moments_noalloc(lbm_handle *h, double *rho, double *u, double *diag);

/* Copy the populations f_i(x, t) at the current time (before collision, the
 * state the paper's algorithm starts a step from) into f (double[19*N], host
 * or device), converting from the storage precision. */
int lbm_get_populations(lbm_handle *h, double *f, int on_device);

/* Replace the state by the populations f (double[19*N], host or device),
 * rounded to the storage precision.  The step counter is kept. */
int lbm_set_populations(lbm_handle *h, const double *f, int on_device);

/* Two-phase lattices (coupled = LBM_COUPLED_PHASE) start from lbm_init_phase
 * instead of lbm_init: phase populations at h_eq(phi, u), flow populations
 * at the paper's equilibrium at density rho(phi) plus (p/cs^2 - rho(phi))
 * times the rest weights.  phi, p: double[N]; u: double[3*N] (host or
 * device).  Resets the step counter.  On such a handle lbm_moments reports
 * rho(phi) and the force-shifted velocity, and lbm_get/set_populations the
 * flow populations g (double[19*N], pull order as for the plain lattice). */
int lbm_init_phase(lbm_handle *h, const double *phi, const double *p, const double *u, int on_device);

/* phi = sum of the phase populations and the pressure p = cs^2 (sum g + S0/2)
 * at the current time (double[N] each, host or device, either may be NULL). */
int lbm_phase_fields(lbm_handle *h, double *phi, double *p, int on_device);

/* Magnetic lattices (coupled = LBM_COUPLED_MAGNETIC) start from
 * lbm_init_magnetic: flow at f_eq(rho, u), magnetic populations at
 * g_eq(b, u).  rho: double[N]; u, b: double[3*N] (host or device).  Resets
 * the step counter.  lbm_moments then reports the velocity shifted by half
 * the total (external + Lorentz) force. */
int lbm_init_magnetic(lbm_handle *h, const double *rho, const double *u, const double *b, int on_device);

/* Magnetic field b = sum of the magnetic populations and current j (double[3*N]
 * each, host or device, either may be NULL) at the current time. */
int lbm_magnetic_fields(lbm_handle *h, double *b, double *j, int on_device);

/* Populations of the coupled lattice at the current time (double[q_c*N],
 * population k at [k*N + n]; D3Q7 order rest, -x, -y, -z, +x, +y, +z;
 * q_c = 7 for the phase field, 21 = 3 x 7 for the magnetic field with
 * k = 7 a + i for component a), host or device; set replaces them (step
 * counter kept). */
/* Colour-gradient lattice: f^k = (rho_k / rho) h_eq(rho, u) from the colour
 * densities rho_red, rho_blue (double[N], rho_red + rho_blue > 0) and u
 * (double[3N]) (host or device); resets the step count. */
int lbm_init_colour(lbm_handle *h, const double *rho_red, const double *rho_blue, const double *u, int on_device);
/* Colour densities (double[N] each, host or device; either may be NULL). */
int lbm_colour_fields(lbm_handle *h, double *rho_red, double *rho_blue, int on_device);
int lbm_get_coupled_populations(lbm_handle *h, double *out, int on_device);
int lbm_set_coupled_populations(lbm_handle *h, const double *in, int on_device);

/* Autotuner of the plain step kernel: runs 2 + trial_steps (rounded up to
 * even) real steps, three times in interleaved rounds, for each work-group
 * shape 256x1, 128x2, 64x4, 128x1, 64x2, 64x1 (those that fit the lattice;
 * for rows of 257..1024 nodes also nx x 1, staged only)
 * with and without non-temporal hints and, where a work-group spans whole x
 * rows (periodic; A-B, or the odd step of AA), with and without staging the
 * x-moving populations through LDS; keeps the fastest (by each candidate's best round) for later
 * lbm_step calls and reports it (block_x, block_y, cache_policy 1 =
 * non-temporal, 2 = cached, row_stage 1 = staged; each may be NULL).  The
 * state advances by the steps taken and the step counter counts them.  The
 * choice is cached for the process per (GPU architecture, lattice size, q,
 * precision, streaming, walls, general rates): a later call with the same key
 * applies it without running steps.  Not for coupled lattices or attached
 * networks (LBM_EUNSUPPORTED). */
int lbm_tune(lbm_handle *h, int32_t trial_steps, int32_t *block_x, int32_t *block_y, int32_t *cache_policy,
             int32_t *row_stage);

/* Number of steps taken since lbm_init. */
int64_t lbm_step_count(const lbm_handle *h);

/* Which plain step kernel lbm_step launches (not the learned or coupled
 * ones): 0 = one node per thread, 1 = x-moving populations staged through LDS
 * along whole rows (the default wherever possible; lbm_tune may choose
 * either); -1 for a NULL handle. */
int32_t lbm_step_variant(const lbm_handle *h);

/* Device bytes held by the handle (population buffers and tables). */
int64_t lbm_device_bytes(const lbm_handle *h);

int lbm_destroy(lbm_handle *h);

/* Message of the last failed call on this thread ("" if none). */
const char *lbm_last_error(void);

/* LBM_ABI_VERSION of the loaded library. */
int lbm_abi_version(void);

/* ---------------------------------------------------------------------------
 * Learned higher-order rates.  Not part of the paper, which fixes the rates of
 * the third- and fourth-order CMs k10..k18 to 1 (Sec. II.B): here a per-node
 * network sets them so that D3Q19 follows D3Q27 (App. D) more closely.  The
 * conserved (k0..k3), bulk (k4) and viscous (k5..k9) rates are never touched.
 *
 * Network: inputs x = (rho - 1, (k4 - rho)/rho, k10..k15 / rho,
 * (k16..k18 - rho/9)/rho) of the node's pre-collision CMs, each multiplied by
 * 1/scale_j; two ReLU layers of 32; outputs z; omega_hi_j = 1 + z_j.  If any
 * omega_hi_j is outside (0, 2) the node uses the paper's rates (all 1) and is
 * counted as a fallback.  Products run on BF16 MFMA with FP32 accumulation.
 * Parameters: LBM_MLP_NPARAM floats W1[32][11], b1[32], W2[32][32], b2[32],
 * W3[9][32], b3[9] (W[out][in], row-major).
 * ------------------------------------------------------------------------- */
#define LBM_MLP_NPARAM 1737

typedef struct lbm_mlp lbm_mlp;

/* params: host float[LBM_MLP_NPARAM] or NULL (all zero: the paper's rates);
 * scales: host float[11], all > 0.  All calls are ordered on `stream`.
 * Errors: LBM_EINVAL (NULL out or scales, a scale <= 0, a non-finite
 * parameter), LBM_EDEVICE (no HIP device), LBM_ENOMEM (device buffers). */
int lbm_mlp_create(const float *params, const float *scales, void *stream, lbm_mlp **out);
int lbm_mlp_set_params(lbm_mlp *m, const float *params);   /* host; resets Adam moments */
int lbm_mlp_get_params(const lbm_mlp *m, float *params);   /* host */
int lbm_mlp_set_scales(lbm_mlp *m, const float *scales);   /* host float[11] */
int lbm_mlp_destroy(lbm_mlp *m);

/* Use network m for the rates of k10..k18 in every later lbm_step of h (NULL
 * detaches).  h must be D3Q19 with FP32, FP16 or BF16 storage; m must outlive
 * its use by h. */
int lbm_set_mlp(lbm_handle *h, const lbm_mlp *m);

/* Number of node updates that fell back to the paper's rates since the
 * network was attached (synchronizes the handle's stream). */
int64_t lbm_fallback_count(lbm_handle *h);

/* Training.  One sample is the one-step map of h's current state f(t) (h:
 * D3Q19, FP32, A-B, periodic, no force, network m attached): the loss is the
 * mean over nodes of sum_k ((m_k(f(t+1)) - target_k) / sigma_k)^2 with the raw
 * moments m = (rho, j_x, j_y, j_z, Pi_xx, Pi_yy, Pi_zz, Pi_xy, Pi_xz, Pi_yz) of
 * the populations after the step.  target: device float[10*N] (component k at
 * [k*N + n]).  The gradient is added to m's accumulator; h's state and step
 * counter are unchanged.  *loss (host, may be NULL) receives the loss. */
int lbm_mlp_zero_grad(lbm_mlp *m);
int lbm_mlp_accumulate_grad(lbm_mlp *m, lbm_handle *h, const float *target, const double sigma[10], double *loss);

/* Rollout training: the loss of lbm_mlp_accumulate_grad taken after each of
 * `steps` learned steps from h's current state f(t) (step k against target
 * k, k = 1..steps) and averaged over the steps with weights w_k:
 *   L = (1/steps) sum_k w_k L_k,
 *   L_k = mean_nodes sum_j ((m_j(f(t+k)) - target_kj) / sigma_j)^2.
 * The gradient is back-propagated through every step, including the way each
 * step's rates depend on the state it starts from, and added to m's
 * accumulator (steps = 1 with w = 1 gives lbm_mlp_accumulate_grad's result).
 * targets: device float[steps][10][N] (target k, component j at
 * [((k-1)*10 + j)*N + n], n = x + nx (y + ny z)); step_weight: host
 * double[steps], each > 0, or NULL (all 1); dstate: device float[19*N] or
 * NULL, receives dL/df_i(x, t) at [i*N + n]; step_loss: host double[steps]
 * or NULL, receives L_1..L_steps; *loss (host, may be NULL) receives L.  h as
 * for lbm_mlp_accumulate_grad; its state and step counter are unchanged.  m
 * keeps `steps` states of h's size as scratch (grown on demand, freed by
 * lbm_mlp_destroy).  Errors: LBM_EINVAL (NULL argument, steps outside
 * [1, LBM_MLP_MAX_ROLLOUT], sigma or a weight <= 0, m not attached to h),
 * LBM_EUNSUPPORTED (h not as required), LBM_ENOMEM. */
#define LBM_MLP_MAX_ROLLOUT 128
int lbm_mlp_accumulate_rollout_grad(lbm_mlp *m, lbm_handle *h, const float *targets, int32_t steps,
                                    const double sigma[10], const double *step_weight, float *dstate,
                                    double *step_loss, double *loss);

/* Weight w_E >= 0 (default 0) of a kinetic-energy term in m's later rollout
 * losses: L gains (w_E / steps) sum_k ((E_k - T_k) / T_k)^2, with E_k =
 * 1/2 sum over the lattice of |j|^2 / rho of the populations after step k and
 * T_k the same of target k's moments (rho, j); its gradient is
 * back-propagated with the rest.  step_loss keeps reporting the moment terms
 * L_k only.  Not used by lbm_mlp_accumulate_grad. */
int lbm_mlp_set_energy_weight(lbm_mlp *m, double w);
int lbm_mlp_get_grad(const lbm_mlp *m, double *grad);      /* host double[LBM_MLP_NPARAM] */
/* One Adam update of the FP32 master parameters with the accumulated gradient. */
int lbm_mlp_adam_step(lbm_mlp *m, double lr, double beta1, double beta2, double eps);

/* Root mean square over all nodes of each of the 11 raw network inputs
 * (before the 1/scale factors) for h's current state (D3Q19, FP32 or 16-bit
 * storage): the natural input scales.  rms: host double[11]. */
int lbm_feature_rms(lbm_handle *h, double rms[11]);

/* Training data: D3Q27 populations f27 (device double[27*n], App. D order) ->
 * D3Q19 populations f19 with the same 19 shared raw moments (device
 * double[19*n], may be NULL) and the 10 raw moments above (device
 * float[10*n], may be NULL).  Ordered on `stream`. */
int lbm_project_q27(const double *f27, int64_t n, double *f19, float *moments, void *stream);

/* Memory-bandwidth reference with the step's access pattern (not part of the
 * method; for measuring how close a step comes to what its loads and stores
 * alone reach).  Copies q arrays of n elements of elem_bytes each, array k at
 * element offset k*n of src (device), to the same places in dst (device, not
 * overlapping src): each thread reads its part of all q arrays, then writes
 * them, as the A-B step does without its collision and neighbour shifts.
 * q: 19 or 27; elem_bytes: 2, 4 or 8 (the storage types); lane_bytes: bytes
 * each thread moves per array -- 0 or elem_bytes (one element, as the step),
 * or 8 or 16 (wider accesses; larger than elem_bytes and dividing
 * n * elem_bytes); nt != 0: the step's non-temporal (streaming) hints.  n = 0
 * enqueues nothing.  Ordered on `stream` (NULL: the default stream),
 * asynchronous.  Returns LBM_EINVAL for a NULL buffer, n < 0 or beyond 2^31
 * work-groups of 256, or another q, element or lane size; LBM_EDEVICE if the
 * launch fails. */
int lbm_stream_copy(const void *src, void *dst, int64_t n, int32_t q, int32_t elem_bytes, int32_t lane_bytes,
                    int32_t nt, void *stream);

/* ---------------------------------------------------------------------------
 * Ensembles: many independent periodic cubic boxes (different sides and
 * viscosities, no force) advanced together, one launch per step over a
 * (box, 256-node tile) work list, walked by a fixed number of work-groups
 * (one per tile by default; lbm_ensemble_tune tries persistent grids of
 * 2..64 work-groups per compute unit); the step loop is captured in a HIP
 * graph and replayed.  Same collision as a single lattice (Sec. II.B for q =
 * 19, App. D for q = 27); A-B streaming; FP32 or FP64 storage.
 * ------------------------------------------------------------------------- */
typedef struct lbm_ensemble lbm_ensemble;

typedef struct {
    int32_t n;    /* box side (nodes), 2..1024 */
    double omega; /* shear rate of the box, in (0, 2) */
} lbm_box;

/* stream: hipStream_t, or NULL for a stream the ensemble creates and owns
 * (the null stream cannot be captured into a graph).  Boxes start at rest. */
int lbm_ensemble_create(const lbm_box *boxes, int32_t nboxes, int32_t q, int32_t precision, void *stream,
                        lbm_ensemble **out);
/* f = f_eq(rho, u) in box `box` (rho: double[n^3], u: double[3 n^3], host or device). */
int lbm_ensemble_init(lbm_ensemble *e, int32_t box, const double *rho, const double *u, int on_device);
/* Learned rates in every box (D3Q19, FP32); NULL detaches. */
int lbm_ensemble_set_mlp(lbm_ensemble *e, const lbm_mlp *m);
int lbm_ensemble_step(lbm_ensemble *e, int64_t nsteps);
/* Per-box FP64 kinetic energy 1/2 sum rho |u|^2 and mass sum rho (host
 * double[nboxes] each, either may be NULL; synchronizes). */
int lbm_ensemble_energy(lbm_ensemble *e, double *ke, double *mass);
int lbm_ensemble_get_populations(lbm_ensemble *e, int32_t box, double *f, int on_device);
int64_t lbm_ensemble_nodes(const lbm_ensemble *e);
int64_t lbm_ensemble_step_count(const lbm_ensemble *e);
int64_t lbm_ensemble_fallback_count(lbm_ensemble *e);
/* Autotuner: times `trial_steps` steps (rounded up to even) for each
 * candidate launch -- 2, 4, 8, 16, 32 or 64 persistent work-groups per
 * compute unit, or one work-group per tile -- and keeps the fastest
 * (*grid_out, may be NULL).  It advances the state by those steps; call it
 * before lbm_ensemble_init (the rest state is a fixed point) to leave the
 * state untouched. */
int lbm_ensemble_tune(lbm_ensemble *e, int32_t trial_steps, int32_t *grid_out);
int lbm_ensemble_destroy(lbm_ensemble *e);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */

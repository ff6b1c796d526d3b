/*
 * lbm.h - C ABI of liblbm.so, the MI355X (gfx950) D2Q9 lattice Boltzmann library for the
 * Onsager-regularized (OReg) scheme with the guided equilibrium (GEq) of Jonnalagadda,
 * Rocchia and Succi, "Generalized Onsager-Regularized Lattice Boltzmann Method for
 * error-free Navier-Stokes models on standard lattices" (arXiv 2602.21242).
 *
 * One time step (eq:lbe) pull-streams the nine populations of every node, takes the
 * moments rho, rho u and the second moment, builds the guided equilibrium (eq:guidedEq),
 * the OReg non-equilibrium population (eq:oreg), optionally the partial
 * (eq:partial-corrections) or complete (eq:complete-corrections) correction populations,
 * and relaxes with tau = nu/theta + 1/2. Plain lattice BGK (with the guided equilibrium)
 * is available for comparison. The box is doubly periodic.
 *
 * Conventions shared by every entry point
 *  - Grid: nx x ny nodes, x fastest. Caller-side fields are dense row-major [ny][nx]
 *    arrays; caller-side population arrays are dense [9][ny][nx], populations numbered as
 *    in the paper's D2Q9 figure: 0 (0,0), 1 (1,0), 2 (0,1), 3 (-1,0), 4 (0,-1), 5 (1,1),
 *    6 (-1,1), 7 (-1,-1), 8 (1,-1).
 *  - Pointers named d_* are device pointers on the device that is current when lbm_init
 *    is called; the library never dereferences them on the host.
 *  - Ownership: the caller owns every device buffer (the workspace included) and the HIP
 *    stream. The library never allocates or frees device memory; it owns only the host
 *    context object, freed by lbm_destroy.
 *  - Asynchrony: lbm_init, lbm_step, lbm_moments, lbm_get_populations,
 *    lbm_set_populations and lbm_adjoint* enqueue work on the context's stream and return
 *    without waiting; lbm_invariants waits for the stream.
 *  - Errors: every call returns an lbm_status; no C++ exception crosses the ABI.
 *    lbm_last_error() returns a thread-local description of the last failure.
 *    Invalid arguments are rejected before any work is enqueued. After LBM_ERR_HIP from
 *    lbm_step or lbm_adjoint* (work already enqueued) the context's state and time are
 *    unspecified; lbm_destroy is still valid. Non-finite populations are not checked per
 *    step; lbm_invariants reports them.
 *  - Compute type: FP64 when storage is LBM_F64, FP32 otherwise. Adjoint inputs and
 *    outputs use the compute type. Stores round to nearest even. With LBM_F32 storage the
 *    collision takes populations 0, 1 and 2 from mass and momentum conservation (the same
 *    values in exact arithmetic), so FP32 rounding adds no drift of mass or momentum; with
 *    LBM_F16 storage and the OReg models it does so in FP16 precision: the axis populations
 *    are rounded to nearest even, the momentum they then miss goes to the four diagonal
 *    populations in a combination that changes no other moment of second order or lower,
 *    each diagonal is rounded once with its share, and g*_0 takes the mass (the stored values
 *    of a node keep its mass up to the rounding of g*_0 and its momentum up to that of the
 *    four diagonals); FP64 and BF16 storage and LBGK with FP16 storage use the direct form.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_ERR_INVALID_ARGUMENT = 1,   /* bad parameter, null pointer or out-of-range enum */
  LBM_ERR_UNSUPPORTED = 2,        /* valid request the library does not implement */
  LBM_ERR_WORKSPACE_TOO_SMALL = 3,/* workspace_bytes below lbm_workspace_bytes() */
  LBM_ERR_HIP = 4,                /* a HIP runtime call or kernel launch failed */
  LBM_ERR_NONFINITE = 5,          /* lbm_invariants found a NaN or infinite population */
  LBM_ERR_STATE = 6               /* call not valid in the context's current state */
} lbm_status;

/* Collision models (Sec. 4 of the paper): LBGK, uncorrected OReg (eq:oreg), partially
 * corrected (eq:partial-corrections), completely corrected (eq:complete-corrections). */
typedef enum {
  LBM_BGK = 0,
  LBM_OREG_UC = 1,
  LBM_OREG_PARTIAL = 2,
  LBM_OREG_COMPLETE = 3
} lbm_model;

/* Element types. Populations are stored shifted, g_i = f_i - w_i(theta) rho0, where
 * w_i(theta) is the guided equilibrium at rest: (1-theta)^2, theta(1-theta)/2, theta^2/4. */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_BF16 = 2, LBM_F16 = 3 } lbm_dtype;

/* Streaming pattern: two buffers (A-B), or one buffer updated in place (AA). */
typedef enum { LBM_AB = 0, LBM_AA = 1 } lbm_pattern;

typedef struct {
  int32_t nx, ny;        /* periodic box, 1 <= nx, ny; with pitch = (nx+63)/64*64 (rows of whole
                            64-node groups): pitch*ny < 2^31, and 9*pitch*E < 2^31 bytes, E the
                            larger of the storage and compute element sizes (8 for LBM_F64, else
                            4), because the kernels address a lattice row with 32-bit byte
                            offsets; wider rows give LBM_ERR_INVALID_ARGUMENT */
  double theta;          /* reduced lattice temperature, 0 < theta < 1 */
  double nu;             /* lattice viscosity > 0; tau = nu/theta + 1/2 (nu = theta (tau - 1/2)) */
  double rho0;           /* reference density > 0 (storage shift) */
  int32_t model;         /* lbm_model */
  int32_t storage;       /* lbm_dtype of the stored populations */
  int32_t pattern;       /* lbm_pattern */
  int32_t ckpt_stride;   /* adjoint checkpoint spacing s in steps (values above record_steps
                            count as record_steps); 0: ceil(sqrt(record_steps)). The reverse
                            sweep recomputes every segment but the last from its checkpoint,
                            so s >= record_steps (one segment, the moments of every step kept:
                            record_steps x 5 x sizeof(compute type) bytes per node) recomputes
                            nothing */
  int64_t record_steps;  /* 0: no adjoint; N > 0: checkpoint the first N steps for lbm_adjoint */
  int32_t two_step;      /* two steps per launch (see lbm_steps_per_launch): 0 where the grid is
                            large enough for it to pay, 1 wherever the layout allows, -1 never */
  int32_t walls;         /* 0: doubly periodic. 1: the columns x = 0 and x = nx - 1 are solid
                            nodes with fullway bounce-back (the isothermal shocktube, Sec. 5):
                            instead of colliding, a wall node sends each population back the way
                            it came, so the wall lies halfway to the first fluid node and the fluid
                            is x = 1 .. nx - 2 (y stays periodic). Requires nx >= 3
                            (INVALID_ARGUMENT); the AA pattern and record_steps > 0 give
                            LBM_ERR_UNSUPPORTED. lbm_moments and lbm_invariants include the wall
                            nodes (their populations are part of the conserved total). */
} lbm_params;

typedef struct lbm_ctx lbm_ctx; /* opaque host-side context */

/* Bytes of device workspace lbm_init needs for *p (populations, reduction scratch, and,
 * when record_steps > 0, checkpoints, moment records and adjoint populations).
 * Returns LBM_ERR_INVALID_ARGUMENT for invalid parameters. */
lbm_status lbm_workspace_bytes(const lbm_params* p, size_t* bytes);

/* Create a context and set the state at time n = 0 to the guided equilibrium
 * f_i = f_i^eq(rho, u) of the given fields (eq:guidedEq).
 *   d_workspace    device buffer of at least lbm_workspace_bytes(p) bytes, 256-byte
 *                  aligned, owned by the caller and used exclusively by this context
 *                  until lbm_destroy.
 *   hip_stream     hipStream_t on which all of this context's work is enqueued (NULL:
 *                  the null stream).
 *   d_rho          FP64 [ny][nx] density, or NULL for rho = rho0 everywhere.
 *   d_ux, d_uy     FP64 [ny][nx] velocity components (required).
 *   out            receives the new context. */
lbm_status lbm_init(const lbm_params* p, void* d_workspace, size_t workspace_bytes,
                    void* hip_stream, const double* d_rho, const double* d_ux,
                    const double* d_uy, lbm_ctx** out);

/* Advance n >= 0 time steps (eq:lbe: collide, then stream); n = 0 does nothing and n < 0
 * is LBM_ERR_INVALID_ARGUMENT. While the context records (record_steps > 0), the state at
 * every checkpoint time below record_steps is saved and the steps of the last checkpoint
 * segment also write their moments for the reverse sweep; stepping past record_steps is
 * allowed but disables lbm_adjoint. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/* Density and velocity rho = sum_i f_i, u = sum_i c_i f_i / rho (the macroscopic densities the
 * paper defines from the populations right after eq:lbe, Sec. 1) of the pre-collision
 * state f^n at the current time n, written to FP64 or FP32 [ny][nx] arrays
 * (out_dtype LBM_F64 or LBM_F32; the 16-bit types give LBM_ERR_UNSUPPORTED). Any output
 * pointer may be NULL. */
lbm_status lbm_moments(lbm_ctx* ctx, lbm_dtype out_dtype, void* d_rho, void* d_ux, void* d_uy);

/* Unshifted pre-collision populations f^n as a dense [9][ny][nx] array of out_dtype
 * (LBM_F64 or LBM_F32; the 16-bit types give LBM_ERR_UNSUPPORTED). d_f must not be NULL. */
lbm_status lbm_get_populations(lbm_ctx* ctx, lbm_dtype out_dtype, void* d_f);

/* Replace the state at the current time by the FP64 [9][ny][nx] populations d_f (not
 * NULL; rounded to the storage type). Disables lbm_adjoint for the recorded run. */
lbm_status lbm_set_populations(lbm_ctx* ctx, const double* d_f);

/* FP64 totals of the pre-collision state: out[0] = sum_x rho, out[1] = sum_x rho u_x,
 * out[2] = sum_x rho u_y, with rho and rho u the population moments of Sec. 1. They are the
 * quantities every collision model keeps (eq:density-momentum: the equilibrium carries the
 * node's rho and rho u; eq:genOReg-constraints: the corrected non-equilibrium populations
 * carry no mass and no momentum), so streaming and collision conserve them, except the
 * uncorrected OReg model's momentum. Computed on the device in FP64, the only FP64
 * reduction of the reduced-precision paths. Waits for the stream. Returns
 * LBM_ERR_NONFINITE (with out filled) if any population is NaN or infinite. */
lbm_status lbm_invariants(lbm_ctx* ctx, double out[3]);

/* For callers that cannot allocate or hand the library device memory for scratch (code
 * around HIP graph capture, tight serving loops, harnesses that forbid allocation): the
 * totals and status of lbm_invariants, from the same kernels in the same order (bit-identical
 * results), with the reduction's 1024 x 4 FP64 partial sums and 4-entry result kept in a
 * static device array of 32 800 bytes instead of the context's workspace. Allocates nothing;
 * the library holds one such array on every device it runs on until the process ends. The
 * array's size does not depend on the grid, so every grid lbm_init accepts fits. Every call
 * on a device shares that device's array and overwrites it completely (nothing to clear):
 * calls that overlap in time on one device (other contexts or streams) race and may return
 * each other's totals. Waits for the stream. */
lbm_status lbm_invariants_static(lbm_ctx* ctx, double out[3]);

/* Discrete adjoint of the recorded run (requires record_steps = N > 0 and lbm_time = N).
 * Given dJ/drho, dJ/du_x, dJ/du_y of the moments at t = N (compute-type [ny][nx]
 * arrays; d_rho_bar may be NULL for zero), writes dJ/du_x and dJ/du_y of the initial
 * velocity fields passed to lbm_init (rho held fixed) to d_ux0_bar, d_uy0_bar.
 * Uses the checkpoints of the forward run (every ckpt_stride steps, sqrt(N) by default) and
 * recomputes each segment but the last, whose moments the forward run kept; the state at
 * t = N is restored before returning, so the call may be repeated (a repeated call also
 * recomputes the last segment unless there is only one). */
lbm_status lbm_adjoint(lbm_ctx* ctx, const void* d_rho_bar, const void* d_ux_bar,
                       const void* d_uy_bar, void* d_ux0_bar, void* d_uy0_bar);

/* Population-level discrete adjoint of the recorded run: given fbar^N = dJ/df^N
 * (compute-type dense [9][ny][nx]), writes fbar^0 = dJ/df^0 to d_fbar0 (same layout).
 * Same requirements and restoration as lbm_adjoint. */
lbm_status lbm_adjoint_populations(lbm_ctx* ctx, const void* d_fbarN, void* d_fbar0);

/* Completed time steps n, or -1 for a NULL context. */
int64_t lbm_time(const lbm_ctx* ctx);

/* Time steps one kernel launch of lbm_step advances for this context: 2 where the two-step
 * LDS-staged kernel applies, else 1 (-1 for a NULL context). It applies to the A-B pattern
 * (every storage type and model), no walls, nx a multiple of 512, more than 2^15 storage
 * positions and two_step >= 0; with two_step = 0 also only where the grid gives at least
 * three quarters of the device's compute units a block of 2 or more rows x 512 columns
 * (roughly (nx/512) floor(ny/2) >= 3 CUs/4), below which the single-step kernel is faster.
 * A pair of steps never passes over a checkpoint time of a recorded run. Results do not
 * depend on it: two steps in one launch are bit-identical to two single steps. */
int32_t lbm_steps_per_launch(const lbm_ctx* ctx);

const char* lbm_status_string(lbm_status s);

/* Thread-local text of the last failure on the calling thread ("" if none). */
const char* lbm_last_error(void);

/* Free the host context (does not synchronise the stream or free caller memory). */
void lbm_destroy(lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */

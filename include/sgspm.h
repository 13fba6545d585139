/*
 * sgspm.h - C ABI of the MI355X (gfx950) library for one time step of the
 * symmetric Gauss-Seidel projection method (SGSPM) for the Landau-Lifshitz
 * equation, and of its adjoint.
 *
 * Method (Miao & Xie, "Improved Energy Stable Symmetric Gauss-Seidel Projection
 * Method for Micromagnetics Simulations"):
 *   model      §2, eq. (c1-large): m_t = -m x h - alpha m x (m x h), |m| = 1,
 *              h = eps Lap m - Q (m2 e2 + m3 e3) + h_s + h_e, Neumann BC
 *              (eq. boundary-large);
 *   SGSPM      §3.2: Step 1 forward then backward Gauss-Seidel sweep with
 *              g_i = (I - eps dt Lap_h)^{-1}(m_i + dt f_i); Step 2 heat flow
 *              (I - alpha eps dt Lap_h) m*** = m** + alpha dt f**; Step 3
 *              projection m^{n+1} = m*** / |m***|;
 *   GSPM       §3.1: forward sweep only, then Steps 2 and 3.
 *
 * Discretisation (the paper states none; these readings are shared with the
 * CPU oracle as a specification): cell-centred cells, 7-point Lap_h with
 * mirror ghosts (exactly diagonalised by DCT-II/III), stray field
 * h_s = -N (*) m with the Newell cell-averaged tensor (point-dipole form for
 * offsets beyond 20 cells in max norm) by 2x zero-padded FFT.  The "f" of
 * every Gauss-Seidel stage is evaluated at the latest component values.
 *
 * Layout of every field argument: device memory, contiguous [3][nz][ny][nx],
 * x fastest, of the plan's precision (float for SGSPM_FP32, double for
 * SGSPM_FP64).  The caller owns every pointer it passes; the library never
 * frees caller memory.  All calls are asynchronous on the plan's HIP stream
 * except sgspm_energy and sgspm_check, which synchronise it.
 *
 * Errors: every function returns 0 (SGSPM_OK) or a negative code;
 * sgspm_last_error() returns a thread-local message for the last failure.
 * Parameters are validated on the host before any HIP call.
 */
#ifndef SGSPM_H
#define SGSPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SGSPM_OK = 0,
  SGSPM_EINVAL = -1,       /* bad argument (null pointer, non-positive size, ...) */
  SGSPM_EUNSUPPORTED = -2, /* valid but not implemented (e.g. an extent with a prime factor above 5) */
  SGSPM_ENOMEM = -3,       /* device allocation failed */
  SGSPM_EHIP = -4,         /* a HIP runtime call failed */
  SGSPM_ENUMERIC = -5      /* a projection met |m***| = 0 or a non-finite value */
};

enum { SGSPM_TERM_EXCHANGE = 1, SGSPM_TERM_ANISO = 2, SGSPM_TERM_STRAY = 4, SGSPM_TERM_ZEEMAN = 8 };
enum { SGSPM_UNITS_SI = 0, SGSPM_UNITS_REDUCED = 1 };
enum { SGSPM_FP32 = 0, SGSPM_FP64 = 1 };
/* SGS: SGSPM (§3.2) with every f of the sweeps at the latest component values;
 * GS: GSPM (§3.1), same reading; SGS_FF: SGSPM with f frozen at m^n through
 * both sweeps and evaluated once more at m** for Step 2 (two stray-field
 * evaluations per step instead of six; the efficiency direction of the
 * Conclusion and the §3.1 remark on where h_s is evaluated). */
enum { SGSPM_SCHEME_SGS = 0, SGSPM_SCHEME_GS = 1, SGSPM_SCHEME_SGS_FF = 2 };

/* Problem statement (paper §2 and §3): grid, cell size, constants, time step. */
typedef struct {
  int32_t nx, ny, nz;   /* cells; each a product of 2, 3 and 5 (1 included), nx <= 2048,
                           ny, nz <= 1024.  Rows must fit one tile: nx <= 2048 (FP32) / 1024 (FP64)
                           without the stray field, nx <= 1024 with it (its tensor is transformed
                           in FP64 at either precision).  With the stray field the last axis of
                           extent > 1 among (ny, nz) is at most 512 (FP32) / 256 (FP64) */
  double dx, dy, dz;    /* cell edges: metres (SI) or reduced lengths */
  int32_t units;        /* SGSPM_UNITS_SI or SGSPM_UNITS_REDUCED */
  double A, Ms, Ku;     /* SI only: exchange J/m, saturation A/m, uniaxial J/m^3 (easy axis x) */
  double eps, Q;        /* REDUCED only: the paper's epsilon and Q */
  double dt;            /* seconds (SI) or reduced time */
  uint32_t terms;       /* bitmask of SGSPM_TERM_* */
  int32_t precision;    /* SGSPM_FP32 or SGSPM_FP64 */
  int32_t scheme;       /* SGSPM_SCHEME_SGS (default), SGSPM_SCHEME_GS or SGSPM_SCHEME_SGS_FF */
  int32_t batch;        /* independent runs of the same grid and constants stepped together
                           (0 or 1: one run).  A batched plan (2 <= batch <= 256) takes fields
                           of shape [3][batch][nz][ny][nx], each run with its own alpha and
                           applied field (sgspm_step_batch); SGS or GS scheme, no source term,
                           ny * nz even, and grids whose heat solve is the fused y-z kernel */
} sgspm_params;

typedef struct sgspm_plan_s* sgspm_plan_t;

/* Host-only checks of a parameter set (no HIP call).  Returns 0 or
 * SGSPM_EINVAL / SGSPM_EUNSUPPORTED with a message. */
int sgspm_validate(const sgspm_params* p);

/* The non-dimensional constants the plan will use: out[0] = eps (m^2 in SI,
 * reduced otherwise), out[1] = Q, out[2] = dt (reduced time), out[3] = field
 * scale (h_e = B * out[3] for B in tesla; 1 in reduced units), out[4] =
 * energy scale (multiplies reduced energy x volume: mu0 Ms^2 in SI, else 1).
 * Host only. */
int sgspm_reduced_constants(const sgspm_params* p, double out[5]);

/* Build a plan: validates, allocates the workspace (device), builds the
 * FP64 twiddle / eigenvalue tables and, if SGSPM_TERM_STRAY, computes the
 * Newell tensor and its spectrum on the GPU in FP64.  hip_stream is a
 * hipStream_t (0 = default stream).  The plan owns its workspace. */
int sgspm_plan(const sgspm_params* p, void* hip_stream, sgspm_plan_t* out);

/* One SGSPM (or GSPM) step, in place: m^n -> m^{n+1} (paper §3.2 / §3.1).
 *   m      device [3][nz][ny][nx], in/out
 *   alpha  damping (>= 0), per call
 *   h_e    applied field, host double[3]: tesla (SI, B = mu0 H) or reduced
 *   src    optional device [3][nz][ny][nx] source s (reduced units, rate per
 *          reduced time) added as dt * s_i to every Gauss-Seidel component
 *          update of Step 1 (forcing of a manufactured solution, §5.1); or NULL.
 * A zero or non-finite |m***| sets a device flag reported by sgspm_check. */
int sgspm_step(sgspm_plan_t plan, void* m, double alpha, const double h_e[3], const void* src);

/* nsteps steps of sgspm_step with the same alpha and h_e and no source, in place,
 * asynchronous: the first call for a given (m, alpha, h_e) captures one step as a
 * HIP graph (on a private stream of the plan) and every step replays it, which
 * removes the host's launch overhead from launch-bound grids (films, strips).
 * A call with another m, alpha or h_e captures again.  Results equal nsteps
 * calls of sgspm_step bit for bit. */
int sgspm_steps(sgspm_plan_t plan, void* m, int nsteps, double alpha, const double h_e[3]);

/* sgspm_step, and the spectral radii of that step's sweep matrices (paper §4,
 * eqs. GS-matrix and SGS-matrix: G_GS = (D - L)^{-1} U and
 * G_SGS = (D - U)^{-1} L (D - L)^{-1} U).  Their entries are the coefficients
 * c_i^s = eps dt Lap_h g_i^s of the step's precession solves, acting cell by
 * cell, so each cell has its own 3x3 matrices; rho_out (host double[2]) =
 * {max over cells of rho(G_GS), max over cells of rho(G_SGS)}, computed in FP64
 * from the solves as stored.  D - U takes the signs of the splitting of the
 * matrix of eq. M (the printed matrix has its off-diagonal signs flipped).  For
 * a GSPM plan rho_out[1] is NaN.  Synchronises the stream. */
int sgspm_step_spectral_radius(sgspm_plan_t plan, void* m, double alpha, const double h_e[3], const void* src,
                               double rho_out[2]);

/* Energies of m (paper §2, with the 1/2 factors that make h = -dE/dm):
 * e_out = {total, exchange, anisotropy, stray, zeeman}, host double[5], in
 * joules (SI) or reduced energy x volume.  FP64 accumulation with a fixed
 * reduction tree (deterministic).  Synchronises the stream. */
int sgspm_energy(sgspm_plan_t plan, const void* m, const double h_e[3], double e_out[5]);

/* max over cells of | |m| - 1 | (the unit-length constraint that the projection
 * of Step 3 restores), FP64, into host *out.  Synchronises the stream. */
int sgspm_unit_error(sgspm_plan_t plan, const void* m, double* out);

/* Effective field h_eff = eps Lap_h m - Q(m2 e2 + m3 e3) + h_s + h_e (paper §2)
 * of m into h_out (device [3][nz][ny][nx], reduced units). */
int sgspm_field(sgspm_plan_t plan, const void* m, const double h_e[3], void* h_out);

/* Stray field h_s = -N (*) m alone into hs_out (device [3][nz][ny][nx]). */
int sgspm_stray(sgspm_plan_t plan, const void* m, void* hs_out);

/* Heat-type solve of §3 (Step 1 with s = 1, Step 2 with s = alpha):
 * g = (I - s eps dt Lap_h)^{-1} r for one scalar field r (device [nz][ny][nx]);
 * r and g may alias. */
int sgspm_heat_solve(sgspm_plan_t plan, const void* r, double s, void* g);

/* The demagnetising tensor the stray field uses, component comp (0..5 = xx,
 * yy, zz, xy, xz, yz), in real space and FP64, exactly as the plan computes it
 * before transforming it: the Newell-Williams-Dunlop cell-averaged tensor for
 * offsets up to 20 cells in max norm, the point-dipole tensor beyond, on the
 * zero-padded grid out = device double [Pz][Py][Px] (P_a = 2 n_a for n_a > 1,
 * else 1), offset d stored at d mod P, zero where |d_a| > n_a - 1.  Lengths in
 * units of the largest cell edge (the tensor is scale free).  For checking the
 * plan-time precomputation; SGSPM_EINVAL if the plan has no stray field. */
int sgspm_demag_tensor(sgspm_plan_t plan, int comp, void* out);

/* Adjoint of one step (the chain rule of the step above; the paper has none):
 * given m_n (the state the step starts from) and lam = dL/dm^{n+1}, overwrite
 * lam with dL/dm^n and ADD dL/dh_e^n (3 values, per unit of the h_e argument:
 * per tesla in SI) and dL/dalpha into grad_dev, a DEVICE double[4] =
 * {dh_e[0], dh_e[1], dh_e[2], dalpha}.  The step is recomputed internally from
 * m_n.  Asynchronous.  Source terms carry no gradient and are not accepted. */
int sgspm_adjoint_step(sgspm_plan_t plan, const void* m_n, double alpha, const double h_e[3],
                       void* lam, double* grad_dev);

/* The adjoint step split at its tape, so that a backward pass that replays a
 * segment of steps does not run each step a second time (the chain rule of the
 * step above; the paper has none).
 *   sgspm_tape_bytes: *bytes = the device bytes of one step's tape (18 fields of
 *     N values in the plan's precision: the step's intermediate fields and its
 *     new state).
 *   sgspm_step_taped: one SGSPM step in place, exactly as sgspm_step (same
 *     result, bit for bit), that also writes its tape into `tape` (device, owned
 *     by the caller, sgspm_tape_bytes long).
 *   sgspm_adjoint_step_taped: sgspm_adjoint_step (same lam and grad_dev
 *     results, bit for bit) from the tape that sgspm_step_taped wrote for the
 *     same m_n, alpha and h_e; the tape is only read.  A tape of other inputs
 *     gives a meaningless result; nothing checks it.
 * SGS scheme only (SGSPM_EUNSUPPORTED otherwise); single-run plans; no source
 * terms.  Asynchronous on the plan's stream. */
int sgspm_tape_bytes(sgspm_plan_t plan, size_t* bytes);
int sgspm_step_taped(sgspm_plan_t plan, void* m, double alpha, const double h_e[3], void* tape);
int sgspm_adjoint_step_taped(sgspm_plan_t plan, const void* m_n, double alpha, const double h_e[3],
                             const void* tape, void* lam, double* grad_dev);

/* For callers that cannot allocate device memory during the call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * adjoint step above with the same arguments, results and errors, whose 16
 * fields of adjoint workspace live in a static device array of 8 MiB instead of
 * memory the plan allocates on the first adjoint call.  It calls no allocating
 * routine.  Grids above 131072 cells (FP32) or 65536 cells (FP64) need more
 * than the array holds and are rejected with SGSPM_EUNSUPPORTED before any
 * launch.  Each GPU holds one copy of the array for the life of the process, and
 * every call on that GPU, from any plan or thread, uses it: calls that overlap
 * on one GPU (concurrent streams, several threads) race on it and must be
 * serialised by the caller.  Nothing in it needs clearing between calls: every
 * field is written before it is read. */
int sgspm_adjoint_step_noalloc(sgspm_plan_t plan, const void* m_n, double alpha, const double h_e[3],
                               void* lam, double* grad_dev);

/* Batched plans (params.batch = B >= 2): B independent runs of the same grid
 * and constants share every launch of a step, so small grids fill the GPU.  m is
 * device [3][B][nz][ny][nx] of the plan's precision (component-major: component c
 * of run b at m + (c B + b) nz ny nx); run b steps with alpha[b] and the applied
 * field h_e[3 b .. 3 b + 2] (host arrays).  The result of each run is bit for bit
 * the one a single-run plan computes from the same input.  Per-run values are
 * staged in a plan-owned device buffer before the launches, so calls on one plan
 * must not overlap.  The single-run entry points (sgspm_step, sgspm_steps,
 * sgspm_energy, sgspm_field, sgspm_stray, sgspm_heat_solve, the adjoint and the
 * spectral-radius step) return SGSPM_EINVAL on a batched plan; sgspm_unit_error
 * returns the maximum over every run. */
int sgspm_step_batch(sgspm_plan_t plan, void* m, const double* alpha, const double* h_e);
/* nsteps batched steps with constant per-run alpha and h_e, replayed from one
 * captured HIP graph of the batched step (captured again when m changes).  The
 * per-run values are read from the plan's device buffer at every replay. */
int sgspm_steps_batch(sgspm_plan_t plan, void* m, int nsteps, const double* alpha, const double* h_e);
/* Energies of every run (as sgspm_energy): e_out = host double[5 B], run b at
 * e_out[5 b]; h_e = host double[3 B].  Synchronises the stream. */
int sgspm_energy_batch(sgspm_plan_t plan, const void* m, const double* h_e, double* e_out);

/* Measurement support.  Kernel classes of the step's launches; each class is
 * one kernel (its float or double instance): */
enum {
  SGSPM_KC_ROW_FWD = 0,     /* k_row_fwd: x rows: [c2r] -> right-hand side -> [DCT-II] / [r2c] */
  SGSPM_KC_ROW_FWD512 = 1,  /* k_row_fwd512: the same for rows of 256, 512-point register FFTs */
  SGSPM_KC_ROW_INV = 2,     /* k_row_inv: x rows: inverse DCT -> Gauss-Seidel update or projection -> [r2c] */
  SGSPM_KC_ROW_INV512 = 3,  /* k_row_inv512: the same for rows of 256, 512-point register FFTs */
  SGSPM_KC_COL_DCT = 4,     /* k_col_dct: y / z pencil DCT passes (grids without the fused solve) */
  SGSPM_KC_YZ_SOLVE = 5,    /* k_yz_solve: y and z DCTs and the diagonal solve of x-major planes */
  SGSPM_KC_YZ_REG = 6,      /* k_yz_reg: the same for 256 x 32 planes, z pass in registers */
  SGSPM_KC_COL_FFT = 7,     /* k_col_fft: y pencils, padded FFT / cropped inverse FFT (any length) */
  SGSPM_KC_FFT512 = 8,      /* k_fft512: the same for length 512, in registers */
  SGSPM_KC_CONV = 9,        /* k_conv: last-axis FFT, demagnetising-tensor multiply, inverse FFT */
  SGSPM_KC_CONV64 = 10,     /* k_conv64: the same for a padded last axis of 64, in registers */
  SGSPM_KC_OTHER = 11,      /* point-wise passes, reductions, energies */
  SGSPM_KC_COUNT = 12
};

/* Enable (1) or disable (0) timing of every later launch with HIP events on
 * the plan's stream; clears what was recorded.  Timing adds two event records
 * per launch. */
int sgspm_timing(sgspm_plan_t plan, int enable);

/* Synchronise and return, per kernel class since the last enable/read: total
 * kernel milliseconds, total launch-level bytes (each input array read once and
 * each output written once per launch) and the number of launches (host
 * arrays of SGSPM_KC_COUNT entries).  Clears the records. */
int sgspm_timing_read(sgspm_plan_t plan, double ms[SGSPM_KC_COUNT], double bytes[SGSPM_KC_COUNT],
                      int64_t launches[SGSPM_KC_COUNT]);

/* Synchronise the stream and report (then clear) the projection flag:
 * SGSPM_ENUMERIC if any projection since the last check met a zero or
 * non-finite |m***|. */
int sgspm_check(sgspm_plan_t plan);

/* Free the plan's device memory (synchronises its stream first). */
int sgspm_destroy(sgspm_plan_t plan);

/* Thread-local message for the last failure on this thread ("" if none). */
const char* sgspm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SGSPM_H */

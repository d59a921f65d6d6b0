/*
 * lbm_lee.h -- C ABI of the MI355X (gfx950) lattice Boltzmann solver for the Linearized
 * Euler Equations without background velocity (Otte & Frank, "Derivation and Analysis of
 * Lattice Boltzmann Schemes for the Linearized Euler Equations").
 *
 * The library computes the fully discrete LBE update (Section "Derivation of the Lattice
 * Boltzmann Equation"):
 *     g_i(t+1, x + c_i) = (1 - 1/tau) g_i(t, x) + (1/tau) g_i^eq(t, x),
 * with the equilibrium of the polyatomic ansatz (Section "Generalization of the Finite
 * Discrete Velocity Ansatz for Polyatomic Gases"; the monoatomic one of Section
 * "Derivation of Finite Discrete Velocity Models for Monoatomic Gases" is its special case)
 *     g_i^eq = f*_i (a1 rho' + a2 theta' + b c_i.u' + |c_i|^2/2 (c1 rho' + c2 theta')),
 * and the moments rho' = sum g, u' = sum c g / rho0,
 *     theta' = ((gamma - 1) sum (|c|^2 + beta)/2 g - theta0 rho') / rho0,
 * on a periodic box, everything in lattice units (dx = dt = 1).  The second-order scheme is
 * tau = 1/2 (Section "Analysis of the LBE").
 *
 * Conventions shared by every entry point
 *   - Memory: the caller allocates and owns every device buffer (populations, initial
 *     fields, outputs, scratch).  The library never allocates or frees device memory; a
 *     handle keeps non-owning pointers and a small host-side table, nothing else.
 *   - Streams: `stream` is a hipStream_t (NULL = the legacy default stream).  Every call
 *     only enqueues work on it, except those documented as synchronising.
 *   - Layout: populations are structure-of-arrays, g[i * N + cell] with
 *     cell = x + nx * (y + ny * z), N = nx * ny * nz, x fastest.  Macroscopic fields are
 *     N-element arrays in the same cell order; a velocity field is D such arrays back to
 *     back (u[a * N + cell]).  Unused dimensions have extent 1.
 *   - Errors: no C++ exception crosses this boundary.  Each call returns an lbm_status;
 *     lbm_lee_last_error() gives a message for the calling thread.  HIP errors are
 *     reported as LBM_E_HIP with the HIP error string in the message.
 */
#ifndef LBM_LEE_H
#define LBM_LEE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;
#define LBM_OK 0
#define LBM_E_INVALID (-1)     /* bad argument: size, alignment, null pointer, tau < 1/2 ... */
#define LBM_E_UNSUPPORTED (-2) /* valid but not implemented combination                     */
#define LBM_E_HIP (-3)         /* a HIP runtime call failed                                  */
#define LBM_E_STATE (-4)       /* call not allowed in the handle's current state             */

/* Velocity sets (Section "Examples of Velocity Sets").  D2Q9 is not in the paper: its
 * weights solve the paper's similarity conditions at theta0 = 1/3 (4/9, 1/9, 1/36). */
#define LBM_D1Q3 0     /* rho0 = 1, theta0 = 1/3                                   */
#define LBM_D2Q5 1     /* rho0 = 1, theta0 = 1/4                                   */
#define LBM_D2Q9 2     /* rho0 = 1, theta0 = 1/3 (derived)                         */
#define LBM_D3Q7 3     /* 3D family, theta0 = 1/5, alpha = 0                       */
#define LBM_D3Q9 4     /* 3D family, theta0 = 3/5, alpha = 3/40                    */
#define LBM_D3Q13 5    /* 3D family, theta0 = 2/5, alpha = 0                       */
#define LBM_D3Q19 6    /* 3D family, theta0 = 3/10, alpha = 0                      */
#define LBM_D2Q5_DIA 7 /* diatomic, rho0 = 20/3, theta0 = 3/10, gamma = 5/3        */
#define LBM_D3Q7_DIA 8 /* diatomic, f1 = 5/42 (rho0 = 1), theta0 = 5/21, gamma = 7/5 */
#define LBM_D3Q27 9    /* 3D family, theta0 = 1/3, alpha = 1/216: all 27 weights positive */
                       /* (8/27, 2/27, 1/54, 1/216); one-step variants only, no LBM_BC_MLP */
#define LBM_NUM_LATTICES 10

/* Population storage.  F64 and F32 store g itself.  F16 and BF16 store the normalised
 * deviation h_i = S g_i / f*_i (S a power of two, see lbm_lee_desc.store_scale) rounded to
 * nearest-even, and compute the collision in FP32.  I16 stores the same h as a signed 16-bit
 * fixed-point integer (round to nearest-even, saturating at +-32767), FP32 collision. */
#define LBM_F64 0
#define LBM_F32 1
#define LBM_F16 2
#define LBM_BF16 3
#define LBM_I16 4
#define LBM_E3M12 5 /* h as a 16-bit float with 3 exponent and 12 mantissa bits (see below)  */
/* E3M12 (not an IEEE format): sign, 3-bit exponent e, 12-bit mantissa m; value
 * (1 + m/4096) 2^(e-7) for e >= 1 and m 2^-18 for e = 0; round to nearest even; saturating at
 * 2 - 2^-12.  Same 2 bytes as FP16, 4x finer spacing over the 8 binades below 2. */

/* Performance knobs of the DPP step kernel (lbm_lee_desc.tune); results do not depend on them. */
#define LBM_TUNE_NT_STORE 1  /* non-temporal (streaming) stores                        */
#define LBM_TUNE_NT_LOAD 2   /* non-temporal (streaming) loads                         */
#define LBM_TUNE_PERSISTENT 4 /* grid sized to the resident wave slots, grid-stride loop */
#define LBM_TUNE_FULL_REST 8  /* also load, collide and store the rest population where it is */
                              /* provably invariant (see lbm_lee_bytes_per_update)            */
#define LBM_TUNE_CLOSURE_STREAM 16 /* LBM_BC_MLP: run the network on the handle's helper stream,  */
                                   /* forked from and joined to the caller's stream each step, so */
                                   /* it overlaps the bulk step (eager launches add two event     */
                                   /* calls per step); no effect with LBM_VARIANT_OPEN2D (one     */
                                   /* launch per step).  In 3D the DPP bulk step then leaves the  */
                                   /* x faces to the boundary pass (it would read this step's     */
                                   /* predictions), which costs more than the overlap gains       */
                                   /* (D3Q7 384^3 FP16: 0.49 against 0.39 ms per step)            */
#define LBM_TUNE_IN_PLACE 32  /* one population buffer instead of two (periodic box only; pop_b */
                              /* of lbm_lee_init may be NULL); see "In-place streaming" below   */
/* LBM_VARIANT_TB2: segment length along the march axis (z in 3D, y in 2D).  Without these bits
 * it is chosen per launch: the length in [4, 64] that minimises (rounds of resident blocks) x
 * (planes per block), from the kernel's occupancy on the device. */
#define LBM_TUNE_TB_SEGMENT_8 64
#define LBM_TUNE_TB_SEGMENT_16 128
#define LBM_TUNE_TB_SEGMENT_32 192
/* LBM_BC_MLP in 1D and 3D: the closure network's kernel runs as one block of four waves that walk
 * every tile of face nodes (the grid-stride loop the kernel takes once the face nodes outnumber
 * 64 per resident block slot of the GPU, exercised on small boxes; slow, for tests).  Same results
 * as without it. */
#define LBM_TUNE_NET_ONE_BLOCK 256

/* Boundary of the box.  The paper's scheme is periodic; the open closures are not in the
 * paper (it leaves boundary conditions to future work) and are defined here.  For a cell x
 * whose population i streams from s = x - c_i outside the box:
 *   ZERO    the streamed value is 0 (the exterior is at rest);
 *   COPY    the value at clamp(s), the nearest cell of the box (zero normal gradient);
 *   SPONGE  as ZERO, and after the collision the state is damped by
 *           1 - sponge_sigma ((W - d) / W)^2 at distance d < W = sponge_width from the faces;
 *   MLP     a learned prediction (lbm_lee_set_closure) for the face node clamp(s); for a source
 *           beyond an edge or corner, the mean of the predictions of every face it lies beyond.
 *           Each face prediction at node p is limited in weighted energy (sum g^2 / f*) to
 *           E_out / (2^n - 1), E_out the energy of p's populations leaving through that face and
 *           n the number of faces p lies on (scaled down, direction kept), so the energy that
 *           enters at p never exceeds the energy that leaves it: at tau = 1/2 the open box's
 *           weighted energy cannot grow, whatever the network predicts.  With sponge_width
 *           W >= 1 the network closes a box whose outer W cells form a sponge layer: after the
 *           collision the state is damped there as SPONGE damps it (W = 0: no layer). */
#define LBM_BC_PERIODIC 0
#define LBM_BC_ZERO 1
#define LBM_BC_COPY 2
#define LBM_BC_SPONGE 3
#define LBM_BC_MLP 4

/* Step kernel variant.  All variants run the same per-cell arithmetic, so their results are
 * bitwise identical; they differ only in how the streamed values are gathered (the multi-step
 * variants TB2/TB3 with 16-bit storage excepted: they round once per launch, see below). */
#define LBM_VARIANT_AUTO 0    /* the fastest measured variant: RESIDENT on periodic boxes     */
                              /* whose state fits it; OPEN2D on 2D open boxes of              */
                              /* <= 2^23 cells (GENERIC on larger ones); on                    */
                              /* periodic 2D/3D boxes of >= 2^20 cells TB3 (sets of <= 9       */
                              /* velocities) or TB2 (4- and 8-byte storage) where supported;  */
                              /* TB2 on periodic 2D boxes of 2^18 to 2^20 cells, TB3 on         */
                              /* periodic 3D boxes of 3 x 2^18 to 2^20 cells (sets of <= 9      */
                              /* velocities, nx even); DPP/DPP2/GENERIC (by nx: nx % 4, nx % 2, */
                              /* odd) on 3D open boxes (but not D3Q27 with 8-byte storage) and  */
                              /* for 2-byte storage on boxes of >= 2^20 cells; else GENERIC     */
#define LBM_VARIANT_GENERIC 1 /* one thread per cell, per-element wrapped gathers            */
#define LBM_VARIANT_DPP 2     /* 4 cells per lane, aligned vector loads, x shift by DPP;   */
                              /* needs nx % 4 == 0                                          */
#define LBM_VARIANT_LDS 3     /* one thread per cell, x-shifted rows staged in LDS + halo   */
#define LBM_VARIANT_DPP2 4    /* 2 cells per lane, as DPP; needs nx % 2 == 0                 */
/* Two steps per launch (temporal blocking), periodic 2D boxes of any extents and 3D boxes with
 * even nx: a block owns a tile of 64 cells along x (and TY along y in 3D) and marches along the
 * last axis, doing step t+1 on the tile and a one-cell ring around it (state t read from HBM) and
 * then step t+2 on the tile (state t+1 from LDS and registers), so the state crosses HBM once per
 * two steps.  In 3D each thread reads and writes two x-adjacent cells per access (hence even nx).
 * The intermediate state is never stored: with F64/F32 storage the result equals two one-step
 * launches bit for bit; with the 16-bit formats it stays in FP32 and a launch rounds to the
 * format once instead of twice (half the rounding error of the one-step kernels, whose error at
 * tau = 1/2 accumulates undamped).  An odd step count ends with one one-step launch.
 * LBM_E_UNSUPPORTED for open boxes, 1D sets, 3D boxes with odd nx, and sets whose in-plane LDS
 * rings do not fit 64 KB at TY = 4 (D3Q19 and D3Q27, and D3Q9 and D3Q13 with FP64). */
#define LBM_VARIANT_TB2 5
/* Three steps per launch, the same scheme one stage deeper (the tile dilated by two cells for
 * step t+1, by one for t+2); LDS rings of two intermediate steps (up to 160 KB per block).  In 3D
 * the tile is 128 x 16 cells where those rings fit with 4-byte ring elements (FP32 storage and
 * the 16-bit formats, whose intermediate steps are kept in FP32; D3Q7), else 64 x TY.  As
 * with TB2, F64/F32 results equal one-step launches bit for bit and the 16-bit formats round
 * once per launch of three steps.
 * LBM_E_UNSUPPORTED where they do not fit at TY = 4 (D3Q13 and D3Q19 with FP64) and in the
 * cases TB2 refuses.  A remainder of the step count (mod 3) runs one-step launches. */
#define LBM_VARIANT_TB3 6
/* 2D open boxes (every boundary but LBM_BC_PERIODIC): one launch per step.  Blocks of the ring
 * (the cells on a face) and blocks of the interior run side by side; with LBM_BC_MLP each wave
 * of the ring evaluates the closure network for the face nodes its ring cells pull from and
 * keeps the predictions in LDS; with LBM_BC_SPONGE each cell of the layer is damped by the
 * thread that stores it.  Same values, ghost buffer and history as the separate network, bulk,
 * boundary and sponge kernels of the other variants; LBM_TUNE_CLOSURE_STREAM has no effect.
 * LBM_E_UNSUPPORTED for periodic boxes and for 1D and 3D lattices. */
#define LBM_VARIANT_OPEN2D 7
/* Every step of one call in a single launch, the whole state held in LDS: periodic boxes whose
 * two copies of the state fit 160 KiB (2 Q N bytes-per-value <= 163840; the paper's 1D runs,
 * small 2D/3D grids), where one launch per step is what bounds the one-step variants.  Same
 * values as GENERIC.  LBM_E_UNSUPPORTED for open boxes and larger states. */
#define LBM_VARIANT_RESIDENT 8

typedef struct lbm_lee_desc {
    int32_t lattice;     /* LBM_D1Q3 ...                                                    */
    int32_t storage;     /* LBM_F64 ...                                                     */
    int64_t n[3];        /* nx, ny, nz >= 1; n[a] must be 1 for a >= D                      */
    double tau;          /* relaxation time, >= 1/2 (1/2 is the second-order scheme)        */
    int32_t variant;     /* LBM_VARIANT_*                                                   */
    int32_t tune;        /* LBM_TUNE_* bits, 0 for the defaults                             */
    double store_scale;  /* S for 16-bit storage: 0 = choose from the initial state so that  */
                         /* max |S g / f*| lies in [1/2, 1) (F16/BF16/E3M12) or [2^13, 2^14)*/
                         /* (I16); otherwise a power of two > 0.  Ignored for F64/F32.     */
    int32_t bc;          /* LBM_BC_*; open boxes need n[a] >= 3 on every axis a < D         */
    int32_t sponge_width;/* LBM_BC_SPONGE: layer width W >= 1 in cells; LBM_BC_MLP: W >= 0  */
                         /* (a sponge layer behind the network, 0 = none); else ignored     */
    double sponge_sigma; /* sigma_max in [0, 1] when there is a sponge layer                */
} lbm_lee_desc;

typedef struct lbm_lattice_info {
    int32_t D, Q;
    int32_t c[27][3];    /* velocities, canonical order: rest, -x,+x,-y,+y,-z,+z, edges, corners */
    double fstar[27];    /* weights f*_i                                                     */
    double beta[27];     /* extra energies beta_i (0 for monoatomic sets)                    */
    double rho0, theta0, gamma, a1, a2, b, c1, c2;
    char name[16];
} lbm_lattice_info;

typedef struct lbm_lee *lbm_lee_handle;

/* Tables of a velocity set as used by the kernels (host only, no GPU work). */
lbm_status lbm_lee_lattice_info(int32_t lattice, lbm_lattice_info *out);

/* Units of a dimensional problem run on a velocity set (Section "The Linearized Euler
 * Equations", non-dimensionalisation): dimensional quantities (underlined in the paper) are the
 * non-dimensional ones times these scales:
 *     rho_dim = rho_star rho (background and fluctuation), theta_dim = theta_star theta,
 *     u_dim = u_star u with u_star^2 = theta_star, x_dim = x_star x, t_dim = t_star t,
 *     t_star = x_star / u_star.
 * Because the non-dimensional LEE keep the same form, a set with background (rho0, theta0) runs any
 * dimensional background (rho0_dim, theta0_dim): rho_star = rho0_dim / rho0, theta_star =
 * theta0_dim / theta0.  The library's lattice units are these non-dimensional units with
 * dx = dt = 1; a grid of spacing dx (non-dimensional) maps cell j to x = j dx and step n to
 * t = n dx. */
typedef struct lbm_lee_scaling {
    double rho_star, theta_star, u_star, x_star, t_star;
} lbm_lee_scaling;

/* Scales for a dimensional background rho0_dim, theta0_dim (both > 0) and length unit x_star > 0
 * on `lattice` (host only, no GPU work).  Errors: LBM_E_INVALID for an unknown lattice, a NULL out
 * or a non-positive or non-finite argument. */
lbm_status lbm_lee_dimensional_scaling(int32_t lattice, double rho0_dim, double theta0_dim, double x_star,
                                       lbm_lee_scaling *out);

/* Time steps for a dimensional end time t_dim >= 0 with non-dimensional step dt = dx > 0 (host
 * only): T = t_dim / t_star, *nsteps = round(T / dt) (half away from zero), *t_end = nsteps dt,
 * the end time the run reaches, and *offset = T - nsteps dt, the mismatch Table 1 of Section
 * "Numerical Results" lists for the 3D diatomic runs.  Any output may be NULL.  Errors:
 * LBM_E_INVALID for a NULL or invalid scaling, a negative or non-finite time, dt <= 0 or a step
 * count beyond 2^62. */
lbm_status lbm_lee_dimensional_steps(const lbm_lee_scaling *s, double t_dim, double dt, int64_t *nsteps,
                                     double *t_end, double *offset);

/* Bytes of one population buffer: Q * N * sizeof(storage element).  0 on a bad desc. */
size_t lbm_lee_state_bytes(const lbm_lee_desc *desc);

/* Bytes of device scratch lbm_lee_init needs (reductions, scale search).  0 on a bad desc. */
size_t lbm_lee_scratch_bytes(const lbm_lee_desc *desc);

/* The collision constants of the step kernels, in FP64 before they are rounded to the compute
 * type (host only, no GPU work).  The paper's update (Section "Derivation of the Lattice Boltzmann
 * Equation": moments, equilibrium of Section "Derivation of Finite Discrete Velocity Models for
 * Monoatomic Gases" / "Generalization of the Finite Discrete Velocity Ansatz for Polyatomic
 * Gases", relaxation with tau) is linear in the per-shell sums S_sh = sum s_i and J_sh =
 * sum c_i s_i of the stored values (shell sh = |c|^2 in 0..3); a population of shell `to` becomes
 *   keep s + sum_from H[to*4 + from] S_from + c . sum_from WB[to*4 + from] J_from.
 * Storage units: F64/F32 store g itself; the 16-bit formats store S g/f* with S =
 * desc->store_scale (1 if 0: the automatic choice is made at lbm_lee_init).  Entries of shells the
 * set lacks are meaningless.  Errors: LBM_E_INVALID for NULL outputs or a bad desc. */
lbm_status lbm_lee_collision_constants(const lbm_lee_desc *desc, double H[16], double WB[16], double *keep);

/* Algorithmic HBM bytes per lattice-cell update of the step kernel: Q loads and Q stores of
 * the storage element (2 Q s), or 2 (Q - 1) s when the rest population is left out of the step.
 * It is left out when the equilibrium map leaves it invariant (E_00 = 1, E_0j = E_j0 = 0:
 * D1Q3, D2Q5, D3Q7, D3Q9, D3Q13 and the diatomic D2Q5/D3Q7 sets), the boundary is not
 * LBM_BC_SPONGE and LBM_TUNE_FULL_REST is not set; both buffers then hold the same (constant)
 * rest population.  0 on a bad desc. */
double lbm_lee_bytes_per_update(const lbm_lee_desc *desc);

/*
 * Create a solver on caller-owned buffers and set the initial state to equilibrium of the
 * given macroscopic fields (Section "Analysis of the LBE": g_i(0, x) = g_i^eq(rho', u', theta')).
 *   pop_a, pop_b  device buffers of bytes_each >= lbm_lee_state_bytes(desc), 256-byte aligned;
 *                 the state ping-pongs between them (with LBM_TUNE_IN_PLACE only pop_a is used
 *                 and pop_b may be NULL).
 *   rho, theta    device FP64 arrays of N values; u: device FP64, D * N values.  All three
 *                 NULL: the state at rest (zero fields; the 16-bit storage scale is then
 *                 desc->store_scale, or 1 when that is 0).
 *   scratch       device buffer of scratch_bytes >= lbm_lee_scratch_bytes(desc), 256-byte aligned.
 * Synchronises `stream` only when desc->store_scale == 0 with 16-bit storage (it reads back
 * the maximum of |g / f*| to choose S).  On failure *out is NULL and nothing is enqueued.
 */
lbm_status lbm_lee_init(const lbm_lee_desc *desc, void *pop_a, void *pop_b, size_t bytes_each,
                        const double *rho, const double *u, const double *theta,
                        void *scratch, size_t scratch_bytes, void *stream, lbm_lee_handle *out);

/* Re-initialise an existing handle from new macroscopic fields (same rules as lbm_lee_init,
 * the storage scale is kept).  Resets the step counter. */
lbm_status lbm_lee_reinit(lbm_lee_handle h, const double *rho, const double *u, const double *theta, void *stream);

/* Re-initialise to the equilibrium of fields given on a sub-box only (n_sub cells at cell
 * offset origin; rho, theta: n_sub cells, u: D * n_sub, same layout rules), with the fields zero
 * (the state at rest) on every other cell.  Lets a large box (e.g. the wider periodic run that
 * judges an open box) start from a small initial state without full-size field arrays.
 * Like lbm_lee_reinit it keeps the handle's storage scale: for the 16-bit formats create the
 * handle with desc.store_scale set when its first fields are at rest (the automatic choice
 * then has no amplitude to go by and takes 1).  Errors: LBM_E_INVALID for a NULL pointer or a
 * sub-box not inside the box. */
lbm_status lbm_lee_reinit_region(lbm_lee_handle h, const int64_t origin[3], const int64_t n_sub[3], const double *rho,
                                 const double *u, const double *theta, void *stream);

/* Advance nsteps >= 0 time steps (Section "Derivation of the Lattice Boltzmann Equation", the
 * fully discrete update: fused pull-stream + moments + equilibrium + relaxation), enqueued on
 * `stream`.  One-step variants launch one kernel per step (plus, on open boxes, the boundary
 * kernels of LBM_BC_*); TB2/TB3 launch one kernel per two/three steps and one-step kernels for a
 * remainder of nsteps.  With F64/F32 storage every kernel gives the same bits, so the result does
 * not depend on how the steps are split over calls; with the 16-bit formats a multi-step launch
 * rounds the state once per launch, so it does (each split is a valid run of the scheme with
 * one rounding per stored state).  The step counter advances by nsteps.  Errors:
 * LBM_E_INVALID for a NULL handle or nsteps < 0, LBM_E_STATE for an LBM_BC_MLP handle without
 * lbm_lee_set_closure, LBM_E_HIP if a launch fails. */
lbm_status lbm_lee_step(lbm_lee_handle h, int64_t nsteps, void *stream);

/*
 * Macroscopic fields of the current state (moments of the monoatomic / polyatomic FDVM
 * sections; p' = rho0 theta' + theta0 rho' from Section "The Linearized Euler Equations").
 * Sums are taken in FP64.  Any output may be NULL.  out_is_f64 != 0: outputs are double,
 * else float.  p, rho, theta: N values; u: D * N values.
 */
lbm_status lbm_lee_moments(lbm_lee_handle h, void *p, void *u, void *rho, void *theta, int32_t out_is_f64,
                           void *stream);

/* lbm_lee_moments restricted to a sub-box (n_sub cells at cell offset origin); the outputs are
 * sub-box arrays (n_sub cells, u: D of them). */
lbm_status lbm_lee_moments_region(lbm_lee_handle h, const int64_t origin[3], const int64_t n_sub[3], void *p, void *u,
                                  void *rho, void *theta, int32_t out_is_f64, void *stream);

/*
 * out[0] = sum_x sum_i g_i^2 / f*_i  (the weighted L2 energy; constant at tau = 1/2 for every
 *          set, non-increasing for tau > 1/2: stability structure of the D3Q19 section),
 * out[1] = sum_x sum_i g_i^2         (the von Neumann L2 norm squared of Section "Analysis of
 *          the LBE"; constant when Gamma(k) is unitary).
 * FP64 accumulation, deterministic two-pass reduction.  SYNCHRONISES the stream.
 */
lbm_status lbm_lee_l2_energy(lbm_lee_handle h, double out[2], void *stream);

/*
 * Error of the current state against reference fields (device FP64, N and D * N values;
 * ref_u may be NULL):  out = { sum (p'-p_ref)^2, sum p_ref^2, max |p'-p_ref|,
 *                              sum |u'-u_ref|^2, sum |u_ref|^2, max_a,x |u'_a-u_ref,a| }.
 * Multiply sums by dx^D for the discrete L2 norm of Section "Numerical Results".
 * SYNCHRONISES the stream.
 */
lbm_status lbm_lee_error_norms(lbm_lee_handle h, const double *ref_p, const double *ref_u, double out[6],
                               void *stream);

/* Decode the current populations into FP64 g (device, Q * N doubles, the layout above). */
lbm_status lbm_lee_export_f64(lbm_lee_handle h, double *g, void *stream);

/* Encode FP64 populations g (device, Q * N doubles) into the current state (checkpoint
 * restore, arbitrary non-equilibrium states).  steps_done is stored as the step counter. */
lbm_status lbm_lee_import_f64(lbm_lee_handle h, const double *g, int64_t steps_done, void *stream);

/*
 * In-place streaming (LBM_TUNE_IN_PLACE): the single buffer holds the post-collision state g*(t)
 * in one of two layouts that alternate step by step, starting (after init, reinit or import)
 * with "swapped": g*_i(x) in slot opposite(i) of cell x (opposite(i): the population with
 * velocity -c_i); after an odd number of steps since then "pushed": g*_i(x) in slot i of cell
 * x + c_i (periodic wrap).  Every step reads and writes, per cell, one fixed set of locations,
 * so no second buffer is needed; moments, norms, export and import translate the layout, and
 * the results are bitwise those of the two-buffer step.  Halves the state's memory (e.g. the
 * 1384^3 D3Q7 FP32 judge of the open-box workload: 74 GB instead of 148 GB).
 */

/* Device pointer of the buffer holding the current state, and the steps taken so far. */
lbm_status lbm_lee_current(lbm_lee_handle h, void **pop, int64_t *steps_done);

/* The storage scale S in use (1 for F64/F32). */
double lbm_lee_store_scale(lbm_lee_handle h);

/* The step-kernel variant the handle runs (LBM_VARIANT_*, never AUTO); -1 for NULL. */
int32_t lbm_lee_resolved_variant(lbm_lee_handle h);

/* Free the handle (host memory only; device buffers stay with the caller). NULL is a no-op. */
void lbm_lee_destroy(lbm_lee_handle h);

/* Bytes of the caller-owned ghost buffer an LBM_BC_MLP handle needs: per face node one FP32
 * value per entering population, then two history strips (3 Q FP32 values each, written and
 * read on alternate steps).  0 for other boundaries or a bad desc. */
size_t lbm_lee_ghost_bytes(const lbm_lee_desc *desc);

/* Attach the closure network (device FP32 parameters, layout of lbm_nrbc_dims) and the ghost
 * buffer to an LBM_BC_MLP handle.  The library keeps the pointers; the caller keeps both
 * buffers alive and may update the parameters between steps.  Steps fail with LBM_E_STATE
 * until this has been called.  The first call creates, on the current device (which must be
 * the handle's), a helper stream and two events; with LBM_TUNE_CLOSURE_STREAM each step forks
 * the network onto that stream so it runs beside the bulk step kernel, and joins it back before
 * the boundary recompute.  lbm_lee_destroy releases them.  Errors: LBM_E_HIP if they cannot be
 * created. */
lbm_status lbm_lee_set_closure(lbm_lee_handle h, const float *params, void *ghost, size_t ghost_bytes);

/*
 * Learned non-reflecting closure network (not in the paper).  Input: the strips of
 * post-collision populations at a face node, 3 cells deep along the inward normal, in the
 * canonical face frame (outward normal -x), of the current step and of the step before:
 * x[h * 3Q + m * Q + j], h = 0 now, h = 1 one step earlier (n_in = 6 Q); output: the populations
 * entering through the face (canonical c_x = +1, in canonical order).  In a step of an
 * LBM_BC_MLP box the earlier strip comes from the history the previous step stored in the ghost
 * buffer; on the first step after the state was set (init, reinit, import) or the closure
 * attached, the current strip stands in for it.  Network:
 *   s = rms(x), z = x / s, h1 = relu(z W1 + b1), h2 = relu(h1 W2 + b2), y = h2 W3 + b3, out = s y,
 * with rms computed as m sqrt(mean((x/m)^2)), m = max |x|; an all-zero strip predicts 0.
 * FP32 parameters, row-major, concatenated: W1[n_in][64], b1[64], W2[64][64], b2[64],
 * W3[64][n_out], b3[n_out].  Every product runs on matrix cores with bfloat16 inputs (round to
 * nearest even) and FP32 accumulation.
 */
/* dims = { n_in = 6 Q, n_out, hidden = 64, n_params }. */
lbm_status lbm_nrbc_dims(int32_t lattice, int32_t dims[4]);

/* Number of face nodes of a box (the id range of lbm_nrbc_gather): faces in the order
 * (x low, x high, y low, y high, z low, z high), nodes over the two in-face axes (ascending,
 * the lower axis fastest).  -1 on a bad desc. */
int64_t lbm_nrbc_face_nodes(const lbm_lee_desc *box);

/* Inference on `count` strips (device FP32 [count][n_in]) -> out (device FP32 [count][n_out]). */
lbm_status lbm_nrbc_forward(int32_t lattice, const float *params, const float *strips, int64_t count, float *out,
                            void *stream);

/* Workspace bytes of lbm_nrbc_loss_grad for a batch of `count` samples. */
size_t lbm_nrbc_workspace_bytes(int32_t lattice, int64_t count);

/*
 * Mean squared error of the network on a batch, in normalised units:
 *   loss = mean over samples with s > 0 and over outputs of (y - target / s)^2,
 * and its gradient with respect to every parameter (device FP32, n_params values).
 * `loss` (device, one float) may be NULL.  Deterministic (fixed reduction order).
 */
lbm_status lbm_nrbc_loss_grad(int32_t lattice, const float *params, const float *strips, const float *targets,
                              int64_t count, float *grad, float *loss, void *workspace, size_t workspace_bytes,
                              void *stream);

/* One Adam step (Kingma & Ba) on n FP32 parameters: m, v are the moment buffers, t >= 1. */
lbm_status lbm_nrbc_adam(int64_t n, float *params, const float *grad, float *m, float *v, int64_t t, float lr,
                         float beta1, float beta2, float eps, void *stream);

/*
 * Training pairs from a larger (e.g. periodic, three times wider) run `outer` whose cell
 * origin + x corresponds to cell x of the box `inner` (origin >= 1 and origin + n + 1 <= outer n
 * on every axis): for each face node id of the inner box (device int64 ids), the strip of the
 * current state at the node (one time level, 3 Q values, written at strips + t * strip_stride
 * floats, strip_stride >= 3 Q) and the true entering populations, i.e. the outer state at the
 * node's outside neighbour (targets [count][n_out]), physical FP32 values.  A network input row
 * [strip(t), strip(t-1)] (n_in = 6 Q) takes two calls with strip_stride = n_in: one on the
 * state before the step (strips + 3 Q, targets NULL), one after it (strips, with targets).
 * targets may be NULL: strips only, and then origin >= 0, origin + n <= outer n suffice, so
 * `outer` may be the open box itself (origin 0, inner = its own desc): the strips its closure
 * sees, for training on the states the closed loop actually visits.  Ids outside
 * [0, lbm_nrbc_face_nodes(inner)) give zero rows.  Errors: LBM_E_INVALID for NULL arguments,
 * count < 0, strip_stride < 3 Q, differing lattices or a misplaced inner box.
 */
lbm_status lbm_nrbc_gather(lbm_lee_handle outer, const int64_t origin[3], const lbm_lee_desc *inner,
                           const int64_t *node_ids, int64_t count, float *strips, int64_t strip_stride, float *targets,
                           void *stream);

/*
 * Compare a field a of a box (n_a[3] cells, device FP64) with the field b of a larger box
 * (n_b[3]) at cell offset origin: out = { sum (a - b)^2, sum b^2, max |a - b| }.
 * scratch as for lbm_lee_init.  SYNCHRONISES the stream.
 */
lbm_status lbm_lee_compare_fields(const double *a, const int64_t n_a[3], const double *b, const int64_t n_b[3],
                                  const int64_t origin[3], double out[3], void *scratch, size_t scratch_bytes,
                                  void *stream);

/* lbm_lee_compare_fields without the scratch argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * no hipMalloc, hipFree or allocating library call.  Its reduction scratch is a file-scope device
 * array of 96 KiB that each GPU the library runs on holds until the process ends (its address is
 * looked up once per device, on the first call there).  The scratch need does not grow with the
 * boxes (a fixed grid of partial sums), so every box lbm_lee_compare_fields accepts fits; other
 * arguments and errors as there.  All calls on one GPU share the array: calls that overlap on one
 * GPU (concurrent streams or threads) race and must be serialised by the caller.
 * SYNCHRONISES the stream. */
lbm_status lbm_lee_compare_fields_static(const double *a, const int64_t n_a[3], const double *b,
                                         const int64_t n_b[3], const int64_t origin[3], double out[3], void *stream);

/* Plain device-to-device copy kernel (16-byte vectors): the reference point for bandwidth
 * and counter calibration.  bytes must be a multiple of 16, both pointers 16-byte aligned. */
lbm_status lbm_lee_device_copy(void *dst, const void *src, size_t bytes, void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *lbm_lee_last_error(void);

/* Library version string. */
const char *lbm_lee_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_LEE_H */

/*
 * esbgk.h - C ABI of the MI355X lattice ES-BGK library (libesbgk.so).
 *
 * The library advances the lattice ES-BGK model of Meng, Zhang,
 * Hadjiconstantinou, Radtke and Shan ("Lattice ellipsoidal statistical BGK
 * model for thermal non-equilibrium flows", arXiv 1209.6548) on one gfx950
 * GPU: one fused pull-stream + collide kernel per time step.
 *
 * Units are the paper's nondimensional ones (Sec. 2.2): lengths in L (the
 * reference length of Kn), velocities in sqrt(R T0), temperature in T0,
 * density in rho0, body force g = L g^ / (R T0). One cell is dx = 1/N_L,
 * one step is dt = dx / r (every population moves by its integer lattice
 * vector e_alpha; c_alpha = r e_alpha).
 *
 * Populations. The model's discrete distribution f_alpha (eq. lbgk) is kept
 * as the deviation h_alpha = f_alpha / w_alpha - 1 in FP64, FP32 or FP16, in
 * structure-of-arrays order [alpha][z][y][x] (x fastest). Population I/O at
 * this boundary is always FP64 h in that order. Velocity order: index 0 is
 * rest, 1..P the vectors whose first non-zero component is positive sorted by
 * |e|^2 then by descending tuple order, alpha + P holds -e_alpha
 * (esbgk_lattice_info returns the table). The stored state is the
 * post-collision population of the last step; the moments of a state are
 * those of the distribution it streams into (the current time level).
 *
 * Conventions.
 *  - Every call returns an int status: ESBGK_OK (0) or a negative code.
 *    Nothing throws or aborts across the ABI.
 *  - Arguments are validated on the host before anything is launched; an
 *    invalid call changes nothing and returns ESBGK_E_INVALID.
 *  - Device memory is owned by the caller: esbgk_workspace_bytes tells how
 *    much, esbgk_create binds it. The library never frees it. The handle owns
 *    only host memory and HIP graph objects.
 *  - All work is queued on the HIP stream given at creation. Calls that
 *    return data to host memory (read_moments, get_populations, get_state,
 *    reduce, last_reduction) synchronise that stream; the others are
 *    asynchronous.
 *  - A HIP failure makes the handle sticky: every later call returns the same
 *    code until esbgk_destroy. esbgk_last_error describes it.
 *  - A handle is not thread-safe. Handles on different streams are
 *    independent.
 */
#ifndef ESBGK_H
#define ESBGK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ESBGK_OK = 0,
  ESBGK_E_INVALID = -1,   /* argument out of range or inconsistent */
  ESBGK_E_NOMEM = -2,     /* workspace smaller than esbgk_workspace_bytes */
  ESBGK_E_HIP = -3,       /* a HIP runtime call failed (sticky) */
  ESBGK_E_NONFINITE = -4, /* a reduction met a non-finite value, rho <= 0 or T <= 0 (sticky) */
  ESBGK_E_UNSTABLE = -5,  /* Euler step with dt/tau or dt/(Pr tau) >= 2 at rho = T = 1 */
  ESBGK_E_STATE = -6      /* call out of order (e.g. step before the state is set) */
};

enum { ESBGK_D2Q37 = 1, ESBGK_D3Q39 = 2,             /* on-lattice velocity sets */
       ESBGK_D2Q36GH = 3,                            /* 6-point Gauss-Hermite product set (esbgk_tvd_*) */
       ESBGK_D2Q16GH = 4, ESBGK_D2Q64GH = 5,         /* 4- and 8-point product sets (esbgk_tvd_*) */
       ESBGK_D3Q216GH = 6 };                         /* 3-D cube of the 6-point rule (esbgk_tvd_*) */
enum { ESBGK_F64 = 0, ESBGK_F32 = 1, ESBGK_F16 = 2 };  /* storage of h; FP64 computes in FP64, the others in FP32 */
enum { ESBGK_TRAPEZOID = 0, ESBGK_EULER = 1 };         /* time discretisation of eq. lbgk */

typedef struct esbgk_ctx esbgk_ctx;
typedef struct esbgk_batch esbgk_batch;

/* Geometry and numerics of one lattice.
 *  velset  ESBGK_D2Q37 (2-D, Hermite order N = 4) or ESBGK_D3Q39 (3-D, N = 3)
 *  nx,ny,nz  cells per axis; nz must be 1 for D2Q37. nx*ny*nz < 2^31.
 *  walls   0: periodic in every axis. 1: diffuse walls (Sec. 3.2) half a cell
 *          outside the first and last layer of the last axis (y in 2-D, z in
 *          3-D); that axis needs at least 6 cells. Other axes are periodic.
 *  storage ESBGK_F64 / ESBGK_F32 / ESBGK_F16.
 *  scheme  ESBGK_TRAPEZOID (second order) or ESBGK_EULER (forward Euler along
 *          the characteristic, the paper's Sec. 3.1 update at Courant 1).
 *  n_ref   N_L, the number of cells across the reference length L of Kn;
 *          0 means the extent of the wall axis (walls = 1) or nx. */
typedef struct {
  int velset, nx, ny, nz, walls, storage, scheme, n_ref;
} esbgk_shape;

/* Velocity set of Sec. 2.2 (abscissae c = r e and weights of a Gauss-Hermite
 * quadrature, eq. weight for the 1-D case), derived on the host by matching
 * the moments of the Gaussian weight function. Any output pointer may be
 * NULL. e receives Q*D ints (row per velocity), w receives Q doubles. Touches
 * no GPU. */
int esbgk_lattice_info(int velset, int* Q, int* D, int* N, double* r, int* e, double* w);

/* Bytes of device workspace a lattice of this shape needs (0 if the shape is
 * invalid). The caller allocates it (e.g. torch.empty(n, dtype=uint8)),
 * 256-byte aligned. The populations live in it slice-blocked: for every
 * layer of the last axis, the Q velocity planes of that layer side by side;
 * a shape whose one layer of populations reaches 4 GiB is invalid. */
size_t esbgk_workspace_bytes(const esbgk_shape* shape);

/* Bind a workspace and a HIP stream (hipStream_t, NULL = default stream) to a
 * new handle. The workspace must stay allocated until esbgk_destroy.
 * Gas defaults: Kn = 0.1, Pr = 1, varpi = 0.5; walls at rest at T = 1; g = 0.
 * Errors: E_INVALID (shape), E_NOMEM (ws_bytes too small), E_HIP. */
int esbgk_create(const esbgk_shape* shape, void* d_workspace, size_t ws_bytes,
                 void* hip_stream, esbgk_ctx** out);

/* Release the handle (never the caller's workspace or stream). */
int esbgk_destroy(esbgk_ctx* ctx);

/* Gas parameters (Sec. 2.1-2.2): Kn = mu0 sqrt(R T0)/(p0 L); Pr = 1/(1-b)
 * with -1/2 <= b <= 1, i.e. Pr >= 2/3; viscosity law mu/mu0 = (T/T0)^varpi,
 * varpi in [0.5, 1]. tau = (Kn/Pr) mu / p per cell. Errors: E_INVALID,
 * E_UNSTABLE (Euler only). */
int esbgk_set_gas(esbgk_ctx* ctx, double Kn, double Pr, double varpi);

/* Diffuse wall state (Sec. 3.2, full accommodation): side 0 = low wall,
 * 1 = high wall; temperature T_w > 0 and velocity u_w[3] (its wall-normal
 * component must be 0). Populations leaving the wall are rho_W S(T_w, u_w),
 * eq. feq0 at the bulk order N, with rho_W from the flux balance of Sec. 3.2.
 * E_INVALID if the lattice has no walls. */
int esbgk_set_wall(esbgk_ctx* ctx, int side, double T_w, const double u_w[3]);

/* Maxwell's wall model (Sec. 3.2): accommodation 0 <= gamma <= 1 of wall
 * `side`, the fraction of the particles reaching it that is re-emitted
 * diffusely (as set by esbgk_set_wall); 1 - gamma is reflected specularly.
 * A population pulled from beyond the wall becomes gamma times the diffuse
 * ghost plus 1 - gamma times its specular image: the mirror velocity (wall-
 * normal component negated) leaving the mirrored layer of the same source
 * column. rho_W keeps its definition, so mass is conserved for every gamma.
 * Default 1 (the paper's full accommodation). E_INVALID if the lattice has no
 * walls or gamma is outside [0, 1]. */
int esbgk_set_wall_accommodation(esbgk_ctx* ctx, int side, double gamma);

/* Unsteady boundary heating (Sec. 4.2): the temperature of wall `side`
 * becomes T_W(t) = T_w + amplitude sin(theta t), T_w as set by
 * esbgk_set_wall, t in units of L / sqrt(R T0) (t = n dt after n steps;
 * theta is the paper's Strouhal number). The step from stored level n
 * re-emits at T_W((n + 1/2) dt), the midpoint of its streaming; the wall
 * tables are rebuilt on the device before every step (also inside the
 * captured graphs), and read-outs of level n use that step's tables.
 * amplitude = 0 restores the static wall. E_INVALID if the lattice has no
 * walls, an argument is not finite or |amplitude| >= T_w. */
int esbgk_set_wall_heating(esbgk_ctx* ctx, int side, double amplitude, double theta);

/* Body force g[3] (eq. esbgk, its Hermite expansion in Sec. 2.2). */
int esbgk_set_body_force(esbgk_ctx* ctx, const double g[3]);

/* Initial state f_alpha = rho S_alpha(T, u) (1 + amplitude * noise_alpha)
 * per cell, S of eq. feq0 at the bulk order N. rho, T: [cells] host FP64;
 * u: [D][cells]; noise: [Q][cells]. NULL fields mean rho = 1, u = 0, T = 1;
 * NULL noise means none. Resets the step counter. */
int esbgk_init_equilibrium(esbgk_ctx* ctx, const double* rho, const double* u,
                           const double* T, const double* noise, double amplitude);

/* Set / read the stored populations as FP64 h[Q][cells] (host memory).
 * set rounds to the storage type (round to nearest even). */
int esbgk_set_populations(esbgk_ctx* ctx, const double* h);
int esbgk_get_populations(esbgk_ctx* ctx, double* h);

/* Raw state for checkpoint / restart: the stored populations h in the
 * storage type as [Q][cells] (cells numbered x fastest, independent of the
 * device layout), then the step counter (int64); esbgk_state_bytes gives the
 * size. Restoring and stepping is bit-identical to never having saved. */
size_t esbgk_state_bytes(const esbgk_ctx* ctx);
int esbgk_get_state(esbgk_ctx* ctx, void* h_raw, size_t nbytes);
int esbgk_set_state(esbgk_ctx* ctx, const void* h_raw, size_t nbytes);

/* Advance n >= 0 time steps (asynchronous). Each step streams every
 * population along e_alpha (pull, periodic wrap, wall re-emission) and
 * collides: fbar* = fbar - omega (fbar - f_ES^N) + phi dt F, with f_ES^N the
 * Hermite projection of the anisotropic Gaussian (eq. approxfeq, lambda of
 * eq. cfeq) and F the force expansion of Sec. 2.2. Every R steps
 * (esbgk_set_reduce_interval) the step also forms the FP64 reductions. */
int esbgk_step(esbgk_ctx* ctx, int64_t n);

/* Runs of `steps` consecutive step launches (even, default 32) are captured
 * once per starting buffer in a HIP graph and replayed on the handle's
 * stream; 0 disables graphs (one launch per step). Steps that carry a fused
 * reduction are always launched directly. Results are identical either way.
 * Changing the length (and esbgk_set_wall_heating switching heating on or
 * off, and esbgk_destroy) first waits for the handle's stream, so that no
 * replay is queued or running when its graph is released. */
int esbgk_set_graph_steps(esbgk_ctx* ctx, int steps);

/* Pairs of steps in place, in one population buffer: the first step pulls
 * (as above) and pushes each post-collision population to the slot of the
 * opposite velocity at the cell it streams to, the only slot that no other
 * cell touches; the second step reads those slots at its own cell and
 * writes its populations back to their own slots, the layout the pair
 * started from. Each cell's arithmetic is that of the two-buffer step, so
 * the bits are the same; a run of pairs works on half the memory, which
 * can then stay in the GPU's 256 MB memory-side cache. mode = 1: pairs;
 * 0: always two buffers; 2 (default): pairs when the two buffers of one
 * lattice exceed 256 MB and one buffer does not exceed 384 MB (where they
 * were measured faster on MI355X). Pairs need a periodic lattice or fully
 * diffuse walls (gamma = 1: a specular image would need the populations
 * pushed across a wall). Of an odd step count, the first step uses two
 * buffers and the rest run in pairs. */
int esbgk_set_inplace(esbgk_ctx* ctx, int mode);
/* 1 if esbgk_step advances this handle in pairs (mode, walls and size as
 * above), 0 if in two buffers; E_INVALID for a null handle. */
int esbgk_inplace_active(const esbgk_ctx* ctx);

/* Macroscopic fields of eq. mac at the current level, FP64 [F][cells] host:
 * rho, u[D], T, sigma (trace-free, components xx,xy,yy or
 * xx,xy,xz,yy,yz,zz), q[D]. F = 9 (2-D) or 14 (3-D); *F receives it. */
int esbgk_read_moments(esbgk_ctx* ctx, double* h_out, int* F);

/* FP64 reductions of the current level (out[8]): total mass sum rho,
 * energy sum 1/2 sum_alpha f c^2, momentum sum rho u (3), mass flow rate
 * through a plane normal to x, dx^(D-1)/nx sum rho u_x, the relative change
 * ||u - u_prev||_2/||u||_2 since the previous reduction (0 for the first),
 * and the step count. Computed in a fixed order (deterministic). Returns
 * E_NONFINITE (sticky) if a cell has a non-finite value, rho <= 0 or
 * T <= 0. */
int esbgk_reduce(esbgk_ctx* ctx, double out[8]);

/* For callers that cannot allocate device memory: esbgk_reduce without the
 * handle's workspace scratch. The per-workgroup partials (at most 1024
 * workgroups, each folding every 1024th block of 256 cells in a fixed order)
 * and the 8 final sums live in a static device array of the library
 * (1024 * 8 + 8 doubles, about 64 KiB per GPU, held until the process ends;
 * its address is looked up once per GPU, with that GPU current). Every
 * lattice a handle accepts fits. Same results as esbgk_reduce up to the
 * order of the FP64 additions (the cells are grouped differently); it also
 * becomes the handle's latest reduction and u_prev, as esbgk_reduce does.
 * Calls no allocation routine. All calls on one GPU share the array:
 * calls that overlap in time on one GPU (other streams, other threads) race;
 * serialise them. Synchronises the handle's stream. */
int esbgk_reduce_noalloc(esbgk_ctx* ctx, double out[8]);

/* R > 0: fuse the reductions into every R-th step (R = 0 disables);
 * esbgk_last_reduction returns the latest such result. */
int esbgk_set_reduce_interval(esbgk_ctx* ctx, int64_t R);
int esbgk_last_reduction(esbgk_ctx* ctx, double out[8]);

/* Steps taken since the state was last set. */
int64_t esbgk_steps_done(const esbgk_ctx* ctx);

/* Text of the last error on this handle ("" if none); with NULL, the reason
 * the last esbgk_create on this thread failed. */
const char* esbgk_last_error(const esbgk_ctx* ctx);

/* ---- Batches of independent channels -----------------------------------
 * Many small channel problems (all D2Q37 or all D3Q39, same storage and
 * scheme, walls across the last axis, any extents) advance together in one
 * persistent kernel launch: each workgroup owns whole problems and loops over
 * the steps with workgroup barriers in between. */
typedef struct {
  esbgk_shape shape;          /* velset/storage/scheme must match the batch */
  double Kn, Pr, varpi;
  double T_w[2], u_w[2][3];   /* low / high wall */
  double g[3];
  double specular[2];         /* 1 - gamma of the low / high wall (0 = fully
                                 diffuse, the paper's walls; see
                                 esbgk_set_wall_accommodation) */
} esbgk_problem;

/* Bytes of device workspace for the batch (0 if a problem is invalid). */
size_t esbgk_batch_workspace_bytes(const esbgk_problem* problems, int n);
/* New batch handle on a caller-allocated, 256-byte-aligned workspace and a
 * HIP stream. Errors: E_INVALID (a problem's shape, gas or walls),
 * E_UNSTABLE (an ESBGK_EULER problem with dt/tau or dt/(Pr tau) >= 2 at
 * rho = T = 1, as esbgk_set_gas), E_NOMEM (workspace), E_HIP. */
int esbgk_batch_create(const esbgk_problem* problems, int n, void* d_workspace,
                       size_t ws_bytes, void* hip_stream, esbgk_batch** out);
int esbgk_batch_destroy(esbgk_batch* b);
/* Uniform rest state at rho = 1, T = 1 (optionally times 1 + amplitude*noise;
 * noise holds Q * (sum of all cells) values, problem after problem, each
 * [Q][cells]). */
int esbgk_batch_init_equilibrium(esbgk_batch* b, const double* noise, double amplitude);
/* Advance every problem n steps in one persistent launch (asynchronous). The
 * launch (the persistent kernel, then the update of the device step counter
 * it reads its starting level from) is captured in a HIP graph the first
 * time a step count n is used and replayed afterwards; the graphs are
 * released (after waiting for the stream) when the layout or the reduction
 * interval changes. */
int esbgk_batch_step(esbgk_batch* b, int64_t n);
/* on = 0: launch directly instead of replaying captured graphs (the same
 * kernels and results); on = 1 (default): replay. */
int esbgk_batch_use_graphs(esbgk_batch* b, int on);
/* FP64 reductions of every problem, as esbgk_reduce does for one lattice:
 * out[8 * i + k] for problem i holds its mass sum rho, energy
 * sum 1/2 sum_alpha f c^2, momentum sum rho u (3), mass flow rate through a
 * plane normal to x, dx^(D-1)/nx sum rho u_x, the residual
 * ||u - u_prev||_2/||u||_2 since the problem's previous reduction (0 for the
 * first after the state was set) and the level the sums belong to.
 * esbgk_batch_set_reduce_interval(R > 0) fuses them into the persistent
 * kernel's steps from levels R-1, 2R-1, ... (0 disables): the step's
 * reconstructed state, per-cell terms in FP64, summed per 64-cell chunk by a
 * wavefront butterfly and then over the problem's chunks in order by one
 * thread of the workgroup that owns the problem, or of a kernel after the
 * step when problems are cut (deterministic; no atomics). esbgk_batch_reduce forms them now from the stored state in FP64
 * arithmetic and synchronises; esbgk_batch_last_reduction returns the latest
 * of either kind and synchronises (E_STATE if none has run since the state
 * was set). E_NONFINITE (sticky) if a cell of some problem has a non-finite
 * value, rho <= 0 or T <= 0. out holds 8 * (number of problems) doubles. */
int esbgk_batch_set_reduce_interval(esbgk_batch* b, int64_t R);
int esbgk_batch_reduce(esbgk_batch* b, double* out);
int esbgk_batch_last_reduction(esbgk_batch* b, double* out);
/* Fields of problem i (same layout as esbgk_read_moments); synchronises. */
int esbgk_batch_read_moments(esbgk_batch* b, int i, double* h_out, int* F);
/* Stored populations of problem i as FP64 h[Q][cells_i]; synchronises. */
int esbgk_batch_get_populations(esbgk_batch* b, int i, double* h);
/* Launch layout: workgroup size (multiple of 64, at most 1024 for F32 and
 * F16, 256 for F64 storage) and number of bins (one workgroup each;
 * problems are packed longest first into the lightest bin; at most one bin
 * per problem, or per piece of cut problems: esbgk_batch_layout reports the
 * count in use). The default is the largest workgroup and one bin per
 * resident workgroup. */
int esbgk_batch_set_layout(esbgk_batch* b, int threads, int nbins);
int esbgk_batch_layout(const esbgk_batch* b, int* threads, int* nbins);
/* Shape of the current layout: the most pieces (whole problems, or parts of
 * cut problems) one workgroup owns, and the most cells one thread updates
 * per step (a bin's thread slots, each piece rounded up to 64 cells, over the
 * workgroup size). Either output may be NULL. */
int esbgk_batch_layout_info(const esbgk_batch* b, int* max_pieces_per_bin, int64_t* max_cells_per_thread);
/* Cut problems larger than piece_cells (a positive multiple of 64; 0 keeps
 * every problem whole, the default) into pieces of that many cells, packed
 * into the bins like problems, so that a batch of few large problems
 * occupies every compute unit. A cut problem's pieces may lie in different
 * workgroups, so each step is then its own launch (followed, on reduction
 * steps, by a kernel that adds every problem's chunk sums in chunk order:
 * the same bits as whole problems), replayed from graphs of up to 32 steps.
 * Rebuilds the bins with the current workgroup size and the bin count last
 * asked for (the default, esbgk_batch_set_layout or the autotuner's choice),
 * which the number of pieces caps.
 * E_INVALID for another piece_cells. esbgk_batch_split reports the piece
 * size and whether some problem is cut (active = 1). */
int esbgk_batch_set_split(esbgk_batch* b, int piece_cells);
int esbgk_batch_split(const esbgk_batch* b, int* piece_cells, int* active);
/* Autotuner: time steps_per_trial steps of every candidate layout
 * (workgroups of 256..max threads x 1, 2, 4, 8 bins per compute unit or one
 * problem per workgroup; whole problems and, when the largest problem holds
 * more than twice a quarter compute unit's share of the cells, pieces of
 * that share and of a quarter of it) on the uniform rest state and keep the
 * fastest. Overwrites the state: call esbgk_batch_init_equilibrium
 * afterwards. */
int esbgk_batch_autotune(esbgk_batch* b, int steps_per_trial);
int64_t esbgk_batch_steps_done(const esbgk_batch* b);
const char* esbgk_batch_last_error(const esbgk_batch* b);

/* ---- The paper's own scheme (Sec. 3.1) ----------------------------------
 * The velocity set of the paper: the tensor product of the 6-point
 * Gauss-Hermite rule of eq. weight (ESBGK_D2Q36GH: 36 velocities, exact to
 * degree 11 along each axis, carrying the N = 4 expansion). For
 * velocity-set convergence studies the 4-point (ESBGK_D2Q16GH: degree 7,
 * N = 3) and 8-point (ESBGK_D2Q64GH: degree 15, N = 4) products run the
 * same scheme; the paper's validation runs use D = 3, its set cubed
 * (ESBGK_D3Q216GH: 216 velocities, exact to degree 11 per axis, N = 4). The
 * abscissae lie
 * off the lattice, so streaming is the paper's finite-difference update:
 * forward Euler in time and, along each axis, the second-order TVD flux
 * difference with the minmod limiter,
 *   f^{n+1} = f^n - nu_x [F_{i+1/2} - F_{i-1/2}] - nu_y [F_{j+1/2} - F_{j-1/2}]
 *             + (dt/tau)(f^ES - f^n) + dt F,   nu = c dt / dx,
 * with F_{i+1/2} = f_i + (1 - nu)/2 (f_{i+1} - f_i) Psi(Theta_i) for c > 0 and
 * its mirror image (upwind cell i + 1) for c < 0. Every term is evaluated at
 * level n; one fused kernel launch per step. The stored state is the
 * physical f (deviational h = f/w - 1 in the storage type, in the velocity
 * order of esbgk_tvd_set_info).
 *
 * Boundaries: periodic in every axis but the last (y in 2-D, z in 3-D);
 * across the last axis periodic (walls = 0) or bounded by the diffuse walls
 * of Sec. 3.2 (walls = 1): its first and last node rows (planes) lie on the
 * walls and are updated like every node, the ghost nodes the stencil
 * reaches beyond a wall copy the wall node, and after each step the wall
 * node's populations moving into the gas become rho_W S(T_W, u_W) with
 * rho_W the normal flux toward the wall at the first node off it over that
 * of S (a second small kernel launch). Walls are fully diffuse at fixed
 * T_W, u_W.
 *
 * Shape: velset = ESBGK_D2Q16GH / D2Q36GH / D2Q64GH (nz = 1) or
 * ESBGK_D3Q216GH, walls = 0 or 1 (three or more nodes across the channel),
 * scheme = ESBGK_EULER, storage F64 / F32 / F16 (FP32 compute for the last
 * two), n_ref = N_L (0: nx, or the wall distance in nodes minus one with
 * walls). The
 * time step is dt = cfl dx / max|c| with dx = 1/N_L and 0 < cfl <= 1; the
 * largest root, and so dt, depends on the set. Forward Euler on the
 * collision and the unsplit sum of the axes' fluxes stays bounded while
 * d cfl <= 1 - dt/tau for a field that varies along d axes (every abscissa
 * of these sets is nonzero); that choice is the caller's. */
typedef struct esbgk_tvd esbgk_tvd;

/* Number of velocities Q, Hermite order N, abscissae c[Q][D] and weights
 * w[Q] of a product set (any output may be NULL), derived on the host from
 * the roots of He_n and eq. weight; the velocities are ordered by |c|^2,
 * then by descending tuple of root indices, with the opposite of velocity
 * a < Q/2 at a + Q/2. E_INVALID for another velset. */
int esbgk_tvd_set_info(int velset, int* Q, int* N, double* c, double* w);
/* esbgk_tvd_set_info of ESBGK_D2Q36GH: c[36][2], w[36]. */
int esbgk_tvd_info(double* c, double* w);
/* Device workspace bytes for the shape (0 if invalid): two population
 * buffers and, for ESBGK_D3Q216GH, each level's 20 raw moment sums per cell
 * in the compute type (the step reads them instead of a second pass over the
 * cell's 216 populations), plus constants and staging. */
size_t esbgk_tvd_workspace_bytes(const esbgk_shape* shape);
/* New handle on a caller-allocated, 256-byte-aligned workspace and a HIP
 * stream. Gas defaults: Kn = 0.1, Pr = 1, varpi = 0.5; g = 0. Errors:
 * E_INVALID (shape, cfl), E_NOMEM (workspace), E_HIP; the reason is in
 * esbgk_tvd_last_error(NULL). */
int esbgk_tvd_create(const esbgk_shape* shape, double cfl, void* d_workspace, size_t ws_bytes, void* hip_stream,
                     esbgk_tvd** out);
int esbgk_tvd_destroy(esbgk_tvd* t);
/* dt of the handle (nondimensional). */
double esbgk_tvd_time_step(const esbgk_tvd* t);
/* Boundedness of the TVD step (Sec. 3.1 update with forward Euler on the
 * collision): with w = dt/tau at rho = T = 1 (dt = cfl / (n_ref max|c|),
 * tau = Kn/Pr), one step is a convex combination of the equilibrium (weight
 * w) and a TVD advection step whose Courant number is the sum of |nu| over
 * the axes the field varies along, so it stays bounded while
 * axes * cfl <= 1 - w (every abscissa of these sets is nonzero). Returns
 * ESBGK_OK when that holds, ESBGK_E_UNSTABLE when it does not, ESBGK_E_INVALID
 * for an unknown set, n_ref < 1, cfl outside (0, 1], Kn <= 0, Pr < 2/3 or
 * axes outside [1, D]. Touches no GPU; the library does not enforce it (the
 * number of axes the field varies along is the caller's knowledge). */
int esbgk_tvd_bounded(int velset, int n_ref, double cfl, double Kn, double Pr, int axes);
/* Gas (as esbgk_set_gas); E_UNSTABLE when forward Euler is unstable at
 * rho = T = 1 (dt/tau >= 2 or dt/(Pr tau) >= 2). */
int esbgk_tvd_set_gas(esbgk_tvd* t, double Kn, double Pr, double varpi);
/* Wall side (0: the first node row of the last axis, 1: the last) at
 * temperature T_w > 0 moving in its own plane with u_w (no component
 * across the channel; NULL: at rest); defaults T_w = 1, at rest.
 * E_INVALID on a lattice without walls. */
int esbgk_tvd_set_wall(esbgk_tvd* t, int side, double T_w, const double u_w[3]);
int esbgk_tvd_set_body_force(esbgk_tvd* t, const double g[3]);
/* Initial state f = rho S(T, u) (1 + amplitude noise) as
 * esbgk_init_equilibrium (u is [D][cells], noise [Q][cells]). */
int esbgk_tvd_init_equilibrium(esbgk_tvd* t, const double* rho, const double* u, const double* T,
                               const double* noise, double amplitude);
/* Stored populations as FP64 h[Q][cells] (host); set rounds to the storage
 * type and resets the step counter. */
int esbgk_tvd_set_populations(esbgk_tvd* t, const double* h);
int esbgk_tvd_get_populations(esbgk_tvd* t, double* h);
/* Advance n steps (asynchronous on the handle's stream). */
int esbgk_tvd_step(esbgk_tvd* t, int64_t n);
/* rho, u[D], T, sigma (i <= j: xx, xy, yy or xx, xy, xz, yy, yz, zz), q[D]
 * of the stored f per cell, as [F][cells] FP64 (F = 9 in 2-D, 14 in 3-D;
 * FP64 arithmetic); synchronises. */
int esbgk_tvd_read_moments(esbgk_tvd* t, double* h_out, int* F);
int64_t esbgk_tvd_steps_done(const esbgk_tvd* t);
/* Text of the last error on the handle; with NULL, why the last create on
 * this thread failed. */
const char* esbgk_tvd_last_error(const esbgk_tvd* t);

#ifdef __cplusplus
}
#endif

#endif /* ESBGK_H */

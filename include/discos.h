/*
 * discos.h - C ABI of the DISCOS slit-channel particle-grid core for MI355X (gfx950).
 *
 * Method: Ladiges et al., "Modeling electrokinetic flows with the discrete ion
 * stochastic continuum overdamped solvent algorithm", arXiv:2204.14167.  Ions in a
 * channel periodic in x and y with walls at z = 0 ("lo") and z = Lz ("hi").
 *
 * Conventions shared by every entry point
 *   - FP64 everywhere.  All array arguments are DEVICE pointers (hipMalloc'd or
 *     torch tensors on the GPU) unless the comment says "host".  The caller owns
 *     every array it passes; the context owns its own scratch.
 *   - Ion arrays are structure-of-arrays: pos is [3][n] (all x, then all y, then
 *     all z), q is [n].
 *   - Grid (nx, ny, nz, h): cell-centred scalars (rho, phi, pressure) are
 *     [nz][ny][nx] with x fastest, the cell (i, j, k) centred at
 *     ((i+1/2)h, (j+1/2)h, (k+1/2)h).  Face fields (electric field, fluid velocity,
 *     force density) use the staggered MAC layout: the x component at
 *     (i h, (j+1/2) h, (k+1/2) h) as [nz][ny][nx], y likewise, and the z component
 *     at ((i+1/2) h, (j+1/2) h, k h) as [nz+1][ny][nx] (k = 0 and nz on the walls).
 *   - nx and ny are powers of two in [8, 1024]; nz >= 4.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call only
 *     enqueues work on that stream; nothing synchronises except discos_check.
 *   - Return value: DISCOS_OK (0) or a negative status.  Argument errors are
 *     detected on the host before anything is enqueued.  Conditions that only the
 *     device can see (an ion outside the channel, a non-finite position, a
 *     non-neutral all-Neumann system) set a sticky flag that discos_check reports;
 *     the kernels never read or write out of bounds because of them.
 *   - One context per stream at a time: calls that overlap on two streams with the
 *     same context race on its scratch.
 */
#ifndef DISCOS_H
#define DISCOS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------- */
#define DISCOS_OK 0
#define DISCOS_E_ARG (-1)          /* null pointer, bad enum, bad scalar */
#define DISCOS_E_SHAPE (-2)        /* grid / size outside the supported range */
#define DISCOS_E_HIP (-3)          /* a HIP runtime call failed */
#define DISCOS_E_OUT_OF_DOMAIN (-4) /* sticky: an ion had z outside [0, Lz] or |x|, |y| huge */
#define DISCOS_E_NOT_NEUTRAL (-5)  /* sticky: both walls Neumann and the system is charged */
#define DISCOS_E_NONFINITE (-6)    /* sticky: a non-finite position or force */
#define DISCOS_E_CAPACITY (-7)     /* n larger than the context's n_max; host memory exhausted */
#define DISCOS_E_NOT_CONVERGED (-8) /* the iterative Poisson solve of mixed walls did not reach
                                       its tolerance in 1000 iterations */

/* ---- wall boundary conditions for the potential (Sec. II.B.1) --------------- */
#define DISCOS_BC_DIRICHLET 0 /* fixed potential phi_b (eq esbc1) */
#define DISCOS_BC_NEUMANN 1   /* dielectric wall, surface charge sigma, eps >> eps_b (eq esbc3);
                                 sign from Gauss's law: -eps dphi/dz(0+) = sigma_lo and
                                 +eps dphi/dz(Lz-) = sigma_hi */

typedef struct discos_grid {
    int32_t nx, ny, nz; /* cells */
    double h;           /* cell size; Lx = nx h, Ly = ny h, Lz = nz h */
} discos_grid;

/*
 * Physical and numerical parameters, following the paper's statement of the
 * problem.  Scalars are by value; the array members are DEVICE pointers.
 */
typedef struct discos_params {
    /* electrostatics (Sec. II.B.1) */
    double eps;                 /* solvent permittivity */
    int32_t bc_type[2];         /* DISCOS_BC_* for the wall at z = 0 [0] and z = Lz [1] */
    const double* bc_value[2];  /* device [ny][nx] per wall: phi_b (Dirichlet) or sigma
                                   (Neumann) of the column above / below cell (i, j);
                                   NULL means 0 */
    double e_ext[3];            /* applied field; adds q E_ext to each ion (eq totalforce) */
    /* P3M near-field correction (eqs coulomb, fullElectro, LC) */
    double psi;                 /* cutoff radius */
    const double* p3m_table;    /* device [p3m_len]: g(i p3m_dr), free-space grid pair force
                                   in units of q_i q_j / (4 pi eps h^2), argument r / h: the
                                   mean radial force between two unit charges through
                                   S^es, the periodic Poisson solve and J^es, tabulated
                                   offline as the paper describes (an input, like eps) */
    int32_t p3m_len;
    double p3m_dr;
    /* short-range forces (Sec. II.B.2) */
    int32_t wall_on;            /* 9-3 wall potential (eq LJ93) */
    double wall_sigma, wall_xi, wall_cut;
    int32_t lj_on;              /* ion-ion shifted LJ (eq potential, eq closerange) */
    const double* lj_sigma;     /* device [nspecies][nspecies] */
    const double* lj_xi;        /* device [nspecies][nspecies] */
    double lj_cut_factor;       /* cutoff = factor * sigma_ij (2^(1/6): WCA, 2.5: full LJ) */
    double lj_range;            /* largest LJ cutoff (factor * max sigma_ij); sizes the search */
    /* dynamics (Sec. II.C, II.D) */
    double kT, eta, dt;
    int32_t nspecies;
    const double* radius;       /* device [nspecies]: dry radius a, D = kT / (6 pi eta a)
                                   (eq einstein); +INFINITY means no dry diffusion */
    const double* mob_coef;     /* device [nspecies][2][7]: c1..c7 of eq fitfunction for
                                   motion parallel [0] and perpendicular [1] to the walls */
    uint64_t seed;              /* Philox key of every noise term */
    double rfd_delta;           /* step delta of the random finite difference that gives
                                   the thermal forcing f^th = kT div_x S^hy (eq thermforce)
                                   in a DISCOS_STEP_RFD step; (0, 0.1 h] */
    /* hydrodynamic walls (eq fluidbc, Fig. folded) */
    int32_t hydro_bc[2];        /* DISCOS_HYDRO_* for the wall at z = 0 [0] and z = Lz [1]:
                                   no-slip (zero velocity, opposite images) or slip (zero
                                   normal velocity and tangential stress, same-sign
                                   tangential images); with two slip walls the in-plane
                                   mean of the tangential force is solved with its z-mean
                                   removed and zero z-mean flow */
    /* walls of mixed type (Sec. IV.B: a metal strip on a dielectric wall; Sec. II.B.1,
       closing remark: the wall data may vary along the wall) */
    const int32_t* bc_type_map[2]; /* device [ny][nx] per wall, or NULL: the type
                                   (DISCOS_BC_*) of each wall column (i, j), replacing
                                   bc_type[w] for that wall.  Column by column: the image
                                   sign of folded kernel nodes, the wall term, the ghost
                                   values, and the image of a charge (the type of the column
                                   below / above the charge).  A wall whose columns differ
                                   couples the Fourier modes: the Poisson solve is then two
                                   per-mode solves of a uniform wall pair (Dirichlet for a
                                   wall with any Dirichlet column) and, between them, a
                                   capacitance system on the wall layers (Woodbury identity)
                                   iterated by preconditioned conjugate gradients to a
                                   residual below 1e-14 of its right-hand side.
                                   discos_solve_poisson and discos_step copy the maps to the
                                   host (checking every entry) and synchronise the stream,
                                   also to test convergence every few iterations; the other
                                   calls read the maps on the device.
                                   discos_energy_flux(_backward) and batches take uniform
                                   walls only (DISCOS_E_ARG). */
} discos_params;

#define DISCOS_HYDRO_NOSLIP 0
#define DISCOS_HYDRO_SLIP 1

/* Ion state for discos_step.  pos, q, id and species are DEVICE arrays of length n. */
typedef struct discos_ions {
    int64_t n;
    double* pos;      /* [3][n] */
    double* q;        /* [n] */
    int32_t* id;      /* [n] stable ids (key of the ion's noise) */
    int32_t* species; /* [n] in [0, nspecies) */
} discos_ions;

typedef struct discos_ctx discos_ctx;

/*
 * Create a context for one grid and at most n_max ions (n_max < 2^26).  Allocates
 * every scratch buffer the other calls need (FFT twiddles, cell lists, neighbour
 * lists, spectra), so later calls allocate nothing.  flags: DISCOS_CREATE_HYDRO adds
 * the buffers of discos_solve_stokes, DISCOS_SPREAD_FORCE, DISCOS_INTERP_VEL and the
 * wet step (about 200 bytes per cell).  Uses the current HIP device.
 * Errors: DISCOS_E_ARG, DISCOS_E_SHAPE, DISCOS_E_HIP.
 */
#define DISCOS_CREATE_HYDRO 1u /* also allocate the Stokes / wet-step scratch */
/* Walls of mixed type (discos_params.bc_type_map) are solved through a capacitance
 * system on the wall layers.  By default, when it has at most DISCOS_MIXED_DENSE_MAX
 * unknowns, the system's inverse is formed once per set of maps (a dense Cholesky
 * factorisation; the one exception to "later calls allocate nothing": up to
 * 8 DISCOS_MIXED_DENSE_MAX^2 bytes, allocated when a map set is first solved) and each
 * solve applies it; otherwise, and always with this flag, it is solved by conjugate
 * gradients with no allocation. */
#define DISCOS_CREATE_MIXED_ITERATIVE 2u
#define DISCOS_MIXED_DENSE_MAX 16384
/* A dry step runs its near field on a second stream of the context beside the spread,
 * Poisson solve and interpolation (discos_step).  With this flag every stage runs in
 * order on the caller's stream instead (each kernel then has the chip to itself, as a
 * profile of the kernels one by one needs); results are the same. */
#define DISCOS_CREATE_SERIAL 4u
int discos_create(const discos_grid* grid, int64_t n_max, uint32_t flags, discos_ctx** out);
/* Waits for the device, then releases the context and its buffers.  Everything is
 * released even when the runtime reports an error on the way; that error is returned
 * as DISCOS_E_HIP.  DISCOS_E_ARG for a null context. */
int discos_destroy(discos_ctx* ctx);

/*
 * Spreading S (eq kernel2) with the 4-point Peskin kernel (App. B, eq peskin1d) and
 * image folding at the walls (Sec. II.A, Fig. folded).
 *   DISCOS_SPREAD_CHARGE: rho = S^es q, w = q [n], out = rho [nz][ny][nx]; the image
 *     of each charge is opposite at a Dirichlet wall and like-signed at a Neumann
 *     wall (Sec. II.B.1).  With DISCOS_SPREAD_ADD_BC or-ed into op, the wall-condition
 *     terms of the discrete Poisson problem are added to layers 0 and nz-1:
 *     2 eps phi_b / h^2 (Dirichlet) or sigma / h (Neumann).
 *   DISCOS_SPREAD_FORCE: f = S^hy F on the MAC faces, w = F [3][n], out = f_x, f_y, f_z
 *     back to back (sizes nz*ny*nx, nz*ny*nx, (nz+1)*ny*nx); no-slip images: every
 *     component folds with sign -1; the z-faces mirror k -> -k about the wall face.
 * `out` is overwritten.  Ions may come in any order.
 */
#define DISCOS_SPREAD_CHARGE 0
#define DISCOS_SPREAD_FORCE 1
#define DISCOS_SPREAD_ADD_BC 0x100
int discos_spread(discos_ctx* ctx, int op, int64_t n, const double* pos, const double* w,
                  const discos_params* p, double* out, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): S^es charge spreading as
 * discos_spread(DISCOS_SPREAD_CHARGE[ | DISCOS_SPREAD_ADD_BC]) without a context.
 * rho = S^es q (eq kernel2, images folded per Sec. II.B.1; with DISCOS_SPREAD_ADD_BC in
 * flags, the wall terms as for discos_spread).  pos [3][n], q [n] and rho [nz][ny][nx]
 * are DEVICE arrays owned by the caller; rho is overwritten.  p supplies eps, bc_type
 * and bc_value only; bc_type_map must be NULL (walls of one type each), else
 * DISCOS_E_ARG.  status: DEVICE int32 [1] or NULL; receives DISCOS_OK or the
 * sticky device condition of this call (DISCOS_E_NONFINITE, DISCOS_E_CAPACITY,
 * DISCOS_E_OUT_OF_DOMAIN).
 * Allocates nothing: its cell list lives in one fixed device array of about 4.8 MiB
 * per GPU, held until the process ends, which limits a call to
 * n <= DISCOS_NOALLOC_MAX_IONS and (nx/2)(ny/2)ceil(nz/2) <= DISCOS_NOALLOC_MAX_BINS
 * (for example 65,536 ions on 128 x 128 x 64 cells); larger calls return
 * DISCOS_E_CAPACITY before anything is enqueued.  Every call on one GPU shares that
 * array, so calls that overlap on one GPU (two streams, two threads) race.  Runs on the
 * current device.  Errors: DISCOS_E_ARG, DISCOS_E_SHAPE, DISCOS_E_CAPACITY, DISCOS_E_HIP.
 */
#define DISCOS_NOALLOC_MAX_IONS 65536
#define DISCOS_NOALLOC_MAX_BINS 262144
int discos_spread_charge_noalloc(const discos_grid* grid, int64_t n, const double* pos,
                                 const double* q, const discos_params* p, uint32_t flags,
                                 double* rho, int32_t* status, void* stream);

/*
 * Solve -eps lap_h phi = rhs (eq poisson) with the walls' homogeneous ghost rules
 * (phi_{-1} = -phi_0 Dirichlet, +phi_0 Neumann); inhomogeneous wall values enter
 * through rhs (DISCOS_SPREAD_ADD_BC).  In-plane FFTs, then one tridiagonal solve in z
 * per Fourier mode.  When both walls are Neumann the kappa = 0 mode is solved with
 * mean(phi) = 0 after removing the mean of its RHS; if that mean is larger than
 * 1e-10 of the sum of the absolute plane sums the sticky DISCOS_E_NOT_NEUTRAL flag is
 * set.  rhs is read-only; phi [nz][ny][nx] is overwritten (may alias rhs).
 */
int discos_solve_poisson(discos_ctx* ctx, const double* rhs, const discos_params* p,
                         double* phi, void* stream);

/*
 * Fluctuating Stokes solve with no-slip walls (eq disc_stokes / disc_stokes_temp):
 * G p - eta lap_h v = f + sqrt(2 kT eta / (dV dt)) div_h Z,  D v = 0,  with w = 0 on the
 * wall faces and ghosts u_{-1} = -u_0 for the tangential components.  f and v are
 * three face arrays back to back (layout of DISCOS_SPREAD_FORCE); pres ([nz][ny][nx],
 * mean zero) may be NULL.  With DISCOS_STOKES_NOISE the stochastic stress Z is drawn
 * from Philox with key p->seed and counter step `step`: diagonal entries at cell
 * centres (variance 2), off-diagonal entries on cell edges (variance 1, and 2 for the
 * xz / yz edges on the walls, which makes the discrete fluctuation-dissipation balance
 * exact).  Uses p->eta, p->kT, p->dt.  Needs a context created with
 * DISCOS_CREATE_HYDRO.  f is read-only; v and f must not overlap.
 */
#define DISCOS_STOKES_NOISE 1
int discos_solve_stokes(discos_ctx* ctx, const double* f, const discos_params* p, uint64_t step,
                        int flags, double* v, double* pres, void* stream);

/*
 * Interpolation J (eq kernel1), Delta V sum_n delta(x_i - r_n) f_n:
 *   DISCOS_INTERP_E:   field = phi [nz][ny][nx]; out [3][n] = E^P = J^es(-grad_h phi)
 *                      (eq efieldop), E on the faces, ghosts filled from the wall
 *                      conditions in p (exact for potentials affine in z).
 *   DISCOS_INTERP_FORCE: as DISCOS_INTERP_E, out [3][n] = q_i (E^P_i + E_ext), with
 *                      q passed through `aux`.
 *   DISCOS_INTERP_PHI: field = phi; out [n] = J phi (centres, homogeneous ghosts
 *                      plus the wall values in p).
 *   DISCOS_INTERP_VEL: field = v faces (layout of DISCOS_SPREAD_FORCE); out [3][n] = J^hy v
 *                      with no-slip ghosts.
 * out is overwritten; ions may come in any order.
 */
#define DISCOS_INTERP_E 0
#define DISCOS_INTERP_FORCE 1
#define DISCOS_INTERP_PHI 2
#define DISCOS_INTERP_VEL 3
int discos_interpolate(discos_ctx* ctx, int op, int64_t n, const double* pos,
                       const double* field, const double* aux, const discos_params* p,
                       double* out, void* stream);

/*
 * Hydrodynamic kernel per species (App. B, eq eskernel; a project addition on Sec. III.B,
 * where cations and anions use different kernels).  kernel: HOST array [nspecies][2] of
 * (w, beta): w = 0 keeps the 4-point Peskin kernel; w = 2 .. 8 selects the ESC kernel
 *   phi(zeta) = exp(beta (sqrt(1 - (zeta / alpha)^2) - 1)) / I,  alpha = w h / 2,
 * normalised by its integral I, with beta in [0, 100].  Species beyond nspecies use the
 * Peskin kernel; nspecies = 0 (or kernel = NULL) restores it for all.  The kernels apply
 * to discos_spread_force_species, discos_interpolate_vel_species and the hydrodynamic
 * stages of discos_step (S^hy, the random finite difference, J^hy); the plain
 * DISCOS_SPREAD_FORCE and DISCOS_INTERP_VEL keep the Peskin kernel.  Needs
 * DISCOS_CREATE_HYDRO and nz > w for every w > 0.  A set-up call: it synchronises the
 * device before replacing the table that calls in flight may read.
 * Errors: DISCOS_E_ARG, DISCOS_E_SHAPE, DISCOS_E_HIP.
 */
#define DISCOS_HY_MAXSP 8
int discos_set_hydro_kernel(discos_ctx* ctx, int32_t nspecies, const double* kernel);

/* S^hy F (as DISCOS_SPREAD_FORCE) with each ion's kernel chosen by its species (DEVICE
 * [n]; a species without a kernel set, negative ones included, uses the Peskin kernel);
 * out: the three face arrays back to back. */
int discos_spread_force_species(discos_ctx* ctx, int64_t n, const double* pos, const double* F,
                                const int32_t* species, const discos_params* p, double* out,
                                void* stream);

/* J^hy v (as DISCOS_INTERP_VEL) with each ion's kernel chosen by its species; out [3][n]. */
int discos_interpolate_vel_species(discos_ctx* ctx, int64_t n, const double* pos, const double* v,
                                   const int32_t* species, const discos_params* p, double* out,
                                   void* stream);

/*
 * Near-field pass: the P3M correction sum_j (F^C_ij - F^P_ij) over pairs closer than
 * psi (minimum image in x, y) and over the wall images of every ion (charge s q_j at
 * (x_j, y_j, -z_j) and (x_j, y_j, 2 Lz - z_j), s = -1 Dirichlet, +1 Neumann,
 * including an ion's own image) (Sec. II.B.1, eq LC), plus the 9-3 wall force and,
 * if enabled, the ion-ion LJ force (Sec. II.B.2).  F [3][n] is ACCUMULATED (F += ...).
 * species may be NULL when lj_on == 0.  Uses a cell list with bins of two cells.
 */
int discos_near_field(discos_ctx* ctx, int64_t n, const double* pos, const double* q,
                      const int32_t* species, const discos_params* p, double* F,
                      void* stream);

/*
 * One time step (Sec. II.D).  mode DISCOS_STEP_DRY: stages 1-2 (spread, Poisson,
 * interpolation, P3M near-field, wall and applied forces) and the dry update of
 * eq ions3 / eq step2 with the wall-modified diffusion tensor D Gamma(z) of
 * eq diff1 and its Ito drift D dGamma_z/dz, Euler-Maruyama in the Ito sense, noise
 * W ~ N(0,1) from Philox4x32-10 with counter (id, step, 1, pair) and key `seed`;
 * ions crossing a wall are reflected and x, y are wrapped into [0, L).
 * The ion arrays are PERMUTED in place into cell order (ids follow their ions).
 * In a dry step the near-field pass runs on a stream the context owns, forked from
 * `stream` after the cell list and joined back before the update (events only, so the
 * step can be captured into a graph from `stream`); nothing is left running when the
 * step's work on `stream` is done.
 */
#define DISCOS_STEP_DRY 0
/* DISCOS_STEP_WET: the forces as in the dry step, then stage 3 (S^hy F, fluctuating
 * no-slip Stokes solve with noise counter `step`, eq disc_stokes_temp) and stage 4
 * (eq step1 / step2): the midpoint x* = x + dt/2 J(x) v (wrapped and reflected like
 * the final positions), x+ = x + dt J(x*) v plus the dry terms evaluated at x (the
 * dry radius in p->radius; +INFINITY switches the dry part off).  Needs
 * DISCOS_CREATE_HYDRO and kT, dt > 0.
 * DISCOS_STEP_RFD (or-ed with DISCOS_STEP_WET) adds the thermal forcing of
 * eq thermforce by the random finite difference
 *   f^th = (kT / delta) [S^hy(x + delta/2 W) W - S^hy(x - delta/2 W) W],
 * W ~ N(0, I) per ion from Philox counter (id, step, 4, pair), delta = p->rfd_delta. */
#define DISCOS_STEP_WET 1
#define DISCOS_STEP_RFD 0x10
int discos_step(discos_ctx* ctx, discos_ions* ions, const discos_params* p, uint64_t step,
                int mode, void* stream);

/*
 * Energy and electro-osmotic flux of the electrostatic pass (a project addition on
 * Sec. II.B.1 and stages 1-2 of Sec. II.D):
 *   rho = S^es q + b (b: the wall terms), phi = A^+ rho (A = -eps lap_h with homogeneous
 *   ghosts; the mean-zero solution when both walls are Neumann),
 *   U = (1/2) dV <rho, phi>,   Q = sum_i w(z_i) q_i (E^P_x,i + E_ext,x),
 * with E^P from J^es of the staggered field (eq efieldop) and w(z) the channel-mean x
 * velocity per unit x force at height z of the no-slip Stokes flow: the kappa = 0 mode
 * of eq disc_stokes, -eta D_zz g = 1 / nz, spread with S^hy (needs p->eta > 0).
 * phi: DEVICE [nz][ny][nx], receives the potential (the checkpoint of the backward
 * pass); out: DEVICE [2], receives U and Q.  pos [3][n] and q [n] are DEVICE arrays.
 */
int discos_energy_flux(discos_ctx* ctx, int64_t n, const double* pos, const double* q,
                       const discos_params* p, double* phi, double* out, void* stream);

/*
 * Vector-Jacobian product of discos_energy_flux (hand-written adjoint): with the
 * cotangents g = (gU, gQ) (DEVICE [2]) writes gU dU/d(.) + gQ dQ/d(.) with respect to
 * the positions (dpos, [3][n]), the charges (dq, [n]), the wall fields (dbc_lo,
 * dbc_hi, [ny][nx]: phi_b or sigma of each column) and the applied field (de, [3]).
 * Every output is a DEVICE array, may be NULL (not computed), and is overwritten.
 * phi must be the checkpoint written by discos_energy_flux for the same pos, q and p.
 * Cost: one transposed interpolation, one Poisson solve, one gradient gather, and the
 * cell list of the ions unless flags has DISCOS_ADJ_REUSE_CELLS: the caller then states
 * that pos and q are unchanged since the discos_energy_flux call that wrote phi, and
 * the cell list that call built is used again, if no call on the context has rebuilt
 * it since and n is the same (else it is rebuilt); de then also takes the sum of
 * w(z_i) q_i that the forward pass accumulated, when p->eta is the same.
 */
#define DISCOS_ADJ_REUSE_CELLS 1u
int discos_energy_flux_backward(discos_ctx* ctx, int64_t n, const double* pos, const double* q,
                                const discos_params* p, const double* phi, const double* g,
                                double* dpos, double* dq, double* dbc_lo, double* dbc_hi,
                                double* de, uint32_t flags, void* stream);

/*
 * Batches of independent channels (a project addition; each channel is exactly the
 * problem of discos_step in dry mode, with its own grid, ion count, noise key and wall
 * values; Sec. II.D stages 1-2 and the dry update).  All channels share h and the
 * physics of one discos_params (its bc_value and seed are ignored: each channel
 * brings its own).  Every stage is one launch over all channels: tile stages walk a
 * (channel, tile) task table in a persistent grid, per-ion stages look up each ion's
 * channel, and the FFTs run per (nx, ny) size class.
 */
typedef struct discos_replica {
    int32_t nx, ny, nz;         /* nx, ny powers of two in [8, 1024]; nz >= 4 */
    int64_t n;                  /* ions of this channel */
    double bc_value[2];         /* uniform wall values (phi_b or sigma) of the two walls */
    uint64_t seed;              /* Philox key of this channel's noise */
    const double* mob_coef;     /* device [nspecies][2][7] for this channel height, or NULL
                                   for p->mob_coef */
} discos_replica;

typedef struct discos_batch discos_batch;

/* Lays the channels out and allocates every buffer (nothing is allocated later).
 * reps: host array of `count` channels.  The ions of channel r occupy entries
 * [off_r, off_r + n_r) of the batch ion arrays, off_r = n_0 + ... + n_{r-1}. */
int discos_batch_create(const discos_replica* reps, int32_t count, double h,
                        const discos_params* p, discos_batch** out);
/* Releases the batch as discos_destroy does a context (DISCOS_E_HIP if the runtime
 * reported an error on the way, everything released regardless). */
int discos_batch_destroy(discos_batch* b);

/* One dry step of every channel.  pos [3][N], q [N], id [N], species [N] (DEVICE,
 * N = total ions) are permuted in place into cell order within each channel's range.
 * flags & DISCOS_BATCH_GRAPH: run the step as a captured hipGraph (captured on the first
 * call, and again whenever the arrays change); the step counter then lives on the
 * device and advances with each replay. */
#define DISCOS_BATCH_GRAPH 1u
int discos_batch_step(discos_batch* b, double* pos, double* q, int32_t* id, int32_t* species,
                      uint64_t step, uint32_t flags, void* stream);

/* Autotuner: for each cell-list bin edge (2 cells, and 4 cells when every channel is at
 * least 2 (2R + 1) cells wide for the near-field search radius R of 4-cell bins), times
 * the spread tile (8^3 or 16^3) with its persistent block count, the interpolation tile
 * (8x8x8 or 16x16x8) with its block count, the channel densities below which the
 * interpolation reads each ion's window directly instead of staging tiles and the spread
 * adds each ion's window with global atomics (0, 8, 24, 64 ions per 2048 cells, or every
 * channel), and the workgroup size of the per-ion stages on the current ions, without
 * advancing them, and keeps the fastest of each; then keeps the bin edge whose cell list,
 * spread, interpolation and near field take the least time together.  cfg (host [10],
 * nullable) receives spread tile, spread blocks (0 = one per task), interpolation tile,
 * interpolation blocks, per-ion workgroup size, the two densities (interpolation, spread;
 * 2^30: every channel), the bin edge in cells, and the microseconds those four stages
 * took together with bins of 2 and of 4 cells (0: not tried).  Results do not depend on
 * the choices (the bins only order the work). */
int discos_batch_tune(discos_batch* b, const double* pos, const double* q, const int32_t* id,
                      const int32_t* species, int32_t* cfg, void* stream);

/* Sets the cell-list bin edge of the batch to `bin` cells (2, the default, or 4), as the
 * autotuner would; DISCOS_E_ARG for another value, DISCOS_E_SHAPE if some channel is
 * narrower than 2 (2R + 1) bins of that edge.  Synchronises the device; a captured graph
 * is captured again at the next graph step. */
int discos_batch_set_bin(discos_batch* b, int32_t bin);

/* Sticky device flags of the batch (as discos_check) and the last host error. */
int discos_batch_check(discos_batch* b);
const char* discos_batch_last_error(discos_batch* b);

/*
 * Stage timing of discos_step.  discos_profile(ctx, 1) clears the record and makes the
 * next (up to 512) steps record a hipEvent on their stream after each stage;
 * discos_profile(ctx, 0) stops recording.  discos_profile_read synchronises and writes
 * the mean elapsed milliseconds per recorded step of each stage (host array of at
 * least DISCOS_NSTAGE doubles, order: cell list, spread, x-FFT, y-FFT, z-solve,
 * inverse y-FFT, inverse x-FFT, interpolation, the near field's padded cell list, the
 * near-field pass (candidates, pair forces, wall force, and in a dry step the update),
 * S^hy, Stokes solve, the two J^hy passes with the predictor, the update of a wet step;
 * with walls of mixed type the whole iterative Poisson solve is timed as the x-FFT stage)
 * and sets *count (0 when no step was recorded).  In a dry step the padded list and the
 * pass run on the context's second stream beside the spread .. interpolation stages (the
 * stages overlap), S^hy and the Stokes solve read 0, the J^hy stage reads the time the
 * grid stages ran past the end of the pass, and the last stage the dry update.  Each
 * recorded event costs the stream a few microseconds.
 */
#define DISCOS_NSTAGE 14
int discos_profile(discos_ctx* ctx, int enable);
int discos_profile_read(discos_ctx* ctx, double* ms, int* count);

/* As discos_profile(ctx, 1), but only the stages whose bit (1 << k, k in the order
 * above) is set in `stages` are timed: their two bounding events are the only ones
 * recorded (each recorded event costs the stream a few microseconds).  The other
 * stages read 0.  stages = 0 stops recording. */
int discos_profile_stages(discos_ctx* ctx, uint32_t stages);

/* Synchronise the context's last stream and return (and clear) the sticky status:
 * DISCOS_E_NONFINITE, DISCOS_E_ARG (a species index outside [0, nspecies)),
 * DISCOS_E_CAPACITY (a tile's candidate rows exceeded its buffer: results incomplete;
 * the built tile shapes cannot reach it), DISCOS_E_NOT_NEUTRAL or
 * DISCOS_E_OUT_OF_DOMAIN, in that order of precedence. */
int discos_check(discos_ctx* ctx);
/* Text of the last host-side error on this context (static storage, never NULL). */
const char* discos_last_error(discos_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* DISCOS_H */

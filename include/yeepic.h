/*
 * yeepic.h -- C ABI of the MI355X (gfx950) dual-stencil FDTD particle-in-cell
 * hot path of F. Li et al., "A new field solver for modeling of relativistic
 * particle-laser interactions using the particle-in-cell algorithm"
 * (arXiv:2004.03754).
 *
 * Conventions shared by every call
 * --------------------------------
 * Units: normalised, c = m_e = e = 1 (Sec. 2.1).
 * Mesh: Yee staggering, periodic in every direction.  Each field component is
 *   one caller-owned device array laid out [n3][n2][n1] (x1 contiguous).
 *   Index (k, j, i) holds the component at its own staggered location:
 *     E1 (i+1/2, j, k)  E2 (i, j+1/2, k)  E3 (i, j, k+1/2)
 *     B1 (i, j+1/2, k+1/2)  B2 (i+1/2, j, k+1/2)  B3 (i+1/2, j+1/2, k)
 *   J has the E staggering.  A 2D mesh is ndim = 2 (no x3 derivatives).
 *   With n3 > 1 a 2D grid is a stack of n3 independent 2D meshes (a batch):
 *   plane k holds one mesh, and a particle belongs to the plane floor(x3)
 *   (its x3 holds the plane index, clamped into [0, n3); dx3 is 1 in 2D).
 * Time levels: between calls E^n and B^n are both at integer time t^n
 *   (Eq. pusher: the magnetic field seen by the particles is the average of
 *   the two half-step values, which the half-step B update produces).
 *   Particle positions x are at t^n, momenta u = gamma*beta at t^{n-1/2}.
 * Precision: PIC_FP64 keeps fields in double; PIC_FP32_FIELDS keeps E, B, J in
 *   float and advances them in float.  Particles are always double and every
 *   particle computation (gather sums, gamma, pushers, deposit weights) is
 *   done in double.
 * Streams: every device call is asynchronous on the grid's stream (the
 *   hipStream_t given at init; NULL is the default stream).  Errors that
 *   only the device can see surface at pic_sync.
 * Errors: every call returns a pic_status; nothing throws across the ABI.
 *   pic_last_error() gives a thread-local message for the last failure.
 * Ownership: fields and particles belong to the caller and must stay valid
 *   while the grid is used; the grid copies the coefficient arrays and owns
 *   only its handle, a second field buffer set used by the fused sweep, and
 *   the particle sort scratch.
 */
#ifndef YEEPIC_H
#define YEEPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PIC_OK = 0,
  PIC_EINVAL = -1,        /* bad argument: null pointer, size, enum value */
  PIC_ECFL = -2,          /* time step violates the CFL bound of Sec. 3.2 */
  PIC_EHIP = -3,          /* a HIP runtime call failed */
  PIC_ESHAPE = -4,        /* mesh shape or alignment not supported */
  PIC_ENOMEM = -5,        /* device allocation failed */
  PIC_EUNSUPPORTED = -6,  /* valid request outside what is implemented */
  PIC_ENONFINITE = -7,    /* a non-finite value was found */
  PIC_ENOCONV = -8        /* an exact push's proper-time solve hit its iteration cap */
} pic_status;

typedef enum { PIC_FP64 = 0, PIC_FP32_FIELDS = 1 } pic_precision;
/* How the on-chip tile currents of a 3D deposit reach J (Sec. 3.3 current):
 * added with atomics in whatever order the tiles finish (the default), or
 * stored per tile and summed per node in a fixed order, so that the current,
 * and every field and particle state computed from it, is the same bit for
 * bit from run to run. */
typedef enum { PIC_DEPOSIT_ATOMIC = 0, PIC_DEPOSIT_DETERMINISTIC = 1 } pic_deposit_mode;
/* Pushers (Sec. 1, Sec. 4.1): Boris; the exact constant-field (analytic)
 * pusher; Higuera-Cary (the published method the paper cites and uses in its
 * single-particle runs: the Boris splitting with the rotation at the Lorentz
 * factor that keeps relativistic E x B drift exact). */
typedef enum { PIC_PUSH_BORIS = 0, PIC_PUSH_ANALYTIC = 1, PIC_PUSH_HC = 2 } pic_pusher;
/* Coefficient targets (k-space operators divided by k_g1 = 2 pi/dx1, at
 * kappa = k1/k_g1, r = dt/dx1): Eq. (new_op) E and B; the Xu solver's
 * [k]_{1,t} (Sec. 4); the Yee t-stagger pair of Sec. 4, read as Eq. (new_op)
 * with the Yee symbol in place of [k]_{1,t}: sin(pi kappa)/(pi cos(pi kappa r))
 * for E and sin(pi kappa) cos(pi kappa r)/pi for B. */
typedef enum {
  PIC_TARGET_E = 0,
  PIC_TARGET_B = 1,
  PIC_TARGET_XU = 2,
  PIC_TARGET_YEET_E = 3,
  PIC_TARGET_YEET_B = 4
} pic_target;

#define PIC_MAX_M 16

typedef struct pic_grid_desc {
  int ndim;            /* 2 or 3 */
  int64_t n[3];        /* cells n1, n2, n3; in 2D n3 is the number of stacked planes */
  double dx[3];        /* cell sizes; dx[2] unused when ndim == 2 */
  double dt;           /* time step */
  int M;               /* number of x1 coefficients, 1..PIC_MAX_M */
  const double *CE;    /* host, length M: Faraday x1 stencil C^E (App. B) */
  const double *CB;    /* host, length M: Ampere x1 stencil C^B (App. B) */
  int prec;            /* pic_precision */
  void *E[3];          /* device, n1*n2*n3 elements each (double or float) */
  void *B[3];
  void *J[3];          /* device current; may all be NULL for vacuum runs */
  void *stream;        /* hipStream_t or NULL */
} pic_grid_desc;

typedef struct pic_particles {
  int64_t np;          /* number of particles (0 allowed) */
  double *x[3];        /* device positions in [0, n_d dx_d); in 2D x[2] is the plane
                          index (may be NULL when n3 == 1) */
  double *u[3];        /* device momenta gamma*beta (per unit mass) */
  double q, m, w;      /* charge, mass, macro-weight (density per particle) */
  int64_t *id;         /* optional device labels (may be NULL), permuted together
                          with x and u whenever a call reorders the particles */
} pic_particles;

typedef struct pic_grid pic_grid;   /* opaque */

/* Cotangents for pic_adjoint_step (FP64 grids). */
typedef struct pic_adjoint {
  void *lE[3];         /* device, caller-owned, layout of E: dL/dE (in: at t^{n+1}, out: at t^n) */
  void *lB[3];         /* device, caller-owned, layout of B: dL/dB (same) */
  double *gCE;         /* device, PIC_MAX_M doubles: dL/dC^E_j, accumulated (+=) for j < M */
  double *gCB;         /* device, PIC_MAX_M doubles: dL/dC^B_j, accumulated (+=) for j < M */
  const void *En[3];   /* optional (all six or none): the forward state at t^{n+1}, E ... */
  const void *Bn[3];   /* ... and B, read only; when given the step recomputes no sweep */
  const void *Bh[3];   /* optional (with En, Bn; all three or none): B^{n+1/2} of the step,
                          read only; when given the step rebuilds nothing */
  void *lEo[3];        /* optional (all six or none), device, layout of E: receive dL/dE at t^n
                          (out of place); lE and lB are then only read */
  void *lBo[3];        /* ... and dL/dB at t^n */
} pic_adjoint;

/* ---- coefficient design (host only; App. B) ------------------------------
 * Customized x1 coefficients C (length M) fitting the Eq. (new_op) target
 * ``target`` for r = dt/dx1: minimise int_0^{1/2} w (sum_j C_j
 * sin((2j-1) pi kappa)/pi - T(kappa))^2 dkappa subject to the order-p
 * constraint sum_j C_j (2j-1)^(2i-1)/(2i-1)! = delta_i1 (i = 1..p/2), with
 * the super-Gaussian weight w = exp[-ln2 (width_factor kappa / wk1)^n].
 * The paper's values are n = 10, wk1 = 0.3-0.4, width_factor = 2, p = 2.
 * Solved by a null-space least-squares QR in binary128 arithmetic on a
 * composite Gauss-Legendre discretisation of the integral.  ``out`` is host
 * memory of length M.  Returns PIC_EINVAL for M outside 1..PIC_MAX_M, p odd,
 * p/2 > M, r <= 0 or r >= 1, or non-positive weight parameters. */
int pic_design_coeffs(int M, double r, int target, int p, int n, double wk1,
                      double width_factor, double *out);

/* ---- grid ------------------------------------------------------------------
 * Validates the descriptor, copies the coefficients, checks the CFL bound of
 * Sec. 3.2 in its sufficient form dt <= 1/sqrt(sum|C^B| sum|C^E|/dx1^2 +
 * sum_{d>=2} 1/dx_d^2) (PIC_ECFL when violated), allocates the second field
 * buffer set and returns a handle in *out.  Trailing coefficients whose
 * magnitudes sum to at most 2^-70 times sum|C| are treated as zero (their
 * effect is far below double rounding); the remaining widths select the
 * kernels.  The field pointers must be 16-byte aligned; n1 must be a
 * multiple of 64 and at least 2*M (PIC_ESHAPE otherwise). */
int pic_init_grid(const pic_grid_desc *desc, pic_grid **out);

/* Replace the field/current pointers (same shape and precision). */
int pic_set_fields(pic_grid *g, void *const E[3], void *const B[3], void *const J[3]);

/* ---- field steps (Eq. maxwell with the App. B operators) -----------------
 * pic_advance_B_half: B <- B - (dt/2) d_E x E, where along x1
 *   d^E f_i = (1/dx1) sum_j C^E_j (f_{i+j} - f_{i-j+1}) and x2, x3 use Yee
 *   forward differences.  In place.
 * pic_advance_E: E <- E + dt (d_B x B - J_A) with
 *   d^B f_i = (1/dx1) sum_j C^B_j (f_{i+j-1} - f_{i-j}) and Yee backward
 *   differences along x2, x3; J is used only when use_J != 0 (it must then
 *   be set).  In place.
 * pic_field_sweep: one full step (E^n, B^n) -> (E^{n+1}, B^{n+1}) as a
 *   B half step, an E step and a B half step fused in one pass over the
 *   mesh (reads E, B, [J]; writes E, B).  The result ends in the caller's
 *   arrays.
 * J_A, the current of Ampere's law, is J itself when C^B is the Yee stencil;
 * otherwise its x1 component is the corrected one of pic_current_correction
 * (Sec. 3.3), computed into library-owned memory on each such call.  J, which
 * holds the deposited (charge-conserving) current, is never modified. */
int pic_advance_B_half(pic_grid *g);
int pic_advance_E(pic_grid *g, int use_J);
int pic_field_sweep(pic_grid *g, int use_J);

/* ---- x1 current correction (Sec. 3.3, Eq. correction) ----------------------
 * Writes into J1_out the x1 current that Ampere's law uses with the grid's
 * C^B: per Fourier mode along x1,  J_A1 = ([k]_Yee / [k]_B1) J1,  where J1 =
 * J[0] is the deposited current (continuity holds with the Yee divergence) and
 * [k]_B1 = sum_j C^B_j sin((2j-1) k1 dx1/2)/(dx1/2).  This is the direction for
 * which div_B E - rho keeps its initial value; the k1 = 0 mode is kept (the
 * order constraint makes the ratio 1 there).  The multiplier is applied as a
 * periodic x1 convolution whose taps the library computes at pic_init_grid
 * from the ratio on the n1 discrete modes, truncated where they fall below
 * 2^-56 of their sum for FP64 fields, 2^-32 for FP32 fields (at most 64
 * cells each side).  With the Yee stencil it
 * is a copy.  J1_out: device, caller-owned, one array in the field layout and
 * precision, 16-byte aligned, not overlapping J[0].  Returns PIC_EINVAL
 * without J, PIC_EUNSUPPORTED if [k]_B1 vanishes at a nonzero mode or the
 * taps do not decay within 64 cells (or n1/2 - 1). */
int pic_current_correction(pic_grid *g, void *J1_out);

/* ---- particles (App. A gather, Sec. 1 / 4.1 pushers) ---------------------
 * Gathers E^n and B^n at x^n with the linear shape, each component from its
 * own staggered points; pushes u^{n-1/2} -> u^{n+1/2} with the Boris, the
 * exact constant-field (analytic) or the Higuera-Cary pusher; advances
 * x^{n+1} = x^n + dt u/gamma and wraps it periodically.  If x_old is not
 * NULL, x^n is also written to x_old[d] (device, np doubles each; x_old[2]
 * may be NULL in 2D).  Positions outside [0, L) are clamped into the mesh
 * for the gather (never out of bounds) and reported by pic_check. */
int pic_gather_push(pic_grid *g, pic_particles *p, int pusher, double *const x_old[3]);

/* Particle shape of the gather and the deposit: order 1 the linear shape (the
 * default), order 2 the quadratic B-spline the Sec. 4.2 run lists (three
 * nodes around the nearest one per direction in the gather; the Esirkepov
 * decomposition of Sec. 3.3 on four-node stencils in the deposit, so
 * continuity with the Yee divergence still holds exactly).  Applies to every
 * later call on the grid.  PIC_EINVAL for another order; the adjoint refuses
 * order 2 (PIC_EUNSUPPORTED). */
int pic_set_shape(pic_grid *g, int order);

/* ---- current (Sec. 3.3) ----------------------------------------------------
 * Adds the charge-conserving (Esirkepov) current J^{n+1/2} of particles that
 * moved from x_old to p->x (less than one cell per step; the periodic wrap is
 * undone by minimum image) to the grid's J, with the grid's particle shape.
 * If zero_first is non-zero J is cleared first.  J keeps the deposited
 * current for every C^B: the x1 correction of Eq. (correction) is applied
 * where Ampere's law reads J (see pic_advance_E and pic_current_correction).
 * On a 3D grid the (x_old, x) pairs are counting-sorted by the 8^3-cell tile
 * of x_old, and within a tile by its x3 cell plane and pair of x2 cell rows,
 * as a permutation in
 * library scratch (grow-only, 8 bytes of keys and permutation per particle)
 * through which the tile kernel reads them, and each
 * tile's current is summed on chip in 64-bit fixed point whose quantum is
 * set per tile from its particle count, so that no sum can overflow; FP64
 * grids keep two words per node, making each tile's sum exact before one
 * final rounding (see pic_step_n).  The caller's arrays are not reordered.
 * 2D grids deposit each particle with global atomics.  PIC_EUNSUPPORTED for
 * a species of 2^31 or more particles on a 3D grid, and for a 2D grid in the
 * deterministic mode. */
int pic_deposit_J(pic_grid *g, const pic_particles *p, double *const x_old[3], int zero_first);

/* Deposit mode of every later 3D deposit (pic_deposit_J, pic_step_n):
 * PIC_DEPOSIT_ATOMIC (default) or PIC_DEPOSIT_DETERMINISTIC (pic_deposit_mode).
 * The deterministic mode keeps a staging array of 3 (8 + 2m + 3)^3 doubles
 * per tile (m the drift margin of the sort interval; about 103 bytes per
 * cell at the default interval), grow-only; each tile's current is
 * deterministic already (integer sums), and the node sums over the tiles
 * covering a node are taken in a fixed order.  Particles that move faster
 * than c (invalid input) still add through atomics.  PIC_EINVAL for another
 * value. */
int pic_set_deposit_mode(pic_grid *g, int mode);

/* ---- the step loop ----------------------------------------------------------
 * nsteps times: [clear J], for each species gather + push + position update
 * [and charge-conserving deposit], [the x1 current correction when C^B is not
 * the Yee stencil], then the fused field sweep.  No host synchronisation
 * inside; the fields end in the caller's arrays, J holds the last step's
 * deposited current.
 * With deposit on a 3D grid the particles of every species are sorted by
 * spatial tile (8^3 cells), and within a tile by x3 cell plane and pair of x2
 * cell rows, at the first
 * step and then every pic_set_sort_interval steps, and the current of each
 * tile is accumulated in on-chip memory: such calls REORDER the particles
 * (x, u and id together).  Between sorts the particles may sit in the
 * library's second particle set (56 bytes per particle plus 8 bytes of sort
 * keys and permutation, grow-only, PIC_ENOMEM if they cannot be allocated);
 * a call that succeeds returns with them in the caller's arrays (after a
 * failed call their state is unspecified).
 * Vacuum calls and 2D grids keep the order.  A vacuum call on a 3D grid with
 * nsteps >= 2 pushes each species of at least 32768 particles as a copy in
 * library scratch sorted by the same tiles (two copies of 56 bytes per
 * particle plus 4-byte keys, grow-only, PIC_ENOMEM if they cannot be
 * allocated), re-sorted every 16 steps and scattered back to the caller's
 * order at the end: the results equal those of pushing in place, bit for bit. */
int pic_step_n(pic_grid *g, pic_particles *const *species, int nspecies, int nsteps,
               int pusher, int deposit);
/* The on-chip tile current of a 3D deposit (pic_step_n, pic_deposit_J):
 * every Esirkepov contribution is at most |q w| (the particle moves less than
 * c dt), and a node receives at most one per particle of the tile, so with
 * the quantum 2^(e - 61), e = floor(log2(count |q w|)), count the tile's
 * particles, no node sum can exceed 2^62: the 64-bit accumulator cannot
 * overflow for any load; a denser tile only has a coarser quantum.  FP32
 * grids keep one word per node (quantum below 1e-15 |q w| at 8 particles per
 * cell); FP64 grids add a second word holding each contribution's rounding
 * residual, so the tile sum is exact to 2^-(63 - bitlength(count)) of the
 * quantum.  Tile sorts index particles with 32-bit offsets: PIC_EUNSUPPORTED
 * for a species of 2^31 or more particles. */
/* One vacuum step (no deposit) out of place: gather + push + position update
 * of each species at the grid's fields (particles advanced in place), then
 * the fused sweep (Eq. maxwell, App. B operators) from the grid's fields
 * into Eout, Bout (device, same shape and precision, 16-byte aligned, not
 * the grid's own arrays: PIC_EINVAL).  If Bhalf is not NULL, its three
 * arrays (same rules) also receive the half-step field B^{n+1/2} =
 * B^n - dt/2 curl_E E^n.  The grid's fields are not modified.  For callers
 * that keep a sequence of states (e.g. recomputation between adjoint
 * checkpoints) without copying them. */
int pic_step_to(pic_grid *g, pic_particles *const *species, int nspecies, int pusher,
                void *const Eout[3], void *const Bout[3], void *const Bhalf[3]);
/* Steps between particle re-sorts in pic_step_n (1..64, default 3); the
 * on-chip current tile grows with the interval (|v| < c bounds the drift). */
int pic_set_sort_interval(pic_grid *g, int steps);

/* ---- moving window along x1 (Sec. 4.1, the single-particle runs) -----------
 * Moves the window forward (+x1) by ``cells`` whole cells, 0 <= cells < n1
 * (PIC_EINVAL otherwise; 0 does nothing).  The field arrays are a ring along
 * the periodic x1 axis: array column (origin + i) mod n1 holds window cell i,
 * origin starting at 0.  A move clears E and B (and J when attached) in the
 * columns of window cells 0 .. cells-1, which then become the window's last
 * cells (vacuum entering at the front), and adds ``cells`` to the origin; no
 * other field value moves.  Particles keep their (ring) coordinates: window
 * coordinate = (x1 - origin dx1) mod L1, lab coordinate = moved dx1 + window
 * coordinate.  Particles of the given species whose cell column
 * floor(x1/dx1) is one of the cleared columns leave the run: the others are
 * compacted to the front of the caller's arrays in their order (x, u, id
 * together) and species[s]->np is set to their number.  With particles given
 * the call synchronises the stream (the count is needed on the host) and
 * keeps grow-only scratch of 56 bytes per particle; without species it only
 * queues the clearing kernel.  Every other call sees the ring as the periodic
 * mesh it is, so a run with moves equals the run on a physically shifted
 * mesh.  No new plasma is injected at the front. */
int pic_move_window(pic_grid *g, int64_t cells, pic_particles *const *species, int nspecies);
/* The window's ring origin (0 <= origin < n1) and the cells moved so far. */
int pic_window(const pic_grid *g, int64_t *origin, int64_t *moved);

/* ---- absorbing layers at the x1 ends of the window -------------------------
 * The moving-window runs of Sec. 4.1 and 4.2 let light leave through the
 * window's x1 ends; on the ring (periodic) x1 axis it would otherwise
 * re-enter at the other end.  With width W > 0, after every field step
 * (pic_step_n, pic_field_sweep, pic_step_to) the fields in window cells
 * [0, W) and [n1 - W, n1) are multiplied by the graded damping factor of
 * Cerjan et al. (1985), exp(-sigma (d/W)^2), d the depth of each component's
 * own staggered x1 position into the nearest strip (window coordinates, so
 * the strips follow pic_move_window).  J is not damped.  At W = 32 cells of
 * lambda0/32 and sigma = 1 a laser pulse entering a strip leaves less than
 * 1e-9 of its energy reflected.  W = 0 (the default) turns the layers off.
 * PIC_EINVAL unless 0 <= 2W <= n1 and sigma >= 0 is finite; the adjoint
 * step refuses a grid with layers (PIC_EUNSUPPORTED). */
int pic_set_absorber(pic_grid *g, int width, double sigma);

/* ---- adjoint of one vacuum step ---------------------------------------------
 * Reverse mode of one step of pic_step_n without deposit, with the Boris or
 * the exact pusher: gather (App. A) + push (Sec. 1) + position update (Sec. 4.1) of
 * each species, then the field sweep of Eq. maxwell with the App. B
 * operators.  The forward state at t^n is read, not modified: the grid's
 * fields E^n, B^n and species[s] (x^n, u^{n-1/2}).  lambda[s] has the same
 * np; its x and u arrays hold dL/dx^{n+1}, dL/du^{n+1/2} on entry and
 * dL/dx^n, dL/du^{n-1/2} on exit (its q, m, w, id are ignored; in 2D
 * x[2] is left alone, the plane index having no derivative).  adj->lE, lB
 * map dL/d(E,B)^{n+1} to dL/d(E,B)^n, and dL/dC^E_j and dL/dC^B_j (every
 * j < M, also where C_j = 0) are added to adj->gCE, gCB.
 * The field part uses the transposition of the App. B operators
 * (curl_E[C]^T = curl_B[C]).  It needs E^{n+1} and B^{n+1/2}: with adj->En,
 * adj->Bn given (the forward state at t^{n+1}, which must not alias lE, lB
 * or the grid's fields) it uses adj->Bh as B^{n+1/2} if given (as written
 * by pic_step_to), else rebuilds B^{n+1/2} = B^{n+1} + dt/2 curl_E E^{n+1}
 * in the grid's second field set; without En, Bn it first recomputes the
 * forward sweep there.  The position wrap is a constant shift (derivative
 * the identity); at a cell face the shape function has a kink, and the
 * derivative taken is the one of the cell the particle is in.  The exact
 * pusher's proper time tau_r solves t(tau) = dt; its derivative is taken
 * implicitly: d tau_r / d theta = -(d t / d theta at fixed tau) / gamma(tau_r).
 * PIC_EUNSUPPORTED for FP32-field grids and for the Higuera-Cary pusher;
 * PIC_EINVAL for an unknown pusher; the
 * coefficient reduction allocates a scratch of 16 doubles per 1024 cells of
 * 8 x1 rows (32 per 1024 cells of the fused 2D kernel) at the first call
 * (PIC_ENOMEM if that fails).  Scatter into lE, lB uses atomics, so the field
 * cotangents vary in the last bits between runs.
 * With adj->lEo, lBo given (no aliasing of any other array), dL/d(E,B) at t^n
 * go there and lE, lB are left unchanged; on a 2D grid whose C^B has one
 * coefficient (the proposed solver at dt = dx1/2) with En, Bn and Bh given,
 * the three field stages and their dL/dC products then run as one fused pass
 * over the mesh (about a third of the memory traffic of the three in-place
 * stages and their products);
 * in every other case the in-place stages run and their result is copied. */
int pic_adjoint_step(pic_grid *g, const pic_adjoint *adj, const pic_particles *const *species,
                     pic_particles *const *lambda, int nspecies, int pusher);

/* ---- the adjoint step without allocation ------------------------------------
 * For callers that cannot allocate device memory during a step (code under
 * HIP graph capture, tight loops of an optimiser, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as pic_adjoint_step, and
 * the same kernels, but the per-block partial sums of the coefficient
 * gradients live in a fixed device array of the library (1 MiB: 2^17
 * doubles; enough for 8192 reduction blocks of 1024 x1 cells by 8 x1 rows
 * on the in-place path, about 67M cells, and for any mesh on the fused 2D
 * path, whose 256 persistent workgroups need 8192 doubles) instead of grid scratch
 * allocated at the first call; the call makes no hipMalloc, hipFree or other
 * allocating call.  The array's device address is looked up once per device
 * at pic_init_grid.  A mesh needing more partial sums is refused with
 * PIC_EUNSUPPORTED (use pic_adjoint_step).
 * Every grid on one device shares that array and nothing in it needs to
 * start at zero (each call writes the partial sums before it reads them);
 * calls that overlap in time on one device (other streams, other threads)
 * race on it and must be serialised by the caller.  Without adj->En, Bn the
 * step recomputes the forward sweep in the grid's second field set, which
 * pic_init_grid allocated. */
int pic_adjoint_step_noalloc(pic_grid *g, const pic_adjoint *adj, const pic_particles *const *species,
                             pic_particles *const *lambda, int nspecies, int pusher);

/* ---- diagnostics ------------------------------------------------------------
 * Waits for the grid's stream and reports a pending HIP error. */
int pic_sync(pic_grid *g);
/* Scans fields and the given particles for non-finite values and positions
 * outside the periodic box; returns PIC_ENONFINITE if any (synchronous).
 * Then reports, and clears, the grid's count of exact pushes (any call, any
 * species) whose proper-time solve t(tau) = dt ended at the iteration cap
 * instead of converging since the last check: PIC_ENOCONV if non-zero (the
 * pushed momentum of such a particle is not the exact map's). */
int pic_check(pic_grid *g, const pic_particles *p);
/* Iteration cap of the exact pusher's proper-time solve (1..1000, default
 * 100; it converges in 3-12 iterations for fields up to 1e4 at dt = dx1/2).
 * PIC_EINVAL outside the range. */
int pic_set_exact_iterations(pic_grid *g, int max_iter);
/* Effective coefficient widths after trimming (for tests and reports). */
int pic_grid_widths(const pic_grid *g, int *ME, int *MB);
void pic_destroy(pic_grid *g);
const char *pic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* YEEPIC_H */

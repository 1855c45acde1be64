/*
 * pic.h - C ABI of the MI355X (gfx950) hot path of an explicit electromagnetic
 * particle-in-cell step.
 *
 * What a step computes (paper Sec. 2): macro-particles sample the Vlasov
 * equation (eq. 1) through a compact shape g (eq. 2); each step
 *   1. gathers E and B at every particle as the g-weighted average of the grid
 *      fields,
 *   2. advances the momentum with the relativistic Boris rotation and the
 *      position with leap-frog (eq. 3),
 *   3. deposits the current (eq. 4) in the charge-conserving form of
 *      Esirkepov (Comput. Phys. Commun. 135 (2001) 144), so the discrete
 *      continuity equation holds exactly,
 *   4. advances E and B with the two curl equations on the Yee lattice (FDTD).
 *
 * Units (Sec. 2, "suitably normalised"): c = eps0 = 1, charge in units of e,
 * mass in units of m_e, u = p/(m c), v = u/gamma; dE/dt = curl B - J,
 * dB/dt = -curl E.
 *
 * Grid and staggering.  The box has n[0] x n[1] x n[2] cells (n[2] = 1 in 2D),
 * periodic in every dimension, except that the x faces may be open (open_x,
 * below).  Every field component is an array of
 * n[0]*n[1]*n[2] values, x fastest (index i + n0*(j + n1*k)); the entry at
 * (i,j,k) sits at the component's Yee position:
 *   Ex (i+1/2, j, k)     Ey (i, j+1/2, k)     Ez (i, j, k+1/2)
 *   Bx (i, j+1/2, k+1/2) By (i+1/2, j, k+1/2) Bz (i+1/2, j+1/2, k)
 *   Jx, Jy, Jz at the E positions; charge density on nodes (i, j, k).
 * In 2D (dims == 2) nothing varies along z and the k index is dropped.
 * Time levels: positions, E and B at step n; momenta at n-1/2 -> n+1/2;
 * J at n+1/2 (B is advanced in two half steps so that B^n exists).
 *
 * Particles (Sec. 3.3: seven values per particle, positions, momenta, weight,
 * held as separate arrays).  A position is a packed integer cell index plus
 * an offset in [0,1) per dimension: x_d = (cell_d + off_d) * dx_d.  The packed
 * cell is  ix | iy << bx | iz << (bx + by)  with b_d = ceil(log2(n_d)) bits
 * (pic_cell_bits returns them).  Offsets, momenta and weights are float
 * (PIC_FP32) or double (PIC_FP64); so are the fields.  Shapes are B-splines
 * of order 1 (linear) or 2 (quadratic) in cell units.
 *
 * Ownership and streams.  The caller owns every device array (fields,
 * particles, the workspace) and the host structs; the library only borrows
 * pointers for the work it enqueues and never frees them.  Every call
 * enqueues on the given hipStream_t (NULL = default stream) and returns
 * without synchronising, except pic_diagnostics, pic_check and
 * pic_get_timing, which synchronise the stream.  A context is not
 * thread-safe; separate contexts are.
 *
 * Errors.  Every call returns a pic_status and never throws.  Argument errors
 * are found on the host before anything is launched.  HIP errors map to
 * PIC_EHIP with the text kept for pic_last_error.  Conditions found on the
 * device (a particle displaced by a full cell or more in one step, or a
 * non-finite position) set a sticky flag in the workspace that the next
 * pic_check or pic_diagnostics reports; such a particle is left where it was
 * and deposits nothing.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_ABI_VERSION 1

typedef enum {
    PIC_OK = 0,
    PIC_EINVAL = -1, /* bad argument: null pointer, size mismatch, unsupported option */
    PIC_ECFL = -2,   /* dt at or above the Yee limit 1/sqrt(sum_d 1/dx_d^2) */
    PIC_EHIP = -3,   /* HIP runtime error (text in pic_last_error) */
    PIC_ENOMEM = -4, /* no workspace set, or the one set is too small */
    PIC_ECROSS = -5, /* device flag: a particle moved a full cell or more, or became non-finite */
    PIC_ENAN = -6,   /* device flag: a non-finite energy in the diagnostics */
    PIC_ESTATE = -7  /* call out of order, e.g. pic_deposit not preceded by pic_gather_push */
} pic_status;

enum { PIC_FP32 = 0, PIC_FP64 = 1 };

/* Accumulation type of the on-chip current tile of the fused kernel.
 *   FP64: double LDS atomics.
 *   FIX64 (FP32 state only): 64-bit fixed point.  Each contribution, bounded
 *     by |q/dV (dx_d/dt)| w_max (|q|/dA w_max for J_z in 2D) with w_max the
 *     largest |w| among the tile's particles, is scaled by a power of two so
 *     that the bound is at most 2^30, truncated to an integer and added with a
 *     64-bit integer LDS atomic; the merge scales the tile's sums back.  The
 *     truncation is below 2^-30 of the bound per contribution, below the FP32
 *     rounding of the largest contributions.  Integer LDS atomics cost about
 *     half as much as double ones on gfx950 when lanes collide on banks.
 *     w_max is found by the first fused push after each sort of the species
 *     and kept per tile in the workspace for the pushes that follow; a
 *     particle whose |w| has grown past its tile's w_max since then takes the
 *     HBM path (global gather and atomics), so the bound always holds.
 *     Weights that shrink a lot without a sort only coarsen the truncation
 *     relative to the new contributions; sort again after such a change.
 *   FP32: single-precision LDS atomics (accepted for an FP32 state; slow on
 *     gfx950, where the LDS unit serialises them lane by lane).
 *   AUTO (the default): FIX64 for an FP32 state, FP64 for an FP64 state. */
enum { PIC_ACC_AUTO = 0, PIC_ACC_FP32 = 1, PIC_ACC_FP64 = 2, PIC_ACC_FIX64 = 3 };

/* The "grid" element of the paper's object model (Sec. 3.2). */
typedef struct {
    int32_t dims;          /* 2 (2D3V) or 3 (3D3V) */
    int32_t n[3];          /* cells per dimension, each >= 4; n[2] must be 1 when dims == 2 */
    double dx[3];          /* cell sizes (> 0); dx[2] ignored in 2D */
    double dt;             /* time step, 0 < dt < 1/sqrt(sum_d 1/dx_d^2), else PIC_ECFL */
    int32_t shape_order;   /* 1 = linear (cloud in cell), 2 = quadratic */
    int32_t precision;     /* PIC_FP32 or PIC_FP64 */
    int32_t tile[3];       /* cells per sort tile; each divides n[d]; tile[2] = 1 in 2D */
    int32_t slack;         /* guard cells beyond the shape's reach in the LDS tile (0..4):
                              a particle may drift this far out of its tile between sorts
                              and still take the on-chip path */
    int32_t sort_every;    /* pic_step re-sorts every this many steps (>= 1); 0: only species whose
                              sorted flag is 0 (a fixed particle order after the first sort) */
    int64_t max_particles; /* the largest np of any species used with this context */
    int32_t current_accum; /* PIC_ACC_AUTO, PIC_ACC_FP32 (FP32 state only) or PIC_ACC_FP64 */
    /* Open x faces (the paper gives no boundary details, Sec. 2; this is the
     * absorbing boundary of laser-plasma boxes).  0: periodic in x.  1: the
     * node planes i = 0 and i = n[0]-1 are the faces; E_y and E_z on them
     * follow the first-order Mur condition (G. Mur, IEEE Trans. EMC 23 (1981)
     * 377) and y, z stay periodic; a particle whose x cell leaves
     * [absorb, n[0] - absorb) after a move deposits that move's current and
     * is then removed: its weight becomes 0, the fused step skips it, and
     * the next sort moves it behind every tile.  pic_sort then sets the
     * species' np to tile_start[ntiles], the live count (reading it back
     * synchronises the stream); pic_step copies that count to pinned host
     * memory without waiting and drops the removed particles at the
     * species' next sort in a later call or step, once the count has
     * arrived.  Weight-0 particles are always inert when open_x = 1. */
    int32_t open_x;
    int32_t absorb;        /* cells between each x face and the particle region, >= 2 shape_order + 2,
                              and n[0] >= 2 absorb + 2 (open_x only) */
    int32_t sort_levels;   /* levels per tile in the sort: particles sharing a nearest node take
                              distinct levels while they fit (the rest share the last one); 0 means
                              32, else 2..128; about twice the particles per cell suits */
} pic_params;

/* A laser injected as a current sheet on the node plane x = plane dx (open
 * x faces; the paper does not describe its laser source).  At time t the
 * sheet adds to J_y (pol 1) or J_z (pol 2) on that plane
 *   j0 exp(-r^2 / w0^2) exp(-2 ln2 (t - t0)^2 / tau^2) sin(omega (t - t0)),
 * r the distance from the axis (y = yc, z = zc) at each J point, where j0 is
 * chosen so that in the steady state the sheet radiates a plane wave of
 * amplitude e0 to each side on the Yee lattice:
 *   j0 = -e0 dt sin(k dx) / (dx^2 sin(omega dt / 2)),
 *   sin(k dx / 2) = (dx / dt) sin(omega dt / 2),  dx = dx[0].
 * w0 is the 1/e radius of the field, tau the FWHM of the intensity. */
typedef struct {
    int32_t plane;  /* 1 <= plane <= n[0] - 2 */
    int32_t pol;    /* 1: E_y (J_y), 2: E_z (J_z, 3D only) */
    double e0;      /* radiated amplitude, > 0 */
    double omega;   /* angular frequency, below the lattice cut-off */
    double w0;      /* > 0 */
    double tau;     /* > 0 */
    double t0;
    double yc, zc;
} pic_laser;

/* The "em-field" element (Sec. 3.2): E, B and J as nine device arrays of
 * n[0]*n[1]*n[2] float or double values each (layout above).
 *
 * E_alt and B_alt: an optional second set of E and B arrays of the same
 * sizes (all six set, or all null).  With them, in 3D boxes whose n[0] is a
 * multiple of 64 and n[1] a multiple of 8, pic_step and pic_yee_step advance
 * the fields in one pass that reads E^n, B^n, J and writes E^{n+1}, B^{n+1}
 * into the second set, then swap the two sets in this struct (after the
 * call E, B name what were E_alt, B_alt).  Without them, or in other boxes,
 * the Yee step runs in place in three passes.  The other calls read E and
 * B only. */
typedef struct {
    void *E[3];
    void *B[3];
    void *J[3];
    void *E_alt[3];
    void *B_alt[3];
} pic_fields;

/* The "particle" element (Sec. 3.2) for one species (charge q, mass m). */
typedef struct {
    int64_t np;         /* particles in use, 0 <= np <= max_particles */
    double q, m;        /* charge (units of e) and mass (units of m_e), m > 0 */
    int32_t *cell;      /* packed cell index per particle */
    void *off[3];       /* offsets in [0,1) per dimension (off[2] unused in 2D) */
    void *u[3];         /* momentum p/(m c), three components */
    void *w;            /* macro-particle weight (physical particles per macro-particle) */
    /* A second set of arrays of the same sizes.  pic_sort writes the sorted
     * particles into it and then swaps the two sets in this struct, so after a
     * sort the pointers above name what were the *_alt arrays. */
    int32_t *cell_alt;
    void *off_alt[3];
    void *u_alt[3];
    void *w_alt;
    int32_t *tile_start; /* device array of pic_num_tiles()+1 entries, written by pic_sort:
                            particles of tile t are [tile_start[t], tile_start[t+1]) */
    int32_t sorted;      /* set to 1 by pic_sort; the caller sets 0 after it edits particles */
} pic_species;

/* Adjoint (reverse-mode) values of one species: one value per particle and
 * component, in the species' precision.  x[d] is dL/d(position along d in
 * cell units) (x[2] unused in 2D), u[d] is dL/du_d. */
typedef struct {
    void *x[3];
    void *u[3];
} pic_species_adjoint;

typedef struct pic_ctx pic_ctx;

/* Validate the parameters and create a context (host memory only).
 * Returns PIC_EINVAL / PIC_ECFL without creating anything on bad input. */
pic_status pic_init(const pic_params *params, pic_ctx **out);
void pic_destroy(pic_ctx *ctx);

/* Bytes of device workspace the context needs (saved old positions, sort keys,
 * tile counts, diagnostics partials and charge grids).  The caller allocates it
 * (>= 256-byte aligned) and hands it over; it must stay valid while the context
 * is used.  PIC_ENOMEM if bytes is smaller than required. */
size_t pic_workspace_bytes(const pic_ctx *ctx);
pic_status pic_set_workspace(pic_ctx *ctx, void *device_ptr, size_t bytes);

int64_t pic_num_tiles(const pic_ctx *ctx);
void pic_cell_bits(const pic_ctx *ctx, int32_t bits[3]);
/* Bytes of LDS one workgroup of the fused kernel uses (fields + current tile). */
size_t pic_tile_lds_bytes(const pic_ctx *ctx);

/* Steps 1-2 (Sec. 2, eq. 3): gather E^n, B^n at x^n, Boris rotation
 * u^{n-1/2} -> u^{n+1/2}, leap-frog x^n -> x^{n+1}.  x^n is kept in the
 * workspace for the pic_deposit call that must follow for the same species. */
pic_status pic_gather_push(pic_ctx *ctx, pic_species *sp, const pic_fields *f, void *stream);

/* Step 3 (eq. 4 with continuity enforced): J += Esirkepov current of the move
 * recorded by the preceding pic_gather_push of this species.  J is not
 * cleared first (pic_zero_current does that).  PIC_ESTATE if no matching
 * pic_gather_push preceded it. */
pic_status pic_deposit(pic_ctx *ctx, const pic_species *sp, pic_fields *f, void *stream);
pic_status pic_zero_current(pic_ctx *ctx, pic_fields *f, void *stream);

/* Step 4 (Sec. 2, curl equations, Yee FDTD): B^{n+1/2} = B^n - dt/2 curl E^n,
 * E^{n+1} = E^n + dt (curl B^{n+1/2} - J^{n+1/2}), B^{n+1} = B^{n+1/2} - dt/2 curl E^{n+1}.
 * With open_x, E_y and E_z on the two x faces take the Mur update instead. */
pic_status pic_yee_step(pic_ctx *ctx, pic_fields *f, void *stream);

/* Register the laser that pic_step adds to J at t = (step + 1/2) dt of every
 * step (NULL: none; PIC_EINVAL without open_x or for bad parameters). */
pic_status pic_set_laser(pic_ctx *ctx, const pic_laser *laser);
/* Add the registered laser's sheet at time t to J (for callers composing a
 * step from pic_gather_push / pic_deposit / pic_yee_step). */
pic_status pic_laser_current(pic_ctx *ctx, pic_fields *f, double t, void *stream);

/* Bin one species by tile (counting sort by tile index, x-fastest tile
 * numbering); order inside a tile is unspecified.  Writes tile_start, swaps
 * the array sets (see pic_species) and sets sorted = 1.  With open_x it also
 * drops the removed particles (np becomes tile_start[ntiles]) and then
 * synchronises the stream. */
pic_status pic_sort(pic_ctx *ctx, pic_species *sp, void *stream);

/* nsteps whole steps for nspecies species: clear J (and add the laser sheet
 * if one is registered); then, species by species, sort when needed (unsorted
 * species, or every sort_every steps when sort_every > 0) and run the fused
 * gather + push + deposit per tile with fields and current staged on chip
 * (and, with open_x, removal of the particles that left); then the Yee
 * update.  In 3D, after a sort the push reads each particle through the
 * sort's slots and writes it into the second array set, which then becomes
 * the current one: the same swap and tile_start as pic_sort gives.
 * The context keeps state between calls (sorted runs, cached tile weight
 * bounds, which of two counter banks in the workspace the next fused launch
 * takes, its straggler kernel clearing the other): calls on one context run
 * in stream order, one at a time, and a call is not captured into a graph
 * for replay. */
pic_status pic_step(pic_ctx *ctx, pic_species *sp, int32_t nspecies, pic_fields *f, int32_t nsteps, void *stream);

/* FP64 diagnostics of the current state, accumulated in double on the device,
 * synchronising.  out[0..7] =
 *   U_E = 1/2 sum E^2 dV,  U_B = 1/2 sum B^2 dV,  K = sum w m (gamma - 1),
 *   Q = sum q w,  max |rho|,  max |div E - rho|  (the uniform background is
 *   not included), max |G - G_prev| with G = div E - rho from the previous
 *   pic_diagnostics call (NaN if none), and the continuity residual
 *   max |(rho - rho_prev)/dt + div J| when exactly one step separates this
 *   call from the previous one (NaN otherwise). */
#define PIC_NDIAG 8
pic_status pic_diagnostics(pic_ctx *ctx, const pic_species *sp, int32_t nspecies, const pic_fields *f,
                           double *out_host, void *stream);

/* The charge density on the nodes, rho(node) = sum over particles of
 * q w / dV S(x - node) with S the shape of the push (Sec. 2: the densities
 * that the continuity equation ties to J; the uniform neutralising background
 * is not included), accumulated in FP64 into the caller's device array rho of
 * n[0]*n[1]*n[2] doubles (node (i,j,k) at i + n0 (j + n1 k)), which it
 * overwrites.  When gauss is not null it also receives, per node, the
 * residual of Gauss's law div E - rho with the backward-difference
 * divergence from the E points onto the nodes (f must then be valid).  Needs
 * no workspace; enqueues on the stream without synchronising.  PIC_EINVAL for
 * a null rho, bad species, or gauss without fields. */
pic_status pic_charge_density(pic_ctx *ctx, const pic_species *sp, int32_t nspecies, const pic_fields *f,
                              double *rho, double *gauss, void *stream);

/* Allocation-free diagnostics, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the values pic_diagnostics gives on its first call,
 * out[0..5] = U_E, U_B, K, Q, max |rho|, max |div E - rho|, with out[6] and
 * out[7] NaN (no history is kept), synchronising.  Its partial sums, result
 * and charge grid live in a fixed device array of the library (one copy per
 * GPU, held from library load to process exit), so it needs no workspace and
 * calls no allocating routine; grids above PIC_NOALLOC_MAX_CELLS nodes are
 * rejected with PIC_EINVAL.  Every call on one GPU shares that array: calls
 * that overlap on one GPU (other threads, other streams) race and must be
 * serialised by the caller.  Sticky device flags are not read (they live in
 * the workspace; pic_check reports them).  PIC_ENAN for a non-finite energy
 * or charge. */
#define PIC_NOALLOC_MAX_CELLS (1LL << 22)
pic_status pic_diagnostics_noalloc(pic_ctx *ctx, const pic_species *sp, int32_t nspecies, const pic_fields *f,
                                   double *out_host, void *stream);

/* ---- Outputs (Sec. 3.1: reduced-dimension outputs, such as a plane of a 3D
 * box or a line of a 2D one, and subdomain outputs, such as a small box inside
 * a large one; when and how often to write them is the caller's schedule).
 *
 * A box of grid points (or of cells, for particles): along each dimension d
 * the indices lo[d], lo[d] + stride[d], ... below hi[d], with
 * 0 <= lo[d] <= hi[d] <= n[d] and stride[d] >= 1 (in 2D lo[2] = 0, hi[2] = 1).
 * A plane is a box one index thick along one axis, a line one index thick
 * along two; lo[d] == hi[d] selects nothing. */
typedef struct {
    int32_t lo[3];
    int32_t hi[3];
    int32_t stride[3];
} pic_box;

#define PIC_MAX_EXTRACT_GRIDS 16

/* Copy the values of ngrids grids at the points of box into dst, densely
 * packed and bit for bit.  Each grid is a device array laid out as the fields
 * (n[0]*n[1]*n[2] elements, x fastest) of elem_bytes = 4 or 8 bytes: E, B or
 * J components of the state's precision, or FP64 grids such as the charge
 * density of pic_charge_density.  With m_d = ceil((hi[d] - lo[d]) / stride[d])
 * points per axis, grid g's value at the point (a, b, c) of the box (the
 * a-th selected x index, and so on) lands at
 *   dst[((g * m_2 + c) * m_1 + b) * m_0 + a],
 * so dst (device, caller-owned) must hold ngrids * m_0 * m_1 * m_2 elements.
 * Each value keeps its grid's position (the Yee positions above for the field
 * components).  Needs no workspace; enqueues on the stream without
 * synchronising.  PIC_EINVAL for a bad box, elem_bytes, grid count or null
 * pointer. */
pic_status pic_extract_grid(pic_ctx *ctx, const void *const *grids, int32_t ngrids, int32_t elem_bytes,
                            const pic_box *box, void *dst, void *stream);

/* Phase-space records of one species (Sec. 3.1: the particles' phase space
 * output; Sec. 3.3: seven values per particle): the particles whose cell
 * lies in the box of cells (its lo and hi; stride is ignored) and whose
 * storage index is a multiple of every (>= 1, a subsampling of the storage
 * order), with open x faces excluding removed (weight-0) ones.  Each selected
 * particle, in storage order, writes one record of dims + 4 values of the
 * state's precision into dst (device, caller-owned, capacity records):
 *   x_0 .. x_{dims-1}, u_0, u_1, u_2, w,
 * with x_d = (cell_d + off_d) dx_d evaluated in double and rounded once to
 * the state's precision.  *count (a device int64) receives the number
 * selected, also when it exceeds capacity: then only the first capacity
 * records are written.  Uses the workspace (per-chunk counts); enqueues on
 * the stream without synchronising.  PIC_EINVAL for a bad box, every < 1,
 * capacity < 0, a null count, or a null dst with capacity > 0. */
pic_status pic_extract_particles(pic_ctx *ctx, const pic_species *sp, const pic_box *cells, int64_t every,
                                 void *dst, int64_t capacity, int64_t *count, void *stream);

/* ---- Reverse mode (adjoint) of one step, for gradients of a loss of the
 * final fields through K steps (the discrete adjoint of steps 1-4 above).
 *
 * pic_energy_adjoint: lam.E = scale dV E, lam.B = scale dV B (the gradient of
 * scale * (U_E + U_B)); lam.J is not touched.
 *
 * pic_yee_adjoint: maps (lam.E, lam.B) of E^{n+1}, B^{n+1} to those of E^n,
 * B^n through the Yee update (the transpose of pic_yee_step, using
 * C_B = C_E^T), and writes lam.J = dL/dJ^{n+1/2} = -dt (lam.E after the first
 * half).  Call it first for a step.
 *
 * pic_particle_adjoint: for one species given its state at step n (positions
 * x^n, momenta u^{n-1/2}, in the same order as in the forward step, so the
 * rollout must not re-sort between the two) and the fields E^n, B^n: reads
 * lam.J and lsp (dL/dx^{n+1}, dL/du^{n+1/2}), replaces lsp by dL/dx^n,
 * dL/du^{n-1/2}, and adds the transpose of the gather to lam.E and lam.B.
 * Call it after pic_yee_adjoint of the same step, once per species.  When
 * state->tile_start is set (the tile ranges of the last pic_sort of these
 * particles, in this order), it runs per tile with E, B and lam.J staged on
 * chip, provided the tile's boxes fit in LDS; particles further than the
 * slack from their tile, and every particle otherwise, take the HBM path.
 *
 * The adjoint covers periodic boxes only: all three return PIC_EINVAL when
 * open_x is set. */
pic_status pic_energy_adjoint(pic_ctx *ctx, const pic_fields *f, pic_fields *lam, double scale, void *stream);
pic_status pic_yee_adjoint(pic_ctx *ctx, pic_fields *lam, void *stream);
pic_status pic_particle_adjoint(pic_ctx *ctx, const pic_species *state, const pic_fields *f, pic_fields *lam,
                                pic_species_adjoint *lsp, void *stream);

/* Synchronise and report sticky device flags (PIC_ECROSS), then clear them. */
pic_status pic_check(pic_ctx *ctx, void *stream);

/* Per-phase timing with HIP events on the call's stream: when on, pic_step
 * records an event pair around every launch; pic_get_timing synchronises and
 * returns the summed milliseconds and launch counts of each phase, in the
 * order sort, zero_current, push_deposit, yee; then resets them. */
#define PIC_NPHASE 4
pic_status pic_set_timing(pic_ctx *ctx, int32_t on);
pic_status pic_get_timing(pic_ctx *ctx, double *ms, int64_t *launches, int32_t nphase);

/* Number of particles the last fused launch (or tiled adjoint call) handed to the HBM path because
 * their cell was more than `slack` cells outside their tile (synchronising).
 * A large value means the species should be sorted more often. */
pic_status pic_straggler_count(pic_ctx *ctx, int64_t *count, void *stream);

/* Step counter (pic_step and pic_yee_step each count one per step). */
int64_t pic_step_count(const pic_ctx *ctx);

const char *pic_last_error(const pic_ctx *ctx);
const char *pic_status_string(pic_status s);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */

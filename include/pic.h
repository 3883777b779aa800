/*
 * pic.h -- C ABI of the MI355X (gfx950) library for the charge-conserving
 * particle-in-cell step with alternating-order field interpolation
 * (Sokolov, arXiv:1101.0809).
 *
 * One time step (paper Appendix) is: half step of B (Eq. updateB); for every
 * particle, the alternating form factor (order 1 1/2, or 2 1/2) at x^n (Section 4.5),
 * gather of E with the alpha weights (Eq. alphax) and of B with the beta
 * weights (Eq. betax), relativistic momentum advance of the equation of
 * motion Eq. (1) as split in the Appendix (Eq. p2), position advance
 * (Eq. coordscheme), charge-conserving current from the six-box-path
 * average (Eq. current); second half step of B; E update (Eq. escheme).
 *
 * Conventions used by every call
 *   - Units: Gaussian.  Positions are in cell units (x/dx, y/dy, z/dz) and lie
 *     in [0, N) per axis; every axis is periodic.  Momenta are w = gamma v
 *     (momentum over mass), in the same velocity units as c.
 *   - Grid functions are FP64 arrays [k][j][i], i fastest, N = nx*ny*nz
 *     points each, packed in one field buffer as 9 planes:
 *       Ex Ey Ez  at the face centres (i, j+1/2, k+1/2), (i+1/2, j, k+1/2),
 *                 (i+1/2, j+1/2, k)                       (paper Section 2)
 *       Bx By Bz  at the edge midpoints (i+1/2, j, k), (i, j+1/2, k),
 *                 (i, j, k+1/2)
 *       Jx Jy Jz  located like E; J is the current density of Eq. xi.
 *     Between steps the buffer holds E^n, B^{n-1/2} and J = 0.
 *   - Memory: the caller owns every buffer (typically PyTorch tensors on the
 *     GPU) and passes device pointers; sizes come from pic_query_sizes.  The
 *     library keeps borrowed pointers until pic_destroy, never frees them and
 *     performs no device allocation of its own.
 *   - Streams: a stream argument is a hipStream_t passed as void*; NULL is
 *     the null stream.  Calls are asynchronous on that stream unless stated
 *     otherwise.  One context must not be used from two host threads at once.
 *   - Errors: every int-returning call returns PIC_OK (0) or a negative
 *     pic_status; the message is available from pic_last_error.  No C++
 *     exception crosses this interface.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_ctx pic_ctx;

enum pic_status {
    PIC_OK = 0,
    PIC_EINVAL = -1,   /* bad argument (null pointer, size, unsupported option) */
    PIC_ERANGE = -2,   /* particle position outside [0, N) or not finite */
    PIC_ECFL = -3,     /* Courant condition of the staggered leapfrog violated */
    PIC_EDEVICE = -4,  /* a HIP call failed; the HIP error text is in pic_last_error */
    PIC_ESTATE = -5,   /* call not valid in the current state */
    PIC_ESIZE = -6     /* a caller buffer is smaller than pic_query_sizes asks */
};

enum pic_precision {
    PIC_FP64 = 0,  /* particles as FP64 absolute positions; all arithmetic FP64 */
    PIC_FP32C = 1  /* particles as int cell + FP32 offset; gather, push and the
                      current's factors in FP32; each contribution the FP64 product
                      of two FP32 factors (exact), summed in FP64 in the LDS tile;
                      grid and reductions FP64 */
};

enum pic_field_op {
    PIC_B_HALF = 1, /* B <- B - (1/2) curl_h E            (Eq. updateB)          */
    PIC_E_FULL = 2  /* B <- B - (1/2) curl_h E; E <- E - 4 pi dt J + curl_h B; J <- 0
                       (second half of Eq. updateB, then Eq. escheme)             */
};

/* Grid and run description (copied by pic_init_grid). */
typedef struct pic_grid_desc {
    int32_t dims;        /* 3, or 2 for 2D3V (requires nz == 1: nothing depends on z) */
    int32_t nx, ny, nz;  /* cells per axis, >= 1 */
    int32_t precision;   /* enum pic_precision */
    int32_t order;       /* alternating form-factor order l_a = order + 1/2 (Section 4.5):
                            1 (l_a = 1 1/2) or 2 (l_a = 2 1/2: quadratic node and cubic
                            cell factors, 5-cell current window; FP64 only, no adjoint) */
    int32_t sort_every;  /* re-sort particles by cell every this many steps (0: only
                            when loaded) */
    int32_t interp;      /* field interpolation: 0 the alternating-order form factor
                            (Eqs. alphax, betax); 1 the "conventional" uniform order of
                            Eq. wrong1, the comparison of Section 5 (mean of the two
                            adjacent order-1 1/2 cell factors on a component's node axes;
                            order 1 and FP64 only, no adjoint) */
    double dx, dy, dz;   /* cell sizes */
    double dt;           /* time step */
    double c;            /* speed of light */
    double bext[3];      /* uniform external B, added to the gathered B; it is not
                            stored in the field buffer and not in field energies */
    /* Plane-wave source (not part of the paper's method; the laser of the slab
     * workload).  src_kind 0: none.  src_kind 1: an E^y plane wave travelling
     * along +x, injected at the total-field / scattered-field plane between the
     * node x = src_plane and the face x = src_plane + 1/2 (2 <= src_plane <= nx-2).
     * The incident wave is carried by an auxiliary 1D line of PIC_AUX cells with
     * the grid's own staggered operators along x; its E^y point at
     * x = src_plane - 2 + 1/2 is driven as src_amp * ramp(t) * sin(src_omega t),
     * ramp = sin^2(pi t / (2 src_ramp)) for t < src_ramp and 1 after, t = n dt.
     * The line is kept in the last 2 * PIC_AUX doubles of the grid workspace
     * (E^y, then B^z, PIC_AUX each). */
    int32_t src_kind;
    int32_t src_plane;
    double src_amp, src_omega, src_ramp;
    /* Field form.  0: the grid carries B (Eq. updateB).  1: it carries the
     * vector potential A at the E points (Section 4.2, Eq. dadt): each step
     * updates A^{n+1/2} = A^{n-1/2} - c dt E^n and takes B = curl_h A (B^n of
     * A^n for the particles, B^{n+1/2} into the field buffer's B planes, which
     * become outputs: div_h B = 0 holds identically).  A lives in the grid
     * workspace, starts at zero (pic_init_grid sets the B planes to
     * curl_h 0 = 0) and is set and read with pic_set_vector_potential /
     * pic_get_vector_potential.  Not with the plane-wave source or the adjoint. */
    int32_t field_form;
    /* x boundary.  0: periodic (every axis is periodic; the paper's tests are
     * periodic boxes).  1: open -- an extension around the paper's field
     * update, which specifies no boundary.  The walls are the node planes
     * x = 0 and x = nx - 1, on which B^y and B^z lie; each step sets their
     * B^{n+1/2} by Mur's first-order absorbing condition (G. Mur, IEEE Trans.
     * Electromagn. Compat. 23, 377 (1981)),
     *   B_wall^{n+1/2} = B_in^{n-1/2} + k (B_in^{n+1/2} - B_wall^{n-1/2}),
     *   k = (c dt - dx) / (c dt + dx), B_in one cell inside the wall,
     * before the E update reads it.  The cell layer x in [nx - 1, nx) is
     * outside the box: the step sets its E^y, E^z and B^x to zero.  A
     * particle whose step ends within PIC_ABSORB cells of a wall
     * (x < PIC_ABSORB or x >= nx - 1 - PIC_ABSORB) is absorbed: its weight
     * becomes zero once its current of that step is deposited, and it
     * moves on as a particle without charge (pic_get_particles returns it
     * with weight 0; pic_load_particles takes weights > 0 only, so a caller
     * moving particles to another context leaves such ones out).  With 1 the Gauss drift of
     * pic_diagnostics covers cells PIC_ABSORB + 1 .. nx - 3 - PIC_ABSORB along
     * x (those no absorbed charge reaches) and div B the nodes 1 .. nx - 2.
     * Needs nx >= 8, the alternating order 1 1/2 with B carried, and a source
     * plane <= nx - 3; pic_field_solve, pic_solve_poisson and the adjoint
     * reject such a context (their operators are periodic). */
    int32_t xbc;
} pic_grid_desc;

#define PIC_ABSORB 2

#define PIC_AUX 8192

/* Particle species (copied by pic_add_species). */
typedef struct pic_species_desc {
    double q;            /* charge per unit weight (macro charge = q * weight) */
    double m;            /* mass per unit weight */
    int32_t mobile;      /* 0: immobile background charge, deposited once into a
                            fixed density and never pushed; 1: pushed and deposited */
    int32_t reserved;    /* must be 0 */
    int64_t capacity;    /* maximum particle count of this species (below 2^32) */
} pic_species_desc;

typedef struct pic_sizes {
    size_t field_bytes;      /* field buffer: 9 * N FP64 */
    size_t workspace_bytes;  /* grid workspace: background and reference charge,
                                diagnostics, sort histogram */
    size_t particle_bytes;   /* particle buffer for one species of the given capacity
                                (two copies of the particle arrays for out-of-place sorting,
                                sort keys, tile table) */
} pic_sizes;

/* Diagnostics of the state at a step boundary (paper Sections 2, 4.1). */
typedef struct pic_diag {
    int64_t step;            /* steps taken since pic_init_grid */
    int64_t n_particles;     /* mobile particles */
    double kinetic;          /* sum m_p c^2 (gamma^{n-1/2} - 1) over mobile particles */
    double field_e;          /* V/(8 pi) sum E^2 */
    double field_b;          /* V/(8 pi) sum (B^n)^2, B^n = B^{n-1/2} advanced a half
                                step with E^n (external B excluded) */
    double charge;           /* V * sum_cells (rho_mobile + rho_background) */
    double gauss_abs;        /* max_cells |R^n - R^0|, R = div_h E - 4 pi rho */
    double gauss_rel;        /* gauss_abs / max_cells |4 pi rho_mobile^n| */
    double rho_mobile_max;   /* max_cells |4 pi rho_mobile^n| */
    double divb_max;         /* max over nodes of |div_h B^{n-1/2}| */
    int64_t nonfinite;       /* count of non-finite field values and particle momenta */
    double kinetic_half_step; /* sum (q_p dt / 2) u^{n-1/2} . E^n(x^n), E gathered with the
                                 run's interpolation: with kinetic, the particle energy at
                                 t^n of Section 4.1 */
} pic_diag;

/* Buffer sizes for a grid and a particle capacity.  Any pointer in g may be
 * NULL; only the numeric fields are read. */
int pic_query_sizes(const pic_grid_desc* g, int64_t particle_capacity, pic_sizes* out);

/* Validate the grid description and create a context bound to the caller's
 * field buffer (field_bytes from pic_query_sizes; contents are used as the
 * initial E^0, B^{-1/2}; J must be zero) and grid workspace.  Fails with
 * PIC_ECFL unless sum_a (c dt / d_a)^2 < 1 over the axes that have more than one
 * cell (the Courant limit of the staggered leapfrog, Appendix), with
 * PIC_EINVAL for unsupported sizes (FP32 mode: nx, ny <= 2048, nz <= 1024). */
int pic_init_grid(const pic_grid_desc* g, void* fields, size_t field_bytes, void* workspace,
                  size_t workspace_bytes, pic_ctx** out);

/* Register a species and bind its particle buffer (particle_bytes for its
 * capacity; ignored for an immobile species, which may pass NULL and 0).
 * Returns the species index in *species (0, 1, ...; at most 4 species). */
int pic_add_species(pic_ctx* ctx, const pic_species_desc* s, void* buffer, size_t bytes,
                    int* species);

/* Append n particles to a species from device arrays: x [3][n] positions in
 * cell units (the z row is ignored when dims == 2), w [3][n] momentum over
 * mass at t = n - 1/2, weight [n] > 0.  Positions must lie in [0, N) and be
 * finite (else PIC_ERANGE, nothing appended).  Immobile species add their
 * charge density (Eq. rho) to the fixed background instead.  Synchronizes the
 * stream (it checks the positions).  Particles get consecutive ids in load
 * order.  Resets the Gauss reference R^0, which is recaptured before the next
 * step or diagnostics. */
int pic_load_particles(pic_ctx* ctx, int species, int64_t n, const double* x, const double* w,
                       const double* weight, void* stream);

/* Advance nsteps full time steps (Appendix order).  Asynchronous. */
int pic_step(pic_ctx* ctx, int nsteps, void* stream);

/* Current of n particles moving from x0 to x1 (device arrays [3][n] in cell
 * units; x1 need not be wrapped but |x1 - x0| < 1 per axis is required) with
 * macro charges charge[n], added into J_out (device, 3 * N FP64 in the Jx Jy Jz
 * layout of the field buffer).  Uses the same per-particle deposit code as
 * pic_step in the context's precision (FP32 mode converts the positions to
 * cell + FP32 offset first); the sums go through global atomics.  Eq. current,
 * Eq. xi.  Asynchronous. */
int pic_deposit_J(pic_ctx* ctx, const double* x0, const double* x1, const double* charge,
                  int64_t n, double* J_out, void* stream);

/* One field operation on the bound fields (enum pic_field_op).  Asynchronous. */
int pic_field_solve(pic_ctx* ctx, int what, void* stream);

/* Compute pic_diag in FP64 on the GPU.  Synchronizes the stream. */
int pic_diagnostics(pic_ctx* ctx, pic_diag* out, void* stream);

/* pic_diagnostics for callers that cannot allocate device memory or take a
 * workspace of their own: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation.  Same results and errors as
 * pic_diagnostics, but its scratch (the mobile charge density, N FP64, and
 * the reduction partials) lives in a fixed static device array of the
 * library (20 MiB per GPU, held until the process ends) instead of the
 * context's workspace; no allocation is made.  Grids of more than about
 * 2.57 million cells are rejected with PIC_ESIZE.  Every call on one GPU
 * uses that GPU's array, so calls that overlap on one GPU (other streams,
 * other host threads) race and must be serialized by the caller.  Like
 * pic_diagnostics it may capture the Gauss reference R^0 into the context
 * first.  Synchronizes the stream. */
int pic_diagnostics_static(pic_ctx* ctx, pic_diag* out, void* stream);

/* Adjoint (reverse-mode derivative) of the time step, for gradients of a
 * loss with respect to the initial momenta and the external field (FP64 mode,
 * no plane-wave source; PIC_EINVAL otherwise).  An adjoint field buffer holds
 * 6 planes of N FP64 in the layout of the field buffer's first six (dL/dE then
 * dL/dB); a particle adjoint holds [3][count] FP64 indexed by particle id
 * (load order), dL/dx (cell units) and dL/dw.  The caller owns all of them.
 *
 * pic_adjoint_seed_field_energy: write into lam_fields the derivative of the
 * field energy V/(8 pi) sum E^2 + (B^n)^2 of the current state (E^n,
 * B^{n-1/2}; B^n advanced a half step, Section 4.1) with respect to E^n and
 * B^{n-1/2}.  Asynchronous.
 *
 * pic_adjoint_step: the context must hold the state a step was taken from
 * (E^n, B^{n-1/2}, x^n, w^{n-1/2}), e.g. restored from a copy of its buffers
 * and pic_set_host_state; it is not changed (the workspace is).  On entry
 * lam_fields, lam_x[s], lam_w[s] hold the adjoint of the state after the step
 * (E^{n+1}, B^{n+1/2}, x^{n+1}, w^{n+1/2}); on return the adjoint of the state
 * before it, by the chain rule through the Appendix step: both B half steps
 * (Eq. updateB), gather (Eqs. alphax, betax), push (Eq. p2), position advance
 * (Eq. coordscheme), current (Eq. current) and E update (Eq. escheme).  The
 * derivative of the loss with respect to the uniform external field is added
 * into lam_bext[3].  lam_x and lam_w are host arrays with one device pointer
 * per species (ignored for immobile species).  Asynchronous. */
int pic_adjoint_seed_field_energy(pic_ctx* ctx, double* lam_fields, void* stream);
int pic_adjoint_step(pic_ctx* ctx, double* lam_fields, double* const* lam_x, double* const* lam_w,
                     double* lam_bext, void* stream);

/* Records for a reverse sweep without restoring the context.  A record holds
 * what one reverse step reads of the state a step starts from: E^n and
 * B^{n-1/2} (6 N FP64) and, per mobile species, its particles in the
 * library's storage order (positions, momenta, weights, ids) with the tile
 * table of its last sort, in a layout private to the library.
 *
 * pic_adjoint_record_bytes: size of one record for the context's current
 * particle counts (PIC_EINVAL on a null argument).
 * pic_adjoint_record: copy the context's current state into record (caller-
 * owned device memory of at least that size; PIC_ESIZE if smaller).  Taken
 * before each pic_step(ctx, 1) of a forward pass, the records are the tape of
 * that pass.  Asynchronous.
 * pic_adjoint_step_record: pic_adjoint_step with the state before the step
 * read from a record written on this context while its particle counts were
 * what they are now; the context's fields and particles are not read (its
 * workspace is used).  Same adjoint arguments and errors as pic_adjoint_step,
 * plus PIC_ESIZE for a record smaller than pic_adjoint_record_bytes. */
int pic_adjoint_record_bytes(const pic_ctx* ctx, size_t* bytes);
int pic_adjoint_record(pic_ctx* ctx, void* record, size_t bytes, void* stream);
int pic_adjoint_step_record(pic_ctx* ctx, const void* record, size_t bytes, double* lam_fields,
                            double* const* lam_x, double* const* lam_w, double* lam_bext, void* stream);

/* Particle adjoints in storage order.  Reading them by id costs a scattered
 * access per particle; a reverse sweep can keep them in the order of the
 * particles in its records instead, which stays the same between sorts.
 *
 * pic_adjoint_step_record_ordered: pic_adjoint_step_record with lam_x[s],
 * lam_w[s] ([3][n] FP64) indexed by the particle's position in the record.
 * pic_adjoint_reorder: out[k] = in[position, in the order of record `from`,
 * of the particle at position k in the order of record `to`], per species;
 * a NULL record stands for id order.  A sweep calls it across every step that
 * sorted (pic_sort, a first step after loading, or a periodic sort: the host
 * state tells), and once at the end to return to id order.  Out of place
 * (PIC_EINVAL if an output aliases an input); bytes is the size of the
 * records (PIC_ESIZE if smaller than pic_adjoint_record_bytes, unused when
 * both are NULL).  Uses the species' sort scratch in its particle buffer.
 * Asynchronous. */
int pic_adjoint_step_record_ordered(pic_ctx* ctx, const void* record, size_t bytes, double* lam_fields,
                                    double* const* lam_x, double* const* lam_w, double* lam_bext, void* stream);
int pic_adjoint_reorder(pic_ctx* ctx, const void* from, const void* to, size_t bytes,
                        const double* const* in_x, const double* const* in_w, double* const* out_x,
                        double* const* out_w, void* stream);

/* Electrostatic field of the current charge (Section 4.3): solve the
 * discrete Poisson equation of Eq. poiphi on the periodic grid for the
 * cell-centred potential of the total charge density (mobile species plus the
 * immobile background) and set E = -grad_h Phi (Eq. egradphidis), so that
 * div_h E = 4 pi rho cell by cell; B is left as it is.  The periodic problem
 * needs a neutral total: the mean charge density is removed from the right
 * side, and with neutralize = 1 it is also added, with the opposite sign, to
 * the background as a uniform charge (the uniform neutralizing background of
 * a start without co-located ions).  Conjugate gradients on the GPU to a
 * relative residual tol (<= 0: 1e-13); *iterations and *residual (either may
 * be NULL) report the count and the reached relative residual.  The Gauss
 * reference R^0 is recaptured before the next step.  Synchronizes the
 * stream.  PIC_ESTATE if the tolerance was not reached. */
int pic_solve_poisson(pic_ctx* ctx, int neutralize, double tol, int64_t* iterations, double* residual,
                      void* stream);

/* Vector-potential form (field_form 1): pic_set_vector_potential copies A
 * (3 N FP64 device array, the layout of E: A^x at (i, j+1/2, k+1/2), ...)
 * as A^{n-1/2} of the current state and sets the B planes to curl_h A;
 * pic_get_vector_potential copies A^{n-1/2} out.  PIC_ESTATE in field form 0.
 * Asynchronous. */
int pic_set_vector_potential(pic_ctx* ctx, const double* A, void* stream);
int pic_get_vector_potential(pic_ctx* ctx, double* A, void* stream);

/* Number of particles currently held by a species (host-side count). */
int64_t pic_particle_count(const pic_ctx* ctx, int species);

/* Copy a species out as FP64 device arrays (capacity >= count): x [3][n],
 * w [3][n], weight [n], id [n] (any of them may be NULL).  The order is the
 * library's current (cell-sorted) order; ids identify particles.
 * Asynchronous. */
int pic_get_particles(pic_ctx* ctx, int species, double* x, double* w, double* weight,
                      int64_t* id, void* stream);

/* Sort every mobile species by cell now (counting sort, out of place).
 * Asynchronous. */
int pic_sort(pic_ctx* ctx, void* stream);

/* Tuning of the particle-step kernel: fraction of particle updates that took
 * the global-memory path (grid gathers and global atomics) during the last
 * pic_step call, or -1 if not recorded.  Synchronizes the stream. */
double pic_last_fallback_fraction(pic_ctx* ctx, void* stream);

/* Tuning of the 3D particle step: fraction of particle updates during the
 * last pic_step call that were made by the migrant pass (particles found
 * outside their sorted tile's region -- more than one cell off the tile, or
 * in FP32 mode more than two along x -- and advanced with the LDS tiles of
 * the tile that holds them now), or -1 if not recorded.  Synchronizes the
 * stream. */
double pic_last_migrant_fraction(pic_ctx* ctx, void* stream);

/* Per-phase timing with HIP events recorded on the stream of each pic_step
 * (a profiling aid; events only, no device memory).  pic_timing_start begins
 * recording the next max_steps steps (earlier records are dropped).
 * pic_timing_stop waits for the recorded events and returns the summed
 * durations in milliseconds of the phases of those steps:
 *   ms[0] B half step, ms[1] particle kernels, ms[2] second B half step and E
 *   update, ms[3] periodic sorts;  *steps = number of steps recorded. */
int pic_timing_start(pic_ctx* ctx, int max_steps);
int pic_timing_stop(pic_ctx* ctx, double ms[4], int64_t* steps);

/* Host-side state of a context: everything that is not in the caller's
 * buffers.  A checkpoint is the field buffer, the grid workspace, every
 * particle buffer (byte copies) and this struct; restoring copies the buffers
 * into a context created with the same descriptions and then sets the
 * struct.  Synchronizes nothing. */
typedef struct pic_host_state {
    int64_t step;          /* steps taken */
    int32_t since_sort;    /* steps since the last sort */
    int32_t r0_valid;      /* Gauss reference R^0 captured in the workspace */
    int32_t nsp;           /* species registered */
    int32_t reserved;
    int64_t n[4];          /* particles per species */
    int32_t sorted[4];     /* species sorted since its last load */
    int32_t copy[4];       /* which of the two particle-array copies is current */
} pic_host_state;

int pic_get_host_state(const pic_ctx* ctx, pic_host_state* out);
/* Fails with PIC_ESTATE unless the context has the same species count and each
 * count fits its capacity. */
int pic_set_host_state(pic_ctx* ctx, const pic_host_state* in);

/* Destroy a context (does not free caller buffers). */
void pic_destroy(pic_ctx* ctx);

/* Last error message of a context (never NULL; "" if none).  With ctx == NULL,
 * the last error of a failed pic_init_grid / pic_query_sizes in this thread. */
const char* pic_last_error(const pic_ctx* ctx);

/* Version string of the library build. */
const char* pic_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */

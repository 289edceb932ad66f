/*
 * misa.h -- C ABI of the MI355X EAM lattice molecular-dynamics library.
 *
 * The library implements the hot path of MISA-MD (Chu, Li et al., "MD
 * Simulation of Hundred-Billion-Metal-Atom Cascade Collision on Sunway
 * Taihulight"): EAM forces over a lattice-indexed atom store (the Lattice
 * List of Sec. 3 with its Neighbor Offset Index), atoms that leave their
 * lattice sites (the hash-clash atoms of Algorithms 1 and 2), interpolated
 * potential tables (Sec. 4.1) and the MD time loop of Sec. 2.1.
 *
 * Conventions (every entry point):
 *   - Returns MISA_OK (0) or a negative MISA_E* code; no exception crosses the
 *     ABI.  misa_last_error() gives a readable message for the last failure
 *     on a handle.
 *   - Units: Angstrom, eV, fs, amu.  Positions and velocities are float64,
 *     row-major (N, 3) arrays, indexed by atom id 0 .. N-1.
 *   - "where" arguments: MISA_HOST for host memory, MISA_DEVICE for device
 *     memory of the handle's GPU.
 *   - All GPU work is enqueued on the HIP stream given at creation; calls that
 *     return data to host memory synchronise that stream.  A handle is not
 *     thread safe.
 *   - State memory (lattice slots and run-away atoms) is owned by the caller:
 *     query misa_state_bytes(), allocate that many bytes of device memory
 *     (256-byte aligned) and pass it to misa_bind_state().  The library never
 *     frees it; it must stay valid until the handle is destroyed or rebound.
 *     Tables, the neighbour stencil and scratch (hash, counters, partial
 *     sums) are allocated and freed by the library.
 */
#ifndef MISA_H
#define MISA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MISA_OK 0
#define MISA_EINVAL -1     /* bad argument or descriptor */
#define MISA_ENOMEM -2     /* device or host allocation failed */
#define MISA_EHIP -3       /* a HIP runtime call failed (message kept) */
#define MISA_ESTATE -4     /* call made out of order (no tables, no state, ...) */
#define MISA_EOVERFLOW -5  /* more atoms left their sites than the run-away capacity holds */

#define MISA_FP64 0 /* pair arithmetic in float64 */
#define MISA_FP32 1 /* pair arithmetic in float32; positions, velocities, integration, energies float64 */

#define MISA_HOST 0
#define MISA_DEVICE 1

/* per-atom fields for misa_get_atom_field */
#define MISA_FIELD_RHO 0    /* electron density rho_i (1 value per atom) */
#define MISA_FIELD_FPRIME 1 /* F'(rho_i) (1 value per atom) */
#define MISA_FIELD_FORCE 2  /* force F_i (3 values per atom) */

/* what for misa_debug_export */
#define MISA_EXPORT_STENCIL 0 /* int64 [2][K][3] lattice-id offsets (dX, dY, dZ) per parity; returns K */
#define MISA_EXPORT_SLOTS 1   /* int64 [N] lattice id holding each atom, -1 for run-away atoms; returns N */

typedef struct misa_lattice misa_lattice;

/*
 * Box and method parameters.  The box is n_cells[0] x n_cells[1] x n_cells[2]
 * cubic BCC cells, periodic on all axes.  Lattice ids follow Sec. 3 (Hash
 * Initialization): id = 2 nx ny Z + 2 nx Y + X with X in [0, 2 nx), odd X
 * the body-centre sites.
 */
typedef struct {
    int32_t n_cells[3];
    int32_t pair_precision;   /* MISA_FP64 or MISA_FP32 */
    double a;                 /* lattice constant, > 0 */
    double rc;                /* cut-off radius, > 0 */
    double delta;             /* slot tolerance: an atom keeps its lattice slot while |x - site| <= delta;
                                 0 < delta < a sqrt(3) / 4 (half the nearest-neighbour distance) */
    double mass;              /* atom mass, > 0 */
    int64_t runaway_capacity; /* max atoms outside the lattice array; <= 0 picks max(16384, sites / 128) */
} misa_lattice_desc;

/* Equidistant samples y[k] = g(x0 + k dx), k = 0 .. n - 1 (host memory; copied, not retained). */
typedef struct {
    double x0;
    double dx;
    int32_t n;
    int32_t reserved;
    const double *y;
} misa_table;

/* Statistics of the last step of a misa_step call. */
typedef struct {
    double dt;          /* length of the last step [fs] */
    double dt_next;     /* length the next step will take [fs] */
    double vmax;        /* max |v| after the last step [A/fs] */
    double e_kin;       /* kinetic energy after the last step [eV] */
    double e_emb;       /* sum_i F(rho_i) [eV] */
    double e_pair;      /* 1/2 sum_i sum_{j != i} phi(r_ij) [eV] */
    double time;        /* accumulated simulated time [fs] */
    int64_t steps;      /* accumulated steps on this handle */
    int64_t n_runaway;  /* atoms outside the lattice array */
    int64_t range_violations; /* densities beyond the embedding table (linearly extrapolated) */
    int32_t overflow;   /* 1 if the run-away capacity was exceeded (forces inexact since) */
    int32_t reserved;
} misa_step_stats;

/*
 * Create a lattice handle: validates the descriptor, builds the lattice-id
 * map and the two per-parity Neighbor Offset Index stencils (Sec. 3: offsets
 * of all sites closer than rc + 2 delta to a site, so every pair of slotted
 * atoms within rc is found) and allocates scratch on the current HIP device.
 * Requires n_cells[i] * a > 2 (rc + 2 delta) so that no stencil offset wraps
 * onto another one.  hip_stream: a hipStream_t (NULL = default stream).
 * On success *out owns the handle (free with misa_destroy_lattice).
 */
int misa_create_lattice(const misa_lattice_desc *desc, void *hip_stream, misa_lattice **out);

/* Release everything the library allocated for h (not the bound state buffer). */
int misa_destroy_lattice(misa_lattice *h);

/* Message of the last failed call on h (static string when h is NULL). */
const char *misa_last_error(const misa_lattice *h);

/* Bytes of caller-owned device memory misa_bind_state needs. */
int misa_state_bytes(const misa_lattice *h, int64_t *bytes);

/* Use `bytes` bytes of device memory at device_ptr (256-byte aligned) as the
 * atom store: lattice slots (displacement, velocity, force, rho, F', atom id per
 * site) and run-away atoms.  Invalidates any previous state. */
int misa_bind_state(misa_lattice *h, void *device_ptr, int64_t bytes);

/*
 * Potential tables (Sec. 4.1): f (electron density contribution of a
 * neighbour at distance r), phi (pair potential) and F (embedding energy).
 * Each is interpolated per segment by a cubic Hermite polynomial whose node
 * slopes are fourth-order central differences of the samples (second-order /
 * one-sided at the two nodes nearest each end), with linear continuation
 * beyond the last node.  Requirements: n >= 8, dx > 0; the f and phi grids
 * must start at or below 0 and reach rc.  Builds float64 and float32
 * coefficient records on the device.
 */
int misa_set_potential_tables(misa_lattice *h, const misa_table *f, const misa_table *phi,
                              const misa_table *emb);

/*
 * Load n_atoms atoms (positions x, velocities v; (n_atoms, 3) float64; atom
 * id = row index) from host or device memory.  Each atom goes to the slot of
 * its nearest site (the hash of Sec. 3) if it lies within delta of it; the
 * lowest atom id wins a contested slot; every other atom becomes a run-away
 * (hash-clash) atom.  Fails with MISA_EOVERFLOW if those exceed the run-away
 * capacity.  Invalidates densities and forces.  Requires a bound state.
 */
int misa_set_state(misa_lattice *h, const double *x, const double *v, int64_t n_atoms, int where);

/* Copy positions (wrapped into the box) and velocities out, in atom-id order,
 * to (n_atoms, 3) float64 arrays in host or device memory; either may be NULL. */
int misa_get_state(misa_lattice *h, double *x, double *v, int where);

/* Number of atoms loaded by the last misa_set_state. */
int misa_atom_count(const misa_lattice *h, int64_t *n_atoms);

/*
 * Electron densities rho_i = sum_{j != i, r_ij < rc} f(r_ij) and embedding
 * derivatives F'(rho_i) of every atom (Sec. 2.2, steps 1-2): the lattice
 * gather over the stencil, the run-away atoms' own sums and their
 * contributions to nearby lattice atoms.  Asynchronous.  Requires tables and state.
 */
int misa_compute_rho(misa_lattice *h);

/*
 * Forces F_i = sum_j [(F'_i + F'_j) f'(r_ij) + phi'(r_ij)] (x_j - x_i) / r_ij
 * (Sec. 2.2, Eq. eam_force_ij, steps 3-5) for every atom.  If energies_dev is
 * not NULL it receives, in device memory, [sum_i F(rho_i), 1/2 sum_i sum_{j!=i}
 * phi(r_ij)].  Requires misa_compute_rho on the same state (MISA_ESTATE
 * otherwise).  Asynchronous.
 */
int misa_compute_force(misa_lattice *h, double *energies_dev);

/*
 * nsteps velocity-Verlet steps (the time loop of Sec. 2.1, Fig. 1, in
 * kick-drift-kick form) with the hash update of Algorithm 2 after each drift.
 * Step length dt = min(dt_max, dx_max / max_i |v_i|) taken at the start of
 * each step; dx_max <= 0 fixes dt = dt_max.  Computes forces first if they
 * are not valid for the current state.  stats (host memory, may be NULL)
 * receives the statistics of the last step (synchronises the stream).
 * Returns MISA_EOVERFLOW (after finishing the steps) if the run-away capacity
 * was exceeded: atoms that could not leave their slots stayed, so forces on
 * them are inexact from then on.
 */
int misa_step(misa_lattice *h, int64_t nsteps, double dt_max, double dx_max, misa_step_stats *stats);

/* Kernel classes timed by misa_set_timing. */
#define MISA_TIMER_RHO 0     /* lattice rho pass (one launch per step) */
#define MISA_TIMER_FORCE 1   /* lattice force pass (one launch per step) */
#define MISA_TIMER_KICK 2    /* kick-drift and final kick of the integrator */
#define MISA_TIMER_RUNAWAY 3 /* hash update, device hash and run-away interactions */
#define MISA_TIMER_OTHER 4   /* step length, energy sums */
#define MISA_TIMER_COUNT 5

typedef struct {
    double ms[MISA_TIMER_COUNT];        /* summed GPU time per class [ms] */
    int64_t launches[MISA_TIMER_COUNT]; /* timed launch groups per class */
} misa_timing;

/* enable != 0: record HIP events on the handle's stream around every kernel
 * group of compute/step calls (profiling; a few microseconds per step).
 * Resets the accumulated times. */
int misa_set_timing(misa_lattice *h, int enable);

/* Accumulated times since misa_set_timing (synchronises the stream). */
int misa_get_timing(misa_lattice *h, misa_timing *out);

/* Per-atom rho, F' or force, in atom-id order, to float64 memory (n_atoms or
 * 3 n_atoms values).  Values are those of the last compute/step. */
int misa_get_atom_field(misa_lattice *h, int field, double *out, int where);

/* Parity and debugging exports to host memory (see MISA_EXPORT_*); capacity
 * counts int64 elements; the return value is the element count (K or N) or a
 * negative error code. */
int64_t misa_debug_export(misa_lattice *h, int what, int64_t *host_out, int64_t capacity);

#ifdef __cplusplus
}
#endif

#endif /* MISA_H */

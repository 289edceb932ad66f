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
#define MISA_EXPORT_NEIGHBOURS 2 /* int64 [N] per atom: partners within rc as the density pass of the
                                    handle's form counts them (Sec. 2.2 step 1; table forms); returns N */

typedef struct misa_lattice misa_lattice;

/*
 * Box and method parameters.  The box is n_cells[0] x n_cells[1] x n_cells[2]
 * cubic BCC cells, periodic on all axes.  Lattice ids follow Sec. 3 (Hash
 * Initialization): id = 2 nx ny Z + 2 nx Y + X with X in [0, 2 nx), odd X
 * the body-centre sites.
 */
typedef struct {
    int32_t n_cells[3];
    int32_t pair_precision;   /* MISA_FP64, MISA_FP32 or MISA_MLP (below) */
    double a;                 /* lattice constant, > 0 */
    double rc;                /* cut-off radius, > 0 */
    double delta;             /* slot tolerance: an atom keeps its lattice slot while |x - site| <= delta;
                                 0 < delta < a sqrt(3) / 4 (half the nearest-neighbour distance) */
    double mass;              /* atom mass, > 0 */
    int64_t runaway_capacity; /* max atoms outside the lattice array; <= 0 picks max(16384, sites / 1024) */
    int32_t periodic[3];      /* boundary per axis: 1 (or 0, the default) = periodic; the lattice store wraps
                                 every axis (Sec. 3 ghost regions), so other values are rejected */
    int32_t ntypes;           /* atom species: 1 (or 0, the default); one set of f, phi, F tables (Sec. 2.2) */
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
    int32_t overflow;   /* 1 if a step's leavers exceeded the run-away capacity (misa_step: MISA_EOVERFLOW) */
    int32_t failed_step; /* with overflow: index in the call (0-based) of that step; -1 otherwise */
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
 * (hash-clash) atom, listed in ascending id.  The placement runs on the GPU
 * (host arrays are uploaded to temporary device memory first; device arrays must
 * be ready in the handle's stream order); the call synchronises the stream.
 * Fails with MISA_EINVAL on a non-finite value and with MISA_EOVERFLOW if the
 * run-away atoms exceed the run-away capacity; after a failure no state is
 * loaded.  Invalidates densities and forces.  Requires a bound state.
 */
int misa_set_state(misa_lattice *h, const double *x, const double *v, int64_t n_atoms, int where);

/*
 * misa_set_state for callers that cannot allocate device memory (serving loops
 * that reload states, harnesses that forbid allocation): the same placement from
 * device arrays x, v ((n_atoms, 3) float64, device memory of the handle's GPU)
 * with no hipMalloc or hipFree.  Its scratch (one bid per atom and a counter) is a
 * static array of MISA_NOALLOC_MAX_ATOMS + 64 words of device memory on every GPU
 * the library runs on, held until the process ends; MISA_EINVAL for more atoms
 * than MISA_NOALLOC_MAX_ATOMS.  The array is shared by every handle on a GPU and
 * keeps the last call's contents: calls that overlap on one GPU (two host
 * threads, or handles on streams that run concurrently) race.  Synchronises the
 * stream; results and errors are those of misa_set_state.
 */
#define MISA_NOALLOC_MAX_ATOMS 4194304 /* 16 MiB of bids per GPU */
int misa_set_state_noalloc(misa_lattice *h, const double *x, const double *v, int64_t n_atoms);

/*
 * misa_set_state with explicit atom ids (Sec. 2.1: the problem starts from every
 * atom's position and velocity; the ids name the atoms): row i of the host arrays
 * x, v ((n_atoms, 3) float64) belongs to atom ids[i] (host int64).  The ids must be
 * a permutation of 0 .. n_atoms - 1, else MISA_EINVAL before anything is loaded.
 * The placement, its id priority and its errors are those of misa_set_state with
 * the rows in id order; misa_get_state returns the atoms in id order.
 */
int misa_set_state_ids(misa_lattice *h, const double *x, const double *v, const int64_t *ids, int64_t n_atoms);

/* Copy positions (wrapped into the box) and velocities out, in atom-id order,
 * to (n_atoms, 3) float64 arrays in host or device memory; either may be NULL. */
int misa_get_state(misa_lattice *h, double *x, double *v, int where);

/*
 * Checkpoint and resume.  misa_save_checkpoint copies the handle's whole state
 * (lattice slots with both copies of u and v, forces, densities, slot ids, the
 * run-away list, the step counters, the time and the step length) and a
 * description of the lattice into misa_checkpoint_bytes() bytes of host memory;
 * misa_load_checkpoint puts it into a handle created with the same descriptor,
 * bound to a state buffer and given the same potential tables (MISA_EINVAL
 * otherwise).  Stepping on after a load is bit for bit what stepping on the saved
 * handle would have given.  (misa_get_state / misa_set_state move atoms between
 * boxes and representations: positions travel as absolute coordinates, so the
 * site-relative displacements come back within rounding, not bit for bit.)
 * Both synchronise the stream.
 */
int misa_checkpoint_bytes(const misa_lattice *h, int64_t *bytes);
int misa_save_checkpoint(misa_lattice *h, void *host_out, int64_t bytes);
int misa_load_checkpoint(misa_lattice *h, const void *host_in, int64_t bytes);

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
 * receives the statistics of the last step.  Synchronises the stream at the end.
 * MISA_EOVERFLOW if a step's leavers (atoms farther than delta from their
 * sites) do not fit in the run-away capacity: that step is undone and the call
 * ends with the state (positions, velocities, slots, run-away atoms, forces,
 * densities, time) exactly as at the start of the failing step; the later
 * steps of the call ran without advancing it.  stats->failed_step says which
 * step failed, stats->steps counts the steps completed.  The caller can read the
 * state out and load it into a handle with a larger capacity.
 *
 * The bound state buffer holds two copies of the displacements and velocities:
 * each step's kick-drift reads one and writes the other (misa_get_state and the
 * other calls always see the current one).
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

/* enable != 0: misa_step replays one captured HIP graph of a step for all its
 * steps but the last, instead of launching the ~20 kernels of each step one by
 * one (the gain is the launch overhead: large for small boxes, small for big
 * ones).  Results are bit-identical to the launched steps.  The graph is captured
 * on first use for the call's (dt_max, dx_max) and captured again when those
 * change or after misa_set_potential_tables, misa_bind_state,
 * misa_set_pair_schedule or misa_set_mlp.  Not used while timing is enabled. */
int misa_set_graph(misa_lattice *h, int enable);

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
 * negative error code.  MISA_EXPORT_NEIGHBOURS runs the handle's own density pass
 * (lattice gather, run-away atoms and their reaction terms) with f = 1 inside rc,
 * so each count is the pair set that pass takes for the current state; it needs
 * tables and state; afterwards the handle is as before (the tables are rebuilt,
 * densities and F' computed again if they were valid, forces untouched); it
 * synchronises the stream.
 * MISA_EINVAL on a MISA_MLP handle. */
int64_t misa_debug_export(misa_lattice *h, int what, int64_t *host_out, int64_t capacity);

/* Pair schedule of the float32 table form (pair_precision MISA_FP32).
 *
 * MISA_PAIRS_GATHER (the default): every atom sums its pairs from its own side,
 * so each pair is evaluated from both ends; no two threads write one atom.
 * MISA_PAIRS_HALF: Newton's third law (Sec. 4.2): each unordered pair is
 * evaluated once, by the end whose lattice offset to the other points into the
 * forward half space, and its terms go to both atoms.  The write conflicts that
 * creates are resolved by the colouring idea of Sec. 4.2: tiles are 2-coloured
 * per axis and run one colour at a time, and inside a tile the partner writes
 * run in phases that no two waves share, so the result is deterministic.  It
 * needs every axis to be a multiple of 16 cells (MISA_EINVAL otherwise, or for
 * a MISA_FP64 handle).  It serves the float32 table form and the learned form
 * (MISA_MLP: each owned pair goes through the networks once instead of twice).
 * Forces agree with the gather schedule to float32 rounding, not bit for bit.
 * Batched replicas always gather. */
#define MISA_PAIRS_GATHER 0
#define MISA_PAIRS_HALF 1
int misa_set_pair_schedule(misa_lattice *h, int schedule);

/* Wigner-Seitz defect count of the current state (the direct defect analysis
 * the paper names in Sec. 1 and applies to cascades in Sec. 5.1): every atom
 * belongs to the cell of its nearest lattice site (the hash rule); a site whose
 * cell is empty is a vacancy, every atom beyond the first in a cell an
 * interstitial.  counts (host int64[4]): vacancies, interstitials, run-away
 * atoms, empty slots.  Uses the handle's sort scratch; synchronises the stream. */
int misa_defects(misa_lattice *h, int64_t *counts);

/* ---------------------------------------------------------------------------
 * Learned form: surrogate networks for the potential functions.
 *
 * An extension beyond the paper, whose f, phi and F always come from the
 * interpolated tables of Sec. 4.1: a handle created with pair_precision
 * MISA_MLP evaluates f(r), phi(r) (and their derivatives) in the lattice rho and
 * force passes, and F(rho), F'(rho) for lattice atoms, with one small network
 * per function inside the network's input range [x_lo, x_hi], and with the
 * spline tables outside it.  Pairs that involve a run-away atom keep the float64
 * tables.  Storage and arithmetic are those of MISA_FP32.
 *
 * Network (one input x, two SiLU layers of MISA_MLP_HIDDEN units, one output):
 *   t = (x - c) s with c = (x_lo + x_hi) / 2, s = 2 / (x_hi - x_lo)
 *   h1 = silu(W1 t + b1), h2 = silu(W2 h1 + b2), y = w3 . h2 + b3,
 *   g(x) = y_shift + y_scale y,  g'(x) = y_scale s dy/dt,  silu(z) = z / (1 + e^-z).
 * params holds W1[32], b1[32], W2[32][32] (row = output unit), b2[32], w3[32], b3.
 * Weights attached to a lattice must be exactly representable in bfloat16; the
 * lattice kernels run the 32 x 32 layer on the matrix cores with bfloat16
 * operands (activations split into two bfloat16 terms) and float32 accumulation.
 */
#define MISA_MLP 2 /* pair_precision: float32 pair arithmetic with surrogate networks for f, phi and F */

#define MISA_FN_F 0   /* electron density contribution f(r) */
#define MISA_FN_PHI 1 /* pair potential phi(r) */
#define MISA_FN_EMB 2 /* embedding energy F(rho) */

#define MISA_MLP_HIDDEN 32
#define MISA_MLP_PARAMS 1153 /* 32 (32 + 4) + 1 */
#define MISA_FM_SLOTS 96     /* pair slots per sampled atom in force-matching data */

typedef struct {
    double x_lo, x_hi;     /* input range served by the network (x_lo < x_hi) */
    double y_shift, y_scale;
    float params[MISA_MLP_PARAMS];
    int32_t reserved;
} misa_mlp_net;

/* Attach the network for function fn to a MISA_MLP handle (copied; host memory).
 * MISA_EINVAL if a weight is not a bfloat16 value or the range is empty;
 * MISA_ESTATE on a handle of another pair precision.  The tables of
 * misa_set_potential_tables remain required (fallback outside the range).
 * The first call also allocates the handle's pair buffer, K x sites floats
 * (16.8 GB for 320^3 cells): the rho pass keeps f'(r) of every pair there and
 * the force pass reads it instead of evaluating the f network again
 * (MISA_ENOMEM if that fails). */
int misa_set_mlp(misa_lattice *h, int fn, const misa_mlp_net *net);

/* The handle's float64 spline tables evaluated at n device-resident points
 * x[n]: g(x) into y[n] and g'(x) into dy[n] (device memory; Sec. 4.1 form).
 * These are the training targets of the surrogates. */
int misa_table_eval(misa_lattice *h, int fn, const double *x, int64_t n, double *y, double *dy);

/* Trainer: float32 master weights, Adam state and scratch for the three
 * networks on the GPU of the given stream.  All arrays are device memory. */
typedef struct misa_mlp_trainer misa_mlp_trainer;

typedef struct {
    int64_t iters;      /* optimiser steps */
    int32_t batch;      /* samples per step (misa_mlp_fit) or sampled atoms per step (force matching) */
    int32_t quantize;   /* 1: forward passes use the weights rounded to bfloat16 (quantisation-aware) */
    double lr;          /* Adam step size at the first step */
    double lr_final;    /* step size at the last step (cosine decay in between) */
    double lambda;      /* weight of the derivative term of the fit loss */
    uint64_t seed;      /* mini-batch draws: SplitMix64 of (seed, step, sample) */
} misa_fit_opts;

int misa_mlp_trainer_create(void *hip_stream, misa_mlp_trainer **out);
int misa_mlp_trainer_destroy(misa_mlp_trainer *t);
const char *misa_mlp_last_error(const misa_mlp_trainer *t);

/* Set network fn (range, scaling and float32 master weights; resets its Adam state). */
int misa_mlp_trainer_set(misa_mlp_trainer *t, int fn, const misa_mlp_net *net);
/* Get network fn with its weights rounded to bfloat16 (ready for misa_set_mlp);
 * master (may be NULL) receives the float32 master weights. */
int misa_mlp_trainer_get(misa_mlp_trainer *t, int fn, misa_mlp_net *net, float *master);

/* g(x) and g'(x) of network fn (bfloat16-rounded weights) at n points: path 0 is
 * the float32 training forward pass, path 1 the matrix-core evaluation that the
 * lattice kernels use. */
int misa_mlp_eval(misa_mlp_trainer *t, int fn, int path, const double *x, int64_t n, double *y, double *dy);

/* Gradient, with respect to the MISA_MLP_PARAMS weights (at their bfloat16
 * rounding), of sum_i c_val[i] y(t_i) + c_der[i] dy/dt(t_i), where y is the
 * network's normalised output and t_i the normalised input of x[i]; into grad
 * (float64, MISA_MLP_PARAMS values).  The backward pass of the training. */
int misa_mlp_grad(misa_mlp_trainer *t, int fn, const double *x, const double *c_val, const double *c_der,
                  int64_t n, double *grad);

/* One Adam step (Kingma and Ba: beta1 0.9, beta2 0.999, eps 1e-8) of network fn
 * with gradient grad[MISA_MLP_PARAMS] and step size lr. */
int misa_mlp_adam(misa_mlp_trainer *t, int fn, const double *grad, double lr);

/* Fit network fn to samples of its function: x[n], y[n] = g(x), dy[n] = g'(x)
 * (for instance from misa_table_eval).  Loss per mini-batch: mean over samples of
 * (y_net - y)^2 + lambda (dy_net - dy)^2 in the network's normalised units.  The
 * arrays stay registered with the trainer (and must stay valid) as the
 * function's samples for misa_mlp_force_match.  *loss: mean loss of the last
 * 1 % of steps. */
int misa_mlp_fit(misa_mlp_trainer *t, int fn, const double *x, const double *y, const double *dy, int64_t n,
                 const misa_fit_opts *o, double *loss);

/* misa_mlp_fit of nnet (1 to 3) different networks fns[k] together, with the same
 * options: network k fits its own samples x[k], y[k], dy[k] (n[k] each, device
 * memory) and draws its own mini-batches exactly as misa_mlp_fit alone would with
 * seed o->seed + fns[k], so the weights are bit for bit those of nnet separate
 * calls with those seeds; one kernel launch per
 * step serves all of them (each step's partial gradients, their sum and the Adam
 * update in that one launch).  loss[k] (host, may be NULL): as misa_mlp_fit's.
 * MISA_EINVAL for a network listed twice or a batch above 65535 * 64. */
int misa_mlp_fit_many(misa_mlp_trainer *t, int nnet, const int *fns, const double *const *x,
                      const double *const *y, const double *const *dy, const int64_t *n, const misa_fit_opts *o,
                      double *loss);

/* Force-matching data from the current state of a lattice handle after
 * misa_compute_rho: for each of the n lattice sites sites[] (lattice ids of
 * Sec. 3, host memory), the pairs of the atom it holds with slotted
 * neighbours within rc: r[n][MISA_FM_SLOTS] (0 = empty slot), unit vectors
 * dhat[n][MISA_FM_SLOTS][3] from the atom to the partner, the partner's F'
 * fp_j[n][MISA_FM_SLOTS], the atom's F' fp_i[n] and its reference force
 * f_ref[n][3] = sum over those pairs of the float64-table pair force.  Device
 * outputs.  A vacant site gives an empty list and a zero force.  Pairs with
 * run-away atoms are not part of the lists (those keep the tables). */
int misa_mlp_collect(misa_lattice *h, const int64_t *sites, int64_t n, double *r, double *dhat, double *fp_j,
                     double *fp_i, double *f_ref);

/* Tune the f and phi networks so that the forces of collected atoms match
 * f_ref: loss = sum |F - f_ref|^2 / (batch <|f_ref|^2>) over a mini-batch of
 * o->batch atoms per step (o->batch == n_env: every atom once, in order), plus
 * the fit loss of each of the two networks on its registered samples.  F'
 * stays that of the data.  *loss: force term, mean of the last 1 % of steps,
 * each evaluated before that step's update. */
int misa_mlp_force_match(misa_mlp_trainer *t, const double *r, const double *dhat, const double *fp_j,
                         const double *fp_i, const double *f_ref, int64_t n_env, const misa_fit_opts *o,
                         double *loss);

/* ---------------------------------------------------------------------------
 * Batched replicas: many independent periodic boxes stepped together.
 *
 * The paper names batch execution of simulations as a use of MISA-MD (Sec. 1);
 * this is its single-GPU form.  A batch owns one lattice handle per box, all on
 * one stream, all with pair_precision MISA_FP32 and the same a, rc, delta and
 * mass (one stencil, one potential).  Boxes may differ in size and in state;
 * each keeps its own adaptive time step, run-away atoms, hash and statistics.
 * misa_batch_step advances every box by the same number of steps with one
 * launch per kernel of the step for the whole batch: the rho and force passes
 * are single persistent launches over a list of (box, tile) items, the passes
 * over run-away atoms take items from one list of all boxes' run-aways, the other
 * kernels take the box from the grid's second dimension.  Results equal those
 * of misa_step on each box alone, bit for bit.
 */
typedef struct misa_batch misa_batch;

/* n_boxes descriptors (host), 1 <= n_boxes <= 8192; on success *out owns the batch.
 * The run-away passes of a batched step run over one work list of all boxes,
 * indexed with 32-bit integers: MISA_EINVAL when the boxes' run-away capacities
 * (or the affected-atom capacities derived from them) sum to 2^31 - 1 or more. */
int misa_batch_create(const misa_lattice_desc *descs, int32_t n_boxes, void *hip_stream, misa_batch **out);
int misa_batch_destroy(misa_batch *b);
const char *misa_batch_last_error(const misa_batch *b);

/* The lattice handle of box k (owned by the batch; bind its state, load atoms,
 * read results and fields with the single-box calls). */
int misa_batch_box(misa_batch *b, int32_t k, misa_lattice **out);

/* misa_set_potential_tables on every box. */
int misa_batch_set_potential_tables(misa_batch *b, const misa_table *f, const misa_table *phi,
                                    const misa_table *emb);

/* nsteps steps of every box (as misa_step); stats: n_boxes records in host
 * memory, or NULL.  Synchronises the stream at the end.  MISA_EOVERFLOW if any
 * box exceeded its run-away capacity (its record says which).  With
 * misa_set_timing on box 0, the batch's kernel times accumulate on box 0. */
int misa_batch_step(misa_batch *b, int64_t nsteps, double dt_max, double dx_max, misa_step_stats *stats);

/* enable != 0: misa_batch_step replays one captured HIP graph of a batched step
 * for all its steps but the last (as misa_set_graph does for one box).  The graph
 * is captured again when the step's arguments change: dt_max, dx_max, tile
 * shapes, or any box's tables, state binding, schedule or networks. */
int misa_batch_set_graph(misa_batch *b, int enable);

/* Tile shapes of the batched rho and force passes.  Every tile has 512 cells (1024
 * lanes, both sublattices) and is staged in LDS with a 2-cell halo; a box whose
 * sides are not multiples of 8 wastes less work on a shape that fits it better.
 * Shapes (x, y, z cells): 0: 8x8x8 (the default and the single-box tiling),
 * 1: 16x8x4, 2: 8x16x4, 3: 16x4x8, 4: 4x16x8, 5: 8x4x16, 6: 4x8x16.
 * Per-atom rho, F' and forces do not depend on the shape (every atom sums its
 * stencil in the same order); the per-tile energy and kinetic sums do, so
 * energies may differ from misa_step's in the last bits. */
#define MISA_TILE_SHAPES 7
int misa_batch_set_tile_shape(misa_batch *b, int32_t k, int32_t shape);
int misa_batch_get_tile_shape(misa_batch *b, int32_t k, int32_t *shape);

/* Autotuner: times probe_steps batched steps (as misa_batch_step, after one
 * untimed step) with every box on 8x8x8 tiles (policy 0) and with every box on the
 * shape that covers it with the fewest cells (policy 1), and keeps the faster
 * policy.  The boxes advance by *steps_done steps (1 + probe_steps per policy
 * tried; one policy is tried when both coincide).  Outputs (host, any may be
 * NULL): *policy, ms_per_step[2] of the two policies, *steps_done.  Synchronises
 * the stream. */
int misa_batch_autotune(misa_batch *b, int64_t probe_steps, double dt_max, double dx_max, int32_t *policy,
                        double *ms_per_step, int64_t *steps_done);

#ifdef __cplusplus
}
#endif

#endif /* MISA_H */

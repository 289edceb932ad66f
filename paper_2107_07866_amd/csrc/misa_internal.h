// Internal declarations of the MI355X EAM lattice MD library (not installed).
//
// Data layout in device memory (one structure-of-arrays slot per BCC site):
//   sites are split into two simple-cubic sublattices p = 0 (cube corners) and
//   p = 1 (body centres); storage index  s = p * ncell + (z * ny + y) * nx + x
//   for cell (x, y, z).  The paper's lattice id (Sec. 3) of the same site is
//   2 nx ny z + 2 nx y + 2 x + p; the library converts at its boundary.
//   Per site: displacement u = atom position - site position (float64 x3;
//   an empty slot stores VACANT_U), velocity (float64 x3), force (x3, float64
//   or float32 by pair precision), rho and F'(rho) (pair precision), atom id
//   (int32; VACANT_ID for an empty slot).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "misa.h"
#include "mlp_device.h"

namespace misa {

// ---------------------------------------------------------------------------
// Compile-time tiling of the lattice kernels.
// A work-group owns a TX x TY x TZ brick of cells (both sublattices) and stages
// it in LDS with a HALO-cell periodic halo; one lane per site; the stencil loop
// runs over a wave-uniform offset, so every wave serves one parity and one z plane.
constexpr int TX = 8, TY = 8, TZ = 4, HALO = 2;
constexpr int PX = TX + 2 * HALO, PY = TY + 2 * HALO, PZ = TZ + 2 * HALO;
constexpr int TILE_SITES = 2 * PX * PY * PZ;   // LDS entries per work-group (with halo)
constexpr int TILE_THREADS = 2 * TX * TY * TZ; // 512: one lane per interior site
static_assert(TX * TY == 64, "one wave covers one TX x TY plane of one parity");
constexpr int KMAX = 96;                       // max stencil entries per parity

// Persistent float32 variant: 8 x 8 x 8-cell tiles, 1024 lanes, and the window
// of the coefficient tables that slotted pairs can reach kept in LDS.
constexpr int T2X = 8, T2Y = 8, T2Z = 8;
constexpr int P2X = T2X + 2 * HALO, P2Y = T2Y + 2 * HALO, P2Z = T2Z + 2 * HALO;
constexpr int TILE2_SITES = 2 * P2X * P2Y * P2Z;
constexpr int TILE2_THREADS = 2 * T2X * T2Y * T2Z;  // 1024
constexpr int LDS_TAB_SEGS = 6144;                  // table segments of the gather passes' LDS window (+ zero record)

// Tile shapes of the batched persistent passes: tx ty tz = 512 cells (1024 lanes for
// both sublattices) whose staged block (with halo) fits beside the table window.
// Shape 0 is the 8 x 8 x 8 tile of the single-box passes.
constexpr int N_TILE_SHAPES = 7;
constexpr int TILE_SHAPES[N_TILE_SHAPES][3] = {{8, 8, 8},  {16, 8, 4}, {8, 16, 4}, {16, 4, 8},
                                               {4, 16, 8}, {8, 4, 16}, {4, 8, 16}};
constexpr int TILE2_SITES_MAX = 2 * 20 * 12 * 8;    // largest staged block of those shapes
constexpr bool tile_shapes_fit() {
    for (int s = 0; s < N_TILE_SHAPES; ++s) {
        const int *t = TILE_SHAPES[s];
        if (t[0] * t[1] * t[2] != 512 || 2 * (t[0] + 4) * (t[1] + 4) * (t[2] + 4) > TILE2_SITES_MAX) return false;
    }
    return TILE_SHAPES[0][0] == 8 && TILE_SHAPES[0][1] == 8 && TILE_SHAPES[0][2] == 8;
}
static_assert(tile_shapes_fit(), "every batch tile shape has 512 cells and fits the staged block");

// Half-stencil variant (each pair once): the same 8 x 8 x 8-cell tiles staged
// with their forward footprint (x, y: -2 .. +10 cells, z: 0 .. +10), LDS
// accumulators for every footprint site, and a smaller table window to make room.
constexpr int HFX = T2X + 2 * HALO, HFY = T2Y + 2 * HALO, HFZ = T2Z + HALO;
constexpr int HT_SITES = 2 * HFX * HFY * HFZ;       // 2880
constexpr int HALF_TAB_SEGS = 2880;                 // LDS: 3 x 46,080 (tile, accumulators, f records) + 23,040 B
constexpr int HALF_PHASES = 6;                      // (dZ in 0..2) x (partner parity same / other)
constexpr int HALF_META = 16;                       // ints per parity: phase starts [7], in-rc counts [6]

constexpr double VACANT_U = 1.0e6;             // displacement stored in an empty slot
constexpr double VACANT_TEST = 0.5e6;          // ux above this means the slot is empty
constexpr int32_t VACANT_ID = 0x7fffffff;      // atom id stored in an empty slot

// run-away scratch
constexpr int SORT_THREADS = 1024;
constexpr int SORT_LDS_MAX = 16384;            // single-block LDS bitonic sort up to this many keys (128 KB)
constexpr int BATCH_MAX_BOXES = 8192;         // boxes per batch (run-away list offsets staged in LDS)
constexpr int SMALL_GRID = 1024;               // blocks of grid-stride kernels over run-away lists
constexpr int MARK_THREADS = 256;              // lanes per block of the mark-bitmap compaction
constexpr int MARK_WORDS = 8;                  // bitmap words per lane (two 16-byte loads)
constexpr int CS_THREADS = 256;                // lanes per block of the coarse-cell scan
constexpr int CS_ITEMS = 16;                   // cells per lane (four 16-byte loads)
constexpr int CS_CHUNK = CS_THREADS * CS_ITEMS;

// 1 eV/(Angstrom amu) in Angstrom/fs^2 (exact SI e, CODATA-2018 amu)
constexpr double ACC_UNIT = (1.602176634e-19 / 1.66053906660e-27) * 1e-10;

template <typename Real>
struct alignas(4 * sizeof(Real)) Q4 {
    Real x, y, z, w;
};

// One Neighbor Offset Index entry, prepared for the LDS tile of a given parity:
// lds = offset of the neighbour's LDS entry from the centre's, o = site offset vector.
template <typename Real>
struct StencilEntry;
template <>
struct alignas(32) StencilEntry<double> {
    int32_t lds, pad;
    double ox, oy, oz;
};
template <>
struct alignas(16) StencilEntry<float> {
    int32_t lds;
    float ox, oy, oz;
};

// Cut-off decisions of float32 pair arithmetic.  A pair counts iff r < rc (Eq.
// eam_base).  For two slotted atoms (|u| < 1.24 A, site offsets below 8 A) the
// float32 r^2 = |o + u_j - u_i|^2 lies within 3e-5 A^2 of the float64 one (each
// displacement and offset rounded once, two rounded sums, three rounded squares and
// their sum), so outside a band of RC_BAND_Q around rc^2 the float32 decision is the
// float64 one.  Inside the band the decision is taken again in float64 from the
// stored displacements, as the float64 passes take it; at 300 K about one pair in
// 10^5 falls there.
constexpr float RC_BAND_Q = 1.0e-4f;   // A^2
constexpr float NEAR_MARGIN = 1.0e-3f; // A: slack of the per-tile test below

// float32 r^2 of a separation, in the one order every float32 pass and the fix-ups
// use, so that all of them see the same bits for the same pair.
__device__ __forceinline__ float pair_r2_f32(float dx, float dy, float dz) {
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dx, dx, dy * dy));
}

// Position (q - q0) / hq of q = r^2 on the q grid of the float32 table window.
__device__ __forceinline__ float win_pos(float r2, float inv_hq, float pcq) {
    return __builtin_fmaf(r2, inv_hq, pcq);
}

// Local segment index and offset t for pp = (q - q0) / hq on the window's q = r^2
// grid.  With kNodeCut the last node sits at the cut-off and the window ends with
// a zero record at local index nwin: pairs at or beyond the cut-off read zeros, so
// no separate cut-off select is needed.
template <bool kNodeCut>
__device__ __forceinline__ int win_seg(float pp, int nwin, float &t) {
    const float top = kNodeCut ? (float)nwin : (float)(nwin - 1);
    t = __builtin_amdgcn_fractf(pp);
    return (int)__builtin_amdgcn_fmed3f(pp, 0.0f, top);
}

// A stencil entry as the float64 re-decision needs it: the lattice-id offset of
// Sec. 3 and the site offset vector, in the order of the kernel's float stencil.
struct alignas(16) NearEntry {
    int32_t dX, dY, dZ, pad;
    double ox, oy, oz, pad2;
};

// What the float32 passes need for that re-decision, in device memory (the kernels
// take a pointer and read it only where they need it: kept out of the scalar
// registers of the pair loops).  thr2[p][k] (k < 64, in the stencil's order; the
// gather stencil is sorted by |o|, the half stencil by |o| inside each phase): a
// tile whose occupied sites all have |u|^2 < thr2[p][k] holds no pair of entry k
// within NEAR_MARGIN of rc, since r <= |o_k| + 2 |u|max; -1 where |o_k| > rc -
// NEAR_MARGIN.
struct NearTab {
    double rc2;
    double pad;
    float thr2[2][64];
    NearEntry st[2][KMAX];
};

// Storage index of the site at lattice-id offset (dX, dY, dZ) from site (cx, cy, cz)
// of sublattice p, wrapped into the periodic box.
__device__ __forceinline__ int64_t offset_site(int cx, int cy, int cz, int p, const NearEntry &e, int nx, int ny,
                                               int nz, int64_t ncell) {
    int X = (2 * cx + p + e.dX) % (2 * nx);
    int Y = (cy + e.dY) % ny;
    int Z = (cz + e.dZ) % nz;
    X = X < 0 ? X + 2 * nx : X;
    Y = Y < 0 ? Y + ny : Y;
    Z = Z < 0 ? Z + nz : Z;
    return (int64_t)(X & 1) * ncell + ((int64_t)Z * ny + Y) * nx + (X >> 1);
}

// The float64 decision r^2 < rc^2 for the pair (i, its neighbour of entry e), with
// the separation formed as the float64 passes form it.
__device__ __forceinline__ bool pair_in_rc64(const double *__restrict__ ux, const double *__restrict__ uy,
                                             const double *__restrict__ uz, int64_t i, int cx, int cy, int cz,
                                             int p, const NearEntry &e, int nx, int ny, int nz, int64_t ncell,
                                             double rc2) {
    const int64_t j = offset_site(cx, cy, cz, p, e, nx, ny, nz, ncell);
    const double dx = (ux[j] - ux[i]) + e.ox;
    const double dy = (uy[j] - uy[i]) + e.oy;
    const double dz = (uz[j] - uz[i]) + e.oz;
    return dx * dx + dy * dy + dz * dz < rc2;
}

// Interpolation table metadata (records live in device memory).
template <typename Real>
struct TabMeta {
    Real x0, inv_h;
    int32_t nseg;          // number of segments = samples - 1
    int32_t pad;
    Real x_last;           // position of the last node
    Real y_last, d_last;   // value and d/dx at the last node (linear continuation)
};

// Device pointers to the coefficient records of one precision.
//  f:     Q4 per segment  {c0, c1, c2, c3}      value of f  = ((c3 t + c2) t + c1) t + c0
//  force: 2 x Q4 per seg. {f'0, f'1, f'2, p'0}, {p'1, p'2, 0, 0}:  f' = (f'2 t + f'1) t + f'0 (per Angstrom)
//  phi:   Q4 per segment  {c0, c1, c2, c3}      value of phi
//  emb:   2 x Q4 per seg. {c0, c1, c2, c3}, {d0, d1, d2, 0}: F and F' (per unit rho)
template <typename Real>
struct Tables {
    const Q4<Real> *f, *force, *phi, *emb;
    TabMeta<Real> fm, em;  // f / phi share one grid; emb has its own
    // dense force records, 6 per segment: f'0, f'1, f'2, phi'0, phi'1, phi'2 (the
    // float64 tile force pass; 48 instead of 64 gathered bytes per pair)
    const Real *force6 = nullptr;
};

struct Geom {
    int32_t nx, ny, nz;
    int32_t ntx, nty, ntz;  // tiles per axis
    int32_t ntiles, ntiles_pad;
    int32_t nt2[3];         // tiles per axis of the persistent float32 kernels
    int32_t ntiles2, ntiles2_pad;
    int32_t tshape[3];      // their interior cells per axis (8 x 8 x 8 on a handle; a batch may choose others)
    uint32_t tdiv[3];       // ceil(2^32 / (tshape + 4)): staged-block index division by multiply-high
    int64_t ncell;          // cells per sublattice
    int64_t nsites;
    double a, inv_a;
    double L[3];
    double rc, rc2, delta2;
    double pre2;            // slightly generous rc^2 for candidate searches followed by an exact test
    // coarse cells (edge >= rc) that bucket run-away atoms (the cell grid of the run-away passes)
    int32_t nc[3];
    int32_t pad;
    double inv_cs[3];
    // lattice search window around a run-away atom: cells [lo, lo + win) per axis
    int32_t win;
    int32_t pad2;
    double reach;           // (rc + delta) / a
    double inv_L[3];        // 1 / L: the minimum image of a run-away pair
};

// The other copy of the displacements and velocities.  A step's kick-drift reads
// the current copy and writes this one, which then becomes current; the copy it
// read still holds the state at the start of the step, so a step whose leavers
// overflow the run-away capacity can be undone exactly (Algorithm 2; the state is
// left at the start of the failing step).
struct UV {
    double *ux, *uy, *uz, *vx, *vy, *vz;
};

// Caller-owned state, carved from the bound buffer.
struct State {
    double *ux, *uy, *uz;
    double *vx, *vy, *vz;
    void *fx, *fy, *fz;     // Real
    void *rho, *fp;         // Real
    int32_t *atom;
    // run-away atoms (capacity rcap), list order is deterministic
    int32_t *r_id;
    double *r_x, *r_y, *r_z, *r_vx, *r_vy, *r_vz, *r_fx, *r_fy, *r_fz, *r_rho, *r_fp, *r_e;
};

// Device counters (library scratch).
struct Counters {
    int32_t n_run;        // run-away atoms in the list
    int32_t n_leave;      // atoms that left their slot this step
    int32_t n_affected;   // lattice atoms within rc of a run-away atom
    int32_t overflow;     // 0; 1: this step's leavers exceed the run-away capacity; 2: the state
                          // is back at the start of that step and the call's later steps are frozen
    uint32_t range_viol;  // densities beyond the embedding table
    int32_t steps;        // steps completed in the current misa_step call
    int32_t fail_step;    // with overflow: index in the call of the step that overflowed
    int32_t n_cells;      // coarse cells whose run-aways are summed by cell (entries of Scratch::cellq)
    int32_t n_lone;       // run-aways of the other occupied cells, summed one by one (Scratch::loneq)
    int32_t pad;
};

// Library scratch (hipMalloc'd by the handle).
struct Scratch {
    Counters *cnt;
    double *scal;         // [0] dt of the next step, [1] time, [2] vmax, [3] e_kin, [4] e_emb, [5] e_pair, [6] dt of the last step
    double *part;         // per-tile partial sums (2 per tile) and per-block partials
    double *part_run;     // per-run-away partials
    // leavers of one step
    int32_t *l_site, *l_id;
    double *l_x, *l_y, *l_z, *l_vx, *l_vy, *l_vz;
    // claims / settling
    int32_t *cand;        // candidate site per (run-away or leaver) entry, -1 if none
    uint8_t *settled;
    // sort buffer (the leaver sort, the defect count's sort)
    uint64_t *sortbuf;
    // run-away atoms by coarse cell: the dense cell grid (padded to cs_nblk * CS_CHUNK
    // cells) and the run-aways sorted by (cell, list index)
    int32_t *cell_n;               // run-aways per cell while the grid is built; zero between builds
    int32_t *cell_s;               // first sorted place of each cell (cs_nblk * CS_CHUNK + 1 entries)
    int32_t *cs_blk;               // per-block totals of the cell scan
    int32_t cs_nblk;
    int32_t *skey, *sidx;          // cell and list index of each sorted place
    int32_t *sorder;               // list indices in (cell, list index) order while a build is ordered
    double *srx, *sry, *srz;       // run-away positions in the sorted (cell, list index) order
    double *sfp;                   // run-away F' in that order (written by the density pass)
    int32_t *cellq;                // sorted position of the first run-away of each crowded cell (any order)
    int32_t *loneq;                // sorted positions of the run-aways of the other cells (any order)
    // lattice atoms near run-away atoms
    uint32_t *mark;       // 1 bit per site, padded with zero words to mark_nblk blocks
    int64_t mark_nwords;  // padded length: mark_nblk * MARK_THREADS * MARK_WORDS
    int32_t mark_nblk;
    int32_t *mark_blk;    // marked sites per compaction block
    int64_t *mark_off;    // exclusive prefix of mark_blk
    int32_t *affected;    // ascending site indices, capacity affected_cap
    int64_t affected_cap;
    double *aff_v2;       // |v|^2 of each affected lattice atom after the fused final kick
    double *aff_e;        // pair-energy correction of each affected lattice atom (energy passes)
    double *part_kick;    // per-tile {max |v|^2, sum |v|^2} of the fused final kick
};

template <typename Real>
struct DevTables {
    Q4<Real> *f = nullptr, *force = nullptr, *phi = nullptr, *emb = nullptr;
    Real *force6 = nullptr;
    TabMeta<Real> fm{}, em{};
};

// Force record of one q segment of the half-stencil passes' window: {g_f0, g_f1},
// {g_f2, g_p0}, {g_p1, g_p2} with g_f = f'(r) / r and g_p = phi'(r) / r as quadratics in t.
struct alignas(8) FRec32 {
    float2 a, b, c;
};

// Window of f and phi that pairs of slotted atoms can reach (r >= nearest-site
// distance - 2 delta), re-tabulated on an equidistant grid in q = r^2 for the LDS:
// segment s covers q in [q0 + s hq, q0 + (s + 1) hq], local t in [0, 1], so the pair
// loops need neither sqrt(q) nor 1/r.  Two record forms:
//   gather passes (LDS_TAB_SEGS segments), linear in t between the spline's values at
//   the segment's two grid nodes:
//     lf: {f_0, f_1 - f_0}                                 (8 bytes)
//     lg: {gf_0, gf_1 - gf_0, gp_0, gp_1 - gp_0}           (16 bytes, one LDS read)
//   with gf = f'(r) / r and gp = phi'(r) / r;
//   half-stencil passes (HALF_TAB_SEGS segments, which share LDS with accumulators):
//     f:     f(q)                 = ((c3 t + c2) t + c1) t + c0
//     force: f'(r) / r, phi'(r)/r = (a2 t + a1) t + a0 (quadratics)
struct LdsTables {
    float2 *lf = nullptr;     // gather window: nwin linear value records of f
    float4 *lg = nullptr;     // gather window: nwin linear force records
    Q4<float> *f = nullptr;   // half window: nwin cubic value records of f
    FRec32 *force = nullptr;  // half window: nwin quadratic force records
    int32_t k0 = 0, nwin = 0; // k0: first r segment of the source tables inside the window
    float inv_hq = 0.f;       // 1 / hq
    float pcq = 0.f;          // -q0 / hq:  pp = q inv_hq + pcq
    bool usable = false;
    bool node_cut = false;    // last node at rc: a zero record after the window implements the cut-off
};

// What the fix-up of the affected list needs to correct the float32 gather pass for
// atoms with a pair inside the cut-off band (that pass's window of force records,
// the float64 stencil, the r-grid records of phi for the pair energy).  rec null:
// the force pass used takes that decision itself, or computes in float64.
struct NearFix32 {
    const float2 *frec = nullptr;     // linear value records of f (density)
    const float4 *rec = nullptr;      // linear force records
    const NearTab *nt = nullptr;
    const Q4<float> *phi = nullptr;
    TabMeta<float> fm{};
    float inv_hq = 0.f, pcq = 0.f, rc2 = 0.f;
    int32_t nwin = 0, node_cut = 0, K = 0;
};

// Table records of a persistent float64 pass held in LDS beside its tile, as bands of
// segments: the whole table when it has at most cap - 1 segments (cap: the records the
// pass has room for), else bands around the distances of the stencil's shells (r in
// [d - w, d + w], w as wide as the records allow, overlapping bands merged, the top band
// reaching the last node).  A zero record follows the top band and stands for segment
// nseg, where pairs at or past the cut-off land.  band[p KMAX + k] = {first segment,
// segments (zero record included), first LDS record, 0} for stencil entry k of parity p;
// a pair outside its entry's band reads its record from global memory.
//   force pass: FWIN64_MAX + 1 records of 48 bytes (f' and phi' as quadratics in t);
//   density pass: RWIN64_MAX records of 32 bytes (f as a cubic in t).
constexpr int FWIN64_MAX = 1080;
constexpr int RWIN64_MAX = 2520;
struct BandWin64 {
    double2 *recs = nullptr;  // nrec records (3 or 2 double2 each), in LDS order
    int4 *band = nullptr;     // 2 KMAX entries
    int32_t nrec = 0;
    double halfwidth = 0.0;   // w of the shell bands (0 when the table is held whole)
};


// Forward half of the stencil for the half-stencil passes, per parity: entries
// grouped by phase (dZ, partner parity != own), nearest first inside a phase,
// with LDS offsets in the footprint layout.  meta[p * HALF_META + q] is the first
// entry of phase q (q = 0 .. HALF_PHASES, the last one the end), and
// meta[p * HALF_META + 8 + q] the number of phase-q entries closer than rc.
struct HalfStencil {
    const StencilEntry<float> *st = nullptr;  // device [2][KMAX]
    const int32_t *meta = nullptr;            // device [2][HALF_META]
};

// Per-box pointers of the persistent float32 lattice passes.
struct PassPtrs {
    const double *ux, *uy, *uz;
    float *rho, *fp, *fx, *fy, *fz;
    double *vx, *vy, *vz;
    uint32_t *mark;
    const double *scal;  // scal[0] = dt of the current step
    double *part, *part_kick;
    uint32_t *range_viol;
};

// One box of a batch as the batched kernels read it.
struct BoxPass {
    Geom g;         // with the tiling the batch chose for this box
    PassPtrs P;
    int32_t shape;  // index of that tiling in TILE_SHAPES (and of its stencil)
    int32_t pad;
};
struct BoxRef {
    State S;
    Scratch sc;
    Geom g;
    int64_t rcap;
    UV alt;  // the kick-drift's destination (the other copy)
};

// Surrogate networks attached to a handle of the learned form (device copies).
struct MlpAttached {
    MlpNet net[3];                        // net[f].p -> weights (float32 holding bfloat16 values)
    float *p[3] = {nullptr, nullptr, nullptr};
    uint16_t *w2b[3] = {nullptr, nullptr, nullptr};  // W2 as bfloat16 bits (matrix-core A operand)
    bool set[3] = {false, false, false};
};

}  // namespace misa

struct misa_lattice {
    hipStream_t stream = nullptr;
    int device = 0;
    misa::Geom g{};
    int precision = MISA_FP64;                    // storage / arithmetic precision (MISA_FP32 for MISA_MLP)
    bool use_mlp = false;                         // learned form: networks in the lattice passes
    misa::MlpAttached mlp;
    double mass = 0.0;
    int64_t rcap = 0;
    int K = 0;                                    // stencil entries per parity
    int K_in = 0;                                 // entries closer than rc (the stencil is sorted by distance)
    float u_cut2 = -1.f;                          // tiles whose occupied sites all have |u|^2 below this skip
                                                  // entries K_in .. K - 1 (no pair there can reach rc)
    std::vector<int64_t> stencil_canon;           // [2][K][3] (dX, dY, dZ)
    misa::StencilEntry<double> *st64 = nullptr;   // device [2][KMAX]
    misa::StencilEntry<float> *st32 = nullptr;
    misa::DevTables<double> t64;
    misa::DevTables<float> t32;
    misa::LdsTables lds32;                        // window for the persistent float32 kernels
    double d_min = 0.0;                           // nearest-neighbour site distance
    int n_cu = 0;                                 // compute units of the device
    int persistent_grid = 0;                      // work-groups of the persistent kernels (multiple of 8)
    misa::NearTab *near_g = nullptr;              // float64 cut-off re-decision, gather order (device)
    misa::NearTab *near_h = nullptr;              // the same in half-stencil order
    misa::StencilEntry<float> *st32p = nullptr;   // stencil with LDS offsets of the 8x8x8 tiles
    misa::StencilEntry<double> *st64p = nullptr;  // the same offsets, float64 separations
    misa::BandWin64 fwin64;                       // force records of the persistent float64 force pass
    misa::BandWin64 rwin64;                       // f records of the persistent float64 density pass
    int pair_schedule = 0;                        // MISA_PAIRS_GATHER or MISA_PAIRS_HALF
    bool half_fits = false;                       // every axis a multiple of 16 cells (8 colours of tiles)
    misa::StencilEntry<float> *sth = nullptr;     // half-stencil entries (device [2][KMAX])
    int32_t *hmeta = nullptr;                     // half-stencil phases (device [2][HALF_META])
    misa::HalfStencil half;
    int half_entries = 0;                         // owned entries of the larger half-stencil parity
    float *pairbuf = nullptr;                     // learned form: f'(r) of every stencil candidate (gather) or
                                                  // owned pair (half), [K][nsites], rho pass -> force pass
    misa::LdsTables lds32h;                       // smaller window for the half-stencil passes
    bool tables_set = false;
    // host copy of the last misa_set_potential_tables samples (f, phi, F), kept so the
    // tables can be rebuilt after the neighbour-count export swaps f for a unit table
    std::vector<double> tab_y[3];
    misa_table tab[3] = {};
    misa::Scratch sc{};
    void *state_ptr = nullptr;
    int64_t state_bytes = 0;
    misa::State S{};                              // current view of the state
    misa::UV alt{};                               // the other copy of u and v (kick-drift destination)
    bool state_bound = false, state_set = false, rho_valid = false, force_valid = false;
    bool pending_clear = false;                   // cell lists and marks of a rho pass await the force pass
    int64_t n_atoms = 0;
    int64_t steps_done = 0;
    double *staging = nullptr;                    // device staging for host copies
    int64_t staging_bytes = 0;
    // HIP graph of one regular step (misa_set_graph): captured on a private stream,
    // replayed on the handle's stream; valid for one (dt_max, dx_max) and dropped
    // whenever tables, state binding, pair schedule or networks change
    bool use_graph = false;
    uint64_t gen = 0;                     // advances whenever captured kernel arguments go stale
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};  // one per copy a step starts from
    double graph_dt[2] = {0.0, 0.0}, graph_dx[2] = {0.0, 0.0};
    int parity = 0;                               // which copy of u and v is current (0: the first)
    // optional event timing of kernel groups
    bool timing = false;
    struct TimedGroup {
        hipEvent_t start, stop;
        int cls;
    };
    std::vector<TimedGroup> timed;                // recorded, not yet summed
    std::vector<std::pair<hipEvent_t, hipEvent_t>> event_pool;
    double timer_ms[MISA_TIMER_COUNT] = {0};
    int64_t timer_n[MISA_TIMER_COUNT] = {0};
    std::string err;
};

namespace misa {

// Float64 cut-off re-decision of the float32 passes (gather or half-stencil order).
inline const NearTab *near_args(const misa_lattice *h, bool half) { return half ? h->near_h : h->near_g; }

// ----------------------------------------------------------------------------
// Launchers (defined in the kernel translation units).  All enqueue on h->stream.
void drop_graph(misa_lattice *h);                      // forget the captured step (its arguments changed)
hipError_t launch_rho(misa_lattice *h);
hipError_t launch_force(misa_lattice *h, bool energy, bool kick);
bool lds_path(const misa_lattice *h);                  // persistent float32 kernels usable
NearFix32 near_fix_of(const misa_lattice *h);          // the affected-list correction of the gather pass
hipError_t launch_rho_lds(misa_lattice *h);
bool lds64_path(const misa_lattice *h);                // persistent float64 density pass usable
hipError_t launch_rho_lds64(misa_lattice *h);
bool lds64f_path(const misa_lattice *h);               // persistent float64 force pass usable
hipError_t launch_force_lds64(misa_lattice *h, bool energy, bool kick);
// per-tile partials of the force pass come from the 8 x 8 x 8 tiling
bool force_on_tiles2(const misa_lattice *h);
hipError_t launch_force_lds(misa_lattice *h, bool energy, bool kick);  // kick: fused second half-kick
PassPtrs pass_ptrs(misa_lattice *h);
// batched persistent passes over (box, tile) items; h0 supplies stencil, tables and stream
// st_shapes: [N_TILE_SHAPES][2][KMAX] stencils with the LDS offsets of each tile shape;
// any_shape: some box is not on 8 x 8 x 8 tiles (else the compile-time tiling serves)
hipError_t launch_rho_lds_batch(misa_lattice *h0, const BoxPass *boxes, const int2 *items, int nitems,
                                const StencilEntry<float> *st_shapes, bool any_shape);
hipError_t launch_force_lds_batch(misa_lattice *h0, const BoxPass *boxes, const int2 *items, int nitems,
                                  bool energy, bool kick, const StencilEntry<float> *st_shapes, bool any_shape);
bool fused_kick(const misa_lattice *h);               // the step fuses the final kick into the force pass
bool half_path(const misa_lattice *h);                // half-stencil passes serve this handle
hipError_t launch_rho_half(misa_lattice *h);            // zero, 8 colours, F'(rho)
hipError_t launch_force_half(misa_lattice *h, bool energy);
bool half_mlp_path(const misa_lattice *h);            // learned form on the half-stencil passes
hipError_t launch_rho_half_mlp(misa_lattice *h);        // zero, 8 colours, F'(rho) from the embedding network
hipError_t launch_force_half_mlp(misa_lattice *h, bool energy);
hipError_t launch_energy_reduce(misa_lattice *h, double *energies_dev);
hipError_t launch_rho_mlp(misa_lattice *h);             // learned form: rho pass with the networks
hipError_t launch_force_mlp(misa_lattice *h, bool energy);
hipError_t launch_runaway_build(misa_lattice *h);      // run-aways sorted into the coarse-cell grid
hipError_t launch_runaway_rho(misa_lattice *h);        // run-away rho + affected-site fixup
hipError_t launch_runaway_force(misa_lattice *h, bool energy, bool kick);
hipError_t launch_runaway_clear(misa_lattice *h);      // the pass's affected list spent
// lattice + run-aways, leavers appended; the lattice kick-drift writes the other copy of
// u and v, which becomes current (h->S and h->alt swap); the run-away kick-drift then
// undoes the step if its leavers overflowed
hipError_t launch_kick_drift(misa_lattice *h);
void swap_uv(misa_lattice *h);                         // exchange h->S's u, v with h->alt
hipError_t launch_rehash(misa_lattice *h);             // sort leavers, claims, settle, compact
hipError_t launch_final_kick(misa_lattice *h);         // + vmax / KE partials
hipError_t launch_dt_update(misa_lattice *h, double dt_max, double dx_max, bool first);
hipError_t launch_gather_state(misa_lattice *h, double *x, double *v);
hipError_t launch_fill_u32(misa_lattice *h, uint32_t *a, uint32_t value, int64_t n);  // a[0..n) = value
// placement of (n, 3) device positions / velocities into cleared slots; the rest to the leaver list
hipError_t launch_place(misa_lattice *h, const double *x, const double *v, int64_t n, int32_t *cand,
                        uint32_t *bad);
// batched replicas: one launch per kernel over every box (blockIdx.y = box)
// boxes: the box table of the step's start; boxes_after: the same with each box's u, v copies swapped
hipError_t launchb_kick_drift(hipStream_t st, const BoxRef *boxes, const BoxRef *boxes_after, int nbox, int gx_sites,
                              int gx_small, double kf);
hipError_t launchb_final_kick_runaway(hipStream_t st, const BoxRef *boxes, int nbox, int gx_small, double kf);
hipError_t launchb_dt_update(hipStream_t st, const BoxRef *boxes, int nbox, double mass, double dt_max, double dx_max);
hipError_t launchb_rehash(hipStream_t st, const BoxRef *boxes, int nbox, int gx_small);
hipError_t launchb_runaway_build(hipStream_t st, const BoxRef *boxes, int nbox, int gx_small, int gx_cells);
// off: 2 (nbox + 1) ints of device memory (the offsets of the run-away work list)
hipError_t launchb_runaway_rho(misa_lattice *h0, const BoxRef *boxes, int nbox, int mark_blocks, int32_t *off);
hipError_t launchb_runaway_force(misa_lattice *h0, const BoxRef *boxes, int nbox, bool energy, const int32_t *off);
hipError_t launchb_runaway_clear(hipStream_t st, const BoxRef *boxes, int nbox);
hipError_t launchb_energy_reduce(hipStream_t st, const BoxRef *boxes, int nbox);
hipError_t launch_gather_field(misa_lattice *h, int field, double *out);
hipError_t launch_gather_slots(misa_lattice *h, int64_t *out);
hipError_t launch_defects(misa_lattice *h, unsigned long long *out);  // 3 zeroed device counters

// ----------------------------------------------------------------------------
// Small device helpers shared by the kernel translation units.

__host__ __device__ inline int wrap_index(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

__device__ inline int tile_of_block(int b, const Geom &g) {
    // Work-groups are dispatched round-robin over the 8 XCDs; give every XCD a
    // contiguous run of tiles so halo re-reads of neighbouring tiles hit its own L2.
    int per = g.ntiles_pad >> 3;
    return (b & 7) * per + (b >> 3);
}

// Wrap a coordinate into [0, L).
__host__ __device__ inline double wrap_coord(double x, double L) {
#pragma clang fp contract(off)
    return x - L * floor(x / L);
}

// Site position of storage cell (cx, cy, cz) (unwrapped integers) of sublattice p.
__host__ __device__ inline void site_pos(int cx, int cy, int cz, int p, double a, double out[3]) {
#pragma clang fp contract(off)
    double h = p ? 0.5 : 0.0;
    out[0] = ((double)cx + h) * a;
    out[1] = ((double)cy + h) * a;
    out[2] = ((double)cz + h) * a;
}

// The hash (nearest lattice site), float64 without contraction so host and
// device take identical decisions: position wrapped into the box; nearest
// corner rounds each coordinate / a to the nearest integer (ties to even),
// nearest body centre takes floor + 1/2; the closer wins, the corner on a tie.
// Returns the storage index; u = x - site; *u2 = |u|^2.
__host__ __device__ inline int64_t hash_site(const double x[3], const Geom &g, double u[3], double *u2) {
#pragma clang fp contract(off)
    const int32_t n[3] = {g.nx, g.ny, g.nz};
    double uc[3], ub[3];
    int ic[3], ib[3];
    for (int k = 0; k < 3; ++k) {
        double xw = x[k] - g.L[k] * floor(x[k] / g.L[k]);
        double q = xw * g.inv_a;
        double c = rint(q);
        double fl = floor(q);
        double b = fl + 0.5;
        uc[k] = xw - c * g.a;
        ub[k] = xw - b * g.a;
        ic[k] = (int)c;
        ib[k] = (int)fl;
    }
    double dc = uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2];
    double db = ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2];
    int centre = db < dc ? 1 : 0;
    int c3[3];
    for (int k = 0; k < 3; ++k) {
        int c = (centre ? ib[k] : ic[k]) % n[k];  // full modulo: in range even for non-finite input
        if (c < 0) c += n[k];
        c3[k] = c;
        u[k] = centre ? ub[k] : uc[k];
    }
    *u2 = centre ? db : dc;
    return (int64_t)centre * g.ncell + ((int64_t)c3[2] * g.ny + c3[1]) * g.nx + c3[0];
}

// Storage index <-> lattice id of Sec. 3.
__host__ __device__ inline int64_t lattice_id_of(int64_t s, const Geom &g) {
    int64_t p = s >= g.ncell ? 1 : 0;
    int64_t c = s - p * g.ncell;
    int64_t cx = c % g.nx, cy = (c / g.nx) % g.ny, cz = c / ((int64_t)g.nx * g.ny);
    return 2 * (int64_t)g.nx * g.ny * cz + 2 * (int64_t)g.nx * cy + 2 * cx + p;
}

__host__ __device__ inline int64_t storage_of_lattice_id(int64_t id, const Geom &g) {
    const int64_t X = id % (2 * (int64_t)g.nx), Y = (id / (2 * (int64_t)g.nx)) % g.ny,
                  Z = id / (2 * (int64_t)g.nx * g.ny);
    return (X & 1) * g.ncell + (Z * g.ny + Y) * g.nx + (X >> 1);
}

// ---------------------------------------------------------------------------
// Table evaluation shared by the float64 lattice passes.

template <typename Real>
__device__ __forceinline__ void seg_index(Real x, const TabMeta<Real> &m, int &k, Real &t) {
    const Real p = (x - m.x0) * m.inv_h;
    int kk = (int)p;
    kk = kk < m.nseg - 1 ? kk : m.nseg - 1;
    kk = kk > 0 ? kk : 0;  // below the first node: cubic continuation of segment 0
    k = kk;
    t = p - (Real)kk;
}

// F(rho) and F'(rho); linear continuation beyond the last node (flagged).
template <typename Real>
__device__ __forceinline__ Real emb_eval(Real rho, const Q4<Real> *__restrict__ emb, const TabMeta<Real> &m,
                                         Real &Fval, bool &beyond) {
    if (rho > m.x_last) {
        beyond = true;
        Fval = m.y_last + m.d_last * (rho - m.x_last);
        return m.d_last;
    }
    int k;
    Real t;
    seg_index(rho, m, k, t);
    const Q4<Real> c = emb[2 * k];
    const Q4<Real> d = emb[2 * k + 1];
    Fval = ((c.w * t + c.z) * t + c.y) * t + c.x;
    return (d.z * t + d.y) * t + d.x;
}

// 1/sqrt(x) for x in a normal range (pair distances): hardware estimate refined by
// two Newton steps y <- y (3 - x y^2) / 2, each squaring the relative error, so the
// result is within a few ulp of the correctly rounded value.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// sqrt(x) and 1/sqrt(x) in float64 for the persistent lattice passes: the hardware
// estimate y0 of 1/sqrt(x) (about 23 correct bits) refined by one Newton step for each,
// with the residuals formed by fused multiply-adds:
//   g = x y0,  r = g + (y0 / 2)(x - g^2),  rinv = y0 + (y0 / 2)(1 - g y0),
// which leaves a relative error near 2e-14 (the square of the estimate's).
__device__ __forceinline__ double sqrt_nr1(double x) {
    const double y0 = __builtin_amdgcn_rsq(x);
    const double g = x * y0;
    return fma(0.5 * y0, fma(-g, g, x), g);
}
__device__ __forceinline__ void sqrt_rsqrt_nr1(double x, double &r, double &rinv) {
    const double y0 = __builtin_amdgcn_rsq(x);
    const double g = x * y0;
    const double h = 0.5 * y0;
    r = fma(h, fma(-g, g, x), g);
    rinv = fma(h, fma(-g, y0, 1.0), y0);
}

template <typename Real>
__device__ __forceinline__ Real pair_r(Real r2);
template <>
__device__ __forceinline__ double pair_r<double>(double r2) { return r2 * rsqrt_nr(r2); }
template <>
__device__ __forceinline__ float pair_r<float>(float r2) { return __builtin_amdgcn_sqrtf(r2); }

template <typename Real>
__device__ __forceinline__ void pair_r_rinv(Real r2, Real &r, Real &rinv);
template <>
__device__ __forceinline__ void pair_r_rinv<double>(double r2, double &r, double &rinv) {
    rinv = rsqrt_nr(r2);
    r = r2 * rinv;
}
template <>
__device__ __forceinline__ void pair_r_rinv<float>(float r2, float &r, float &rinv) {
    rinv = __builtin_amdgcn_rsqf(r2);
    r = r2 * rinv;
}

}  // namespace misa

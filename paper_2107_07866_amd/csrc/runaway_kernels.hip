// Atoms outside the lattice array (the hash-clash atoms of Sec. 3):
//   - hash update (Algorithm 2): atoms that drifted more than delta from their
//     site leave the array; run-away atoms take the empty slot of their nearest
//     site when within delta of it (lowest atom id wins, via atomicMin on the
//     slot's id word);
//   - a device hash of run-away atoms bucketed by coarse cells (edge >= rc):
//     atoms sorted by (cell, list index), open-addressing map cell -> first
//     position;
//   - run-away interactions (Algorithm 1, second and third loops) with every
//     unordered pair counted on both ends: a run-away atom gathers from lattice
//     sites in a window around it and from other run-aways through the hash;
//     each lattice atom within rc of a run-away gathers the matching reaction
//     terms itself, with the pair vector computed bit-identically, so no
//     scatter, atomics on floats or colouring are needed and results are
//     deterministic run to run.
// All arithmetic here is float64 regardless of the lattice pair precision.
//
// Multiply-adds are fused only within one source expression: the same item code
// runs inlined into single-box and batched (flattened) kernels, and fusion across
// statements would depend on the loop around it, so the two would round differently.
#pragma clang fp contract(on)
#include "misa_internal.h"

namespace misa {

// ---------------------------------------------------------------------------
// helpers

__device__ __forceinline__ double wave_sum64(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// i mod n for i in (-n, 2n): the lattice cells of a search window around a point of the
// box (the box spans more than two search reaches on every axis), wrapped with two
// conditional corrections instead of an integer division.
__device__ __forceinline__ int wrap_near(int i, int n) {
    i = i < 0 ? i + n : i;
    return i >= n ? i - n : i;
}

template <typename Real>
__device__ __forceinline__ void seg64(double x, const TabMeta<Real> &m, int &k, double &t) {
    const double p = (x - (double)m.x0) * (double)m.inv_h;
    int kk = (int)p;
    kk = kk < m.nseg - 1 ? kk : m.nseg - 1;
    kk = kk > 0 ? kk : 0;
    k = kk;
    t = p - (double)kk;
}

__device__ __forceinline__ double f_val(double r, const Tables<double> &T) {
    int k;
    double t;
    seg64(r, T.fm, k, t);
    const Q4<double> c = T.f[k];
    return ((c.w * t + c.z) * t + c.y) * t + c.x;
}

// f'(r), phi'(r) and phi(r)
__device__ __forceinline__ void fp_phi(double r, const Tables<double> &T, double &df, double &dphi, double &phi) {
    int k;
    double t;
    seg64(r, T.fm, k, t);
    const Q4<double> a = T.force[2 * k];
    const Q4<double> b = T.force[2 * k + 1];
    const Q4<double> c = T.phi[k];
    df = (a.z * t + a.y) * t + a.x;
    dphi = (b.y * t + b.x) * t + a.w;
    phi = ((c.w * t + c.z) * t + c.y) * t + c.x;
}

template <typename Real>
__device__ __forceinline__ Real emb_any(Real rho, const Q4<Real> *__restrict__ emb, const TabMeta<Real> &m,
                                        Real &Fval, bool &beyond) {
    if (rho > m.x_last) {
        beyond = true;
        Fval = m.y_last + m.d_last * (rho - m.x_last);
        return m.d_last;
    }
    const Real p = (rho - m.x0) * m.inv_h;
    int k = (int)p;
    k = k < m.nseg - 1 ? k : m.nseg - 1;
    k = k > 0 ? k : 0;
    Real t = p - (Real)k;
    const Q4<Real> c = emb[2 * k];
    const Q4<Real> d = emb[2 * k + 1];
    Fval = ((c.w * t + c.z) * t + c.y) * t + c.x;
    return (d.z * t + d.y) * t + d.x;
}

__device__ __forceinline__ int coarse_of(double xw, int nc, double inv_cs) {
    int c = (int)(xw * inv_cs);
    return c >= nc ? nc - 1 : (c < 0 ? 0 : c);
}

// Coarse cell of run-away r (the key the cell grid is indexed by).
__device__ __forceinline__ int32_t run_key(const State &S, const Geom &g, int r) {
    const int kx = coarse_of(S.r_x[r], g.nc[0], g.inv_cs[0]);
    const int ky = coarse_of(S.r_y[r], g.nc[1], g.inv_cs[1]);
    const int kz = coarse_of(S.r_z[r], g.nc[2], g.inv_cs[2]);
    return (kz * g.nc[1] + ky) * g.nc[0] + kx;
}

__device__ __forceinline__ int axis_cells(int c, int n, int out[3]) {
    if (n == 1) {
        out[0] = 0;
        return 1;
    }
    if (n == 2) {
        out[0] = 0;
        out[1] = 1;
        return 2;
    }
    out[0] = c == 0 ? n - 1 : c - 1;
    out[1] = c;
    out[2] = c == n - 1 ? 0 : c + 1;
    return 3;
}

// First cell of the lattice window searched around a run-away atom at q = x / a:
// every integer c with c > q - reach - 1/2 (covers corner sites c and centre sites c + 1/2).
__device__ __forceinline__ int window_lo(double q, double reach) { return (int)floor(q - reach - 0.5) + 1; }

// Separation x_j - x_r of lattice atom (site cell cx,cy,cz unwrapped near the
// run-away, sublattice p, displacement u) from run-away atom x: computed the same
// way by both kernels that see this pair.
__device__ __forceinline__ void lat_sep(int cx, int cy, int cz, int p, const double u[3], const double x[3],
                                        double a, double d[3]) {
    double sp[3];
    site_pos(cx, cy, cz, p, a, sp);
    d[0] = (sp[0] - x[0]) + u[0];
    d[1] = (sp[1] - x[1]) + u[1];
    d[2] = (sp[2] - x[2]) + u[2];
}

// Nearest periodic image of a separation of two wrapped positions (|d| <= L per axis).
// The image shift rint(d / L) is taken as rint(d * (1 / L)): the two differ only where
// |d| is within rounding of L / 2 on some axis, and such a pair lies beyond rc (the box
// exceeds 2 rc), so every pair within rc gets the same separation either way.
__device__ __forceinline__ void min_image3(double d[3], const Geom &g) {
    for (int k = 0; k < 3; ++k) d[k] -= g.L[k] * rint(d[k] * g.inv_L[k]);
}

// ---------------------------------------------------------------------------
// single-block bitonic sort of 64-bit keys (ascending): this step's leavers by atom
// id.  It first freezes a step that the run-away kick-drift has just undone after an
// overflow: no leavers, dt = 0 for the rest of the call (the step length is kept in
// scal[7]), and the step's index.

__device__ __forceinline__ void sort_body(uint64_t *__restrict__ buf, Counters *__restrict__ cnt, int64_t rcap,
                                          const int32_t *__restrict__ l_id, double *__restrict__ scal) {
    __shared__ uint64_t sh[SORT_LDS_MAX];
    if (threadIdx.x == 0 && cnt->overflow == 1) {
        scal[7] = scal[0];
        scal[0] = 0.0;
        cnt->n_leave = 0;
        cnt->fail_step = cnt->steps;
        cnt->overflow = 2;
    }
    __syncthreads();
    // leavers beyond the run-away capacity were not recorded (they kept their slots)
    const int nl = cnt->n_leave;
    const int room = (int)(rcap - cnt->n_run);
    const int n = nl < room ? nl : room;
    __syncthreads();
    if (threadIdx.x == 0) cnt->n_leave = n;
    if (n <= 1) {
        if (n == 1 && threadIdx.x == 0) buf[0] = ((uint64_t)(uint32_t)l_id[0] << 32) | 0u;
        return;
    }
    int P = 1;
    while (P < n) P <<= 1;
    const bool in_lds = P <= SORT_LDS_MAX;
    uint64_t *A = in_lds ? sh : buf;
    for (int i = threadIdx.x; i < P; i += SORT_THREADS)
        A[i] = i < n ? ((uint64_t)(uint32_t)l_id[i] << 32) | (uint32_t)i : ~0ull;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += SORT_THREADS) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint64_t a = A[i], b = A[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        A[i] = b;
                        A[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (in_lds)
        for (int i = threadIdx.x; i < n; i += SORT_THREADS) buf[i] = sh[i];
}

__global__ __launch_bounds__(SORT_THREADS) void k_sort(uint64_t *__restrict__ buf, Counters *__restrict__ cnt,
                                                        int64_t rcap, const int32_t *__restrict__ l_id,
                                                        double *__restrict__ scal) {
    sort_body(buf, cnt, rcap, l_id, scal);
}

__global__ __launch_bounds__(SORT_THREADS) void kb_sort(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    sort_body(B.sc.sortbuf, B.sc.cnt, B.rcap, B.sc.l_id, B.sc.scal);
}


// ---------------------------------------------------------------------------
// hash update

// Claims: each run-away atom and each leaver of this step that lies within
// delta of its nearest site, and finds that slot empty, bids with its atom id.
__device__ __forceinline__ void claim_body(State S, Scratch sc, Geom g) {
    const int nrun = sc.cnt->n_run;
    const int total = nrun + sc.cnt->n_leave;  // leavers admitted this step (clamped by k_sort)
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
        double x[3];
        int32_t id;
        if (q < nrun) {
            x[0] = S.r_x[q];
            x[1] = S.r_y[q];
            x[2] = S.r_z[q];
            id = S.r_id[q];
        } else {
            const int li = (int)(sc.sortbuf[q - nrun] & 0xffffffffu);
            x[0] = sc.l_x[li];
            x[1] = sc.l_y[li];
            x[2] = sc.l_z[li];
            id = sc.l_id[li];
        }
        double u[3], u2;
        const int64_t s = hash_site(x, g, u, &u2);
        int32_t cand = -1;
        if (u2 <= g.delta2 && S.ux[s] > VACANT_TEST) {
            cand = (int32_t)s;
            atomicMin(&S.atom[s], id);
        }
        sc.cand[q] = cand;
    }
}

__global__ void k_claim(State S, Scratch sc, Geom g) {
    claim_body(S, sc, g);
}

__global__ void kb_claim(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    claim_body(B.S, B.sc, B.g);
}


// The lowest bidder of each contested slot moves in.
__device__ __forceinline__ void settle_body(State S, Scratch sc, Geom g) {
    const int nrun = sc.cnt->n_run;
    const int total = nrun + sc.cnt->n_leave;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
        const int32_t s = sc.cand[q];
        uint8_t done = 0;
        if (s >= 0) {
            double x[3], v[3];
            int32_t id;
            if (q < nrun) {
                x[0] = S.r_x[q];
                x[1] = S.r_y[q];
                x[2] = S.r_z[q];
                v[0] = S.r_vx[q];
                v[1] = S.r_vy[q];
                v[2] = S.r_vz[q];
                id = S.r_id[q];
            } else {
                const int li = (int)(sc.sortbuf[q - nrun] & 0xffffffffu);
                x[0] = sc.l_x[li];
                x[1] = sc.l_y[li];
                x[2] = sc.l_z[li];
                v[0] = sc.l_vx[li];
                v[1] = sc.l_vy[li];
                v[2] = sc.l_vz[li];
                id = sc.l_id[li];
            }
            if (S.atom[s] == id) {
                double u[3], u2;
                hash_site(x, g, u, &u2);
                S.ux[s] = u[0];
                S.uy[s] = u[1];
                S.uz[s] = u[2];
                S.vx[s] = v[0];
                S.vy[s] = v[1];
                S.vz[s] = v[2];
                done = 1;
            }
        }
        sc.settled[q] = done;
    }
}

__global__ void k_settle(State S, Scratch sc, Geom g) {
    settle_body(S, sc, g);
}

__global__ void kb_settle(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    settle_body(B.S, B.sc, B.g);
}


// Stable compaction: surviving run-aways keep their order, surviving leavers
// follow in ascending atom id.  Single work-group.
__device__ __forceinline__ void compact_body(State S, Scratch sc) {
    __shared__ int wsum[1024 / 64];
    __shared__ int base_sh;
    const int nrun = sc.cnt->n_run;
    const int nl = sc.cnt->n_leave;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) base_sh = 0;
    __syncthreads();
    const int total = nrun + nl;
    for (int c0 = 0; c0 < total; c0 += 1024) {
        const int q = c0 + threadIdx.x;
        const bool keep = q < total && !sc.settled[q];
        int32_t id = 0;
        double x = 0, y = 0, z = 0, vx = 0, vy = 0, vz = 0;
        if (keep) {
            if (q < nrun) {
                id = S.r_id[q];
                x = S.r_x[q];
                y = S.r_y[q];
                z = S.r_z[q];
                vx = S.r_vx[q];
                vy = S.r_vy[q];
                vz = S.r_vz[q];
            } else {
                const int li = (int)(sc.sortbuf[q - nrun] & 0xffffffffu);
                id = sc.l_id[li];
                x = sc.l_x[li];
                y = sc.l_y[li];
                z = sc.l_z[li];
                vx = sc.l_vx[li];
                vy = sc.l_vy[li];
                vz = sc.l_vz[li];
            }
        }
        const uint64_t m = __ballot(keep);
        const int below = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[w] = __popcll(m);
        __syncthreads();
        int off = base_sh;
        for (int k = 0; k < w; ++k) off += wsum[k];
        int tot = 0;
        for (int k = 0; k < 1024 / 64; ++k) tot += wsum[k];
        __syncthreads();  // every lane has read its record and the wave sums
        if (keep) {
            const int o = off + below;
            S.r_id[o] = id;
            S.r_x[o] = x;
            S.r_y[o] = y;
            S.r_z[o] = z;
            S.r_vx[o] = vx;
            S.r_vy[o] = vy;
            S.r_vz[o] = vz;
        }
        if (threadIdx.x == 0) base_sh += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sc.cnt->n_run = base_sh;
        sc.cnt->n_leave = 0;
    }
}

__global__ __launch_bounds__(1024) void k_compact(State S, Scratch sc) {
    compact_body(S, sc);
}

__global__ __launch_bounds__(1024) void kb_compact(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    compact_body(B.S, B.sc);
}


// ---------------------------------------------------------------------------
// run-away atoms by coarse cell (edge >= rc): a counting sort into a dense grid
//
// count: run-aways per cell; scan: cell_s[c] = run-aways in cells before c (three
// kernels: block totals, their scan, the block scans); scatter: each run-away takes a
// place in its cell's stretch (counting the cell back down to zero, which leaves the
// grid ready for the next build); rank and order: each stretch is put in ascending list
// index, one lane per run-away (so every later pass sees the same order whatever the
// scatter's timing), the sorted copies are written, and the cell (or its atoms) is listed
// for the density and force passes.  cell_s[c + 1] - cell_s[c] is then the cell's
// run-away count.

// Cells with at least this many run-aways have their sums taken by cell (one block
// stages the cell's neighbourhood); the atoms of sparser cells are taken one by one.
constexpr int RC_MIN_HOME = 5;

__device__ __forceinline__ void cell_count_body(const State &S, Scratch sc, const Geom &g) {
    const int n = sc.cnt->n_run;
    if (blockIdx.x == 0 && threadIdx.x == 0) sc.cnt->n_cells = sc.cnt->n_lone = 0;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
        atomicAdd(&sc.cell_n[run_key(S, g, r)], 1);
}

__global__ void k_cell_count(State S, Scratch sc, Geom g) {
    cell_count_body(S, sc, g);
}

__global__ void kb_cell_count(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    cell_count_body(B.S, B.sc, B.g);
}

// Exclusive scan of one value per lane over a CS_THREADS block; total: the block's sum.
__device__ __forceinline__ int cs_block_scan(int v, int *sh_waves, int &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) sh_waves[w] = incl;
    __syncthreads();
    int off = 0;
    total = 0;
    for (int k = 0; k < CS_THREADS / 64; ++k) {
        if (k < w) off += sh_waves[k];
        total += sh_waves[k];
    }
    return off + incl - v;
}

// This lane's CS_ITEMS counts (the grid is padded with zero cells to whole blocks).
__device__ __forceinline__ int cs_load(const Scratch &sc, int (&m)[CS_ITEMS]) {
    const int64_t c0 = ((int64_t)blockIdx.x * CS_THREADS + threadIdx.x) * CS_ITEMS;
    const int4 *p = reinterpret_cast<const int4 *>(sc.cell_n + c0);
    int c = 0;
#pragma unroll
    for (int k = 0; k < CS_ITEMS / 4; ++k) {
        const int4 v = p[k];
        m[4 * k] = v.x, m[4 * k + 1] = v.y, m[4 * k + 2] = v.z, m[4 * k + 3] = v.w;
        c += v.x + v.y + v.z + v.w;
    }
    return c;
}

__device__ __forceinline__ void cell_sum_body(Scratch sc) {
    __shared__ int shw[CS_THREADS / 64];
    if ((int)blockIdx.x >= sc.cs_nblk) return;  // a batched grid sized for a larger box
    int m[CS_ITEMS], total;
    cs_block_scan(cs_load(sc, m), shw, total);
    if (threadIdx.x == 0) sc.cs_blk[blockIdx.x] = total;
}

__global__ __launch_bounds__(CS_THREADS) void k_cell_sum(Scratch sc) {
    cell_sum_body(sc);
}

__global__ __launch_bounds__(CS_THREADS) void kb_cell_sum(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    cell_sum_body(B.sc);
}

// Exclusive scan of the block totals in place; cell_s past the last cell gets the total.
__device__ __forceinline__ void cell_top_body(Scratch sc) {
    __shared__ int base_sh;
    __shared__ int wsum[1024 / 64];
    if (threadIdx.x == 0) base_sh = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nblk = sc.cs_nblk;
    for (int c0 = 0; c0 < nblk; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const int v = i < nblk ? sc.cs_blk[i] : 0;
        int incl = v;
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int off = base_sh, tot = 0;
        for (int k = 0; k < 1024 / 64; ++k) {
            if (k < w) off += wsum[k];
            tot += wsum[k];
        }
        if (i < nblk) sc.cs_blk[i] = off + incl - v;
        __syncthreads();
        if (threadIdx.x == 0) base_sh += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) sc.cell_s[(int64_t)nblk * CS_CHUNK] = base_sh;
}

__global__ __launch_bounds__(1024) void k_cell_top(Scratch sc) {
    cell_top_body(sc);
}

__global__ __launch_bounds__(1024) void kb_cell_top(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    cell_top_body(B.sc);
}

__device__ __forceinline__ void cell_down_body(Scratch sc) {
    __shared__ int shw[CS_THREADS / 64];
    if ((int)blockIdx.x >= sc.cs_nblk) return;
    int m[CS_ITEMS], total;
    int pos = sc.cs_blk[blockIdx.x] + cs_block_scan(cs_load(sc, m), shw, total);
    const int64_t c0 = ((int64_t)blockIdx.x * CS_THREADS + threadIdx.x) * CS_ITEMS;
    int4 *out = reinterpret_cast<int4 *>(sc.cell_s + c0);
#pragma unroll
    for (int k = 0; k < CS_ITEMS / 4; ++k) {
        int4 v;
        v.x = pos;
        pos += m[4 * k];
        v.y = pos;
        pos += m[4 * k + 1];
        v.z = pos;
        pos += m[4 * k + 2];
        v.w = pos;
        pos += m[4 * k + 3];
        out[k] = v;
    }
}

__global__ __launch_bounds__(CS_THREADS) void k_cell_down(Scratch sc) {
    cell_down_body(sc);
}

__global__ __launch_bounds__(CS_THREADS) void kb_cell_down(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    cell_down_body(B.sc);
}

__device__ __forceinline__ void cell_scatter_body(const State &S, Scratch sc, const Geom &g) {
    const int n = sc.cnt->n_run;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const int32_t key = run_key(S, g, r);
        const int q = sc.cell_s[key] + atomicSub(&sc.cell_n[key], 1) - 1;
        sc.skey[q] = key;
        sc.sidx[q] = r;
    }
}

__global__ void k_cell_scatter(State S, Scratch sc, Geom g) {
    cell_scatter_body(S, sc, g);
}

__global__ void kb_cell_scatter(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    cell_scatter_body(B.S, B.sc, B.g);
}

// rank: each run-away's place inside its cell's stretch is the count of the stretch's
// entries with a smaller list index (distinct), so the stretch comes out in ascending
// list index whatever order the scatter left it in.
__device__ __forceinline__ void cell_rank_body(Scratch sc) {
    const int n = sc.cnt->n_run;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const int32_t key = sc.skey[q];
        const int start = sc.cell_s[key], end = sc.cell_s[key + 1];
        const int32_t v = sc.sidx[q];
        int rank = 0;
        for (int i = start; i < end; ++i) rank += sc.sidx[i] < v ? 1 : 0;
        sc.sorder[start + rank] = v;
    }
}

__global__ void k_cell_rank(Scratch sc) {
    cell_rank_body(sc);
}

__global__ void kb_cell_rank(const BoxRef *__restrict__ boxes) {
    cell_rank_body(boxes[blockIdx.y].sc);
}

// order: the ranked list indices and the sorted position copies, and each cell (or its
// atoms) listed for the density and force passes by the run-away at its first place.
__device__ __forceinline__ void cell_order_body(const State &S, Scratch sc) {
    const int n = sc.cnt->n_run;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const int32_t o = sc.sorder[q];
        sc.sidx[q] = o;
        sc.srx[q] = S.r_x[o];
        sc.sry[q] = S.r_y[o];
        sc.srz[q] = S.r_z[o];
        const int32_t key = sc.skey[q];
        if (sc.cell_s[key] != q) continue;  // one lane per cell: the one at its first place
        const int end = sc.cell_s[key + 1];
        if (end - q >= RC_MIN_HOME) {
            sc.cellq[atomicAdd(&sc.cnt->n_cells, 1)] = q;
        } else {
            const int b = atomicAdd(&sc.cnt->n_lone, end - q);
            for (int i = q; i < end; ++i) sc.loneq[b + i - q] = i;
        }
    }
}

__global__ void k_cell_order(State S, Scratch sc) {
    cell_order_body(S, sc);
}

__global__ void kb_cell_order(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    cell_order_body(B.S, B.sc);
}

// End of a pass: the affected list is spent (the step statistics have read it).
__device__ __forceinline__ void runaway_clear_body(Scratch sc) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sc.cnt->n_affected = 0;
}

__global__ void k_runaway_clear(Scratch sc) {
    runaway_clear_body(sc);
}

__global__ void kb_runaway_clear(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    runaway_clear_body(B.sc);
}


// Run-away atoms in one of the (up to) 27 coarse cells around x, cell = ax + 3 (ay + 3 az);
// cells beyond the box's distinct neighbours are empty.  fn(o, xo) for entries first,
// first + stride, ... of the cell's stretch of the sorted list (o: list index, xo: position).
template <typename Fn>
__device__ __forceinline__ void for_runaways_in_cell(const double x[3], int cell, int first, int stride,
                                                     const Scratch &sc, const Geom &g, Fn fn) {
    const int ax = cell % 3, ay = (cell / 3) % 3, az = cell / 9;
    int cx[3], cy[3], cz[3];
    if (ax >= axis_cells(coarse_of(x[0], g.nc[0], g.inv_cs[0]), g.nc[0], cx)) return;
    if (ay >= axis_cells(coarse_of(x[1], g.nc[1], g.inv_cs[1]), g.nc[1], cy)) return;
    if (az >= axis_cells(coarse_of(x[2], g.nc[2], g.inv_cs[2]), g.nc[2], cz)) return;
    const int32_t key = (cz[az] * g.nc[1] + cy[ay]) * g.nc[0] + cx[ax];
    const int start = sc.cell_s[key], end = sc.cell_s[key + 1];
#pragma unroll 2
    for (int q = start + first; q < end; q += stride) {
        const double xo[3] = {sc.srx[q], sc.sry[q], sc.srz[q]};
        fn(sc.sidx[q], xo);
    }
}

// Run-aways of the (up to) 27 coarse cells around x, dealt over the W lanes of a team
// (W = 32: a team of the affected-atom passes; W = 64: a wave of the per-atom forms) as
// one list: the cells' stretches laid end to end (cell 0 first), lane k taking entries
// k, k + W, ..., G at a time with their loads issued together.  Every lane gets
// about the same number of entries (one lane per cell would wait on the fullest cell,
// one memory round trip per entry).  fn(o, xo) as for_runaways_in_cell.  All W lanes
// must call it together.
template <int W, int G, typename Fn>
__device__ __forceinline__ void for_runaways_around(const double x[3], int lane, const Scratch &sc, const Geom &g,
                                                    Fn fn) {
    int start = 0, cnt = 0;
    if (lane < 27) {
        const int ax = lane % 3, ay = (lane / 3) % 3, az = lane / 9;
        int cx[3], cy[3], cz[3];
        if (ax < axis_cells(coarse_of(x[0], g.nc[0], g.inv_cs[0]), g.nc[0], cx) &&
            ay < axis_cells(coarse_of(x[1], g.nc[1], g.inv_cs[1]), g.nc[1], cy) &&
            az < axis_cells(coarse_of(x[2], g.nc[2], g.inv_cs[2]), g.nc[2], cz)) {
            const int32_t key = (cz[az] * g.nc[1] + cy[ay]) * g.nc[0] + cx[ax];
            start = sc.cell_s[key];
            cnt = sc.cell_s[key + 1] - start;
        }
    }
    int incl = cnt;  // inclusive prefix over the team's cells
    for (int o = 1; o < W; o <<= 1) {
        const int t = __shfl_up(incl, o, W);
        if (lane >= o) incl += t;
    }
    const int total = __shfl(incl, W - 1, W);
    const int base = start - (incl - cnt);  // entry f of this lane's cell sits at base + f
    for (int f0 = 0; f0 < total; f0 += G * W) {
        int qv[G];
        bool ok[G];
#pragma unroll
        for (int t = 0; t < G; ++t) {
            const int f = f0 + t * W + lane;
            // the cell holding entry f: how many cells end at or before f (log2 W uniform steps)
            int c = 0;
#pragma unroll
            for (int step = W / 2; step > 0; step >>= 1)
                if (__shfl(incl, c + step - 1, W) <= f) c += step;
            // every lane reads (an operand of ?: would be read only by the lanes that take
            // it, and a shuffle from a lane that does not take part returns garbage)
            const int bq = __shfl(base, c, W);
            ok[t] = f < total;
            qv[t] = ok[t] ? bq + f : 0;
        }
        double xo[G][3];
        int32_t ov[G];
#pragma unroll
        for (int t = 0; t < G; ++t) {
            xo[t][0] = sc.srx[qv[t]];
            xo[t][1] = sc.sry[qv[t]];
            xo[t][2] = sc.srz[qv[t]];
            ov[t] = sc.sidx[qv[t]];
        }
#pragma unroll
        for (int t = 0; t < G; ++t)
            if (ok[t]) fn(ov[t], xo[t]);
    }
}

// Run-away atoms other than self closer than sqrt(cut2) to x, searched by a whole wave:
// with kDealt the 27 cells' run-aways dealt over the 64 lanes (for_runaways_around; the
// per-atom passes of sparse cells), else lanes k and k + 32 share coarse cell k (k < 27)
// and take alternate entries of it (the fall-back inside the cell-staged passes, whose
// registers are budgeted for their occupancy).
// Calls fn(o, d, r2) with d = x_o - x (minimum image).
template <bool kDealt, typename Fn>
__device__ __forceinline__ void for_runaway_neighbours(const double x[3], int self, int lane, double cut2,
                                                       const State &S, const Scratch &sc, const Geom &g,
                                                       Fn fn) {
    auto pair = [&](int o, const double *xo) {
        if (o == self) return;
        double d[3] = {xo[0] - x[0], xo[1] - x[1], xo[2] - x[2]};
        min_image3(d, g);
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (r2 < cut2) fn(o, d, r2);
    };
    if (kDealt) {
        for_runaways_around<64, 2>(x, lane, sc, g, pair);
    } else {
        const int cell = lane & 31;
        if (cell < 27) for_runaways_in_cell(x, cell, lane >> 5, 2, sc, g, pair);
    }
}

// Affected lattice atoms are handled by teams of 32 lanes: lane k looks up coarse cell k
// (lanes 27..31 none), so one atom's 27 cell look-ups run side by side, and the cells'
// run-aways are then dealt over all 32 lanes (for_runaways_around).
constexpr int AFF_TEAM = 32;
constexpr int AFF_THREADS = 256;
constexpr int AFF_GRID = 2048;

__device__ __forceinline__ double team_sum32(double v) {
    // fixed butterfly: the same lanes meet in the same order on every call
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, AFF_TEAM);
    return v;
}

// Separation x_j - x_o of lattice atom j (cell cj, parity p, displacement u) from
// run-away o, taken from the lattice window the run-away itself uses, so both sides see
// the same pair in the same arithmetic.  False if j lies outside that window.
__device__ __forceinline__ bool affected_pair(const double xo[3], const int cj[3], int p, const double u[3],
                                              const Geom &g, double d[3], double &r2) {
    int cc[3];
    const int nn[3] = {g.nx, g.ny, g.nz};
    for (int k = 0; k < 3; ++k) {
        const int lo = window_lo(xo[k] * g.inv_a, g.reach);
        cc[k] = lo + wrap_near(cj[k] - lo, nn[k]);
        if (cc[k] - lo >= g.win) return false;
    }
    lat_sep(cc[0], cc[1], cc[2], p, u, xo, g.a, d);
    r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    return r2 < g.rc2;
}

// ---------------------------------------------------------------------------
// densities

// One wave per run-away atom (the form for home cells too crowded to stage): rho from
// lattice sites in its window and from other run-aways; marks every lattice atom it
// pairs with (they need the reaction term).
// q: the atom's place in the sorted order.
template <bool kDealt>
__device__ __forceinline__ void runaway_rho_one(const State &S, const Scratch &sc, const Geom &g,
                                                const Tables<double> &T, int r, int q, int lane) {
    const int win = g.win, win3 = win * win * win;
    {
        const double x[3] = {S.r_x[r], S.r_y[r], S.r_z[r]};
        const int lo[3] = {window_lo(x[0] * g.inv_a, g.reach), window_lo(x[1] * g.inv_a, g.reach),
                           window_lo(x[2] * g.inv_a, g.reach)};
        double acc = 0.0;
        for (int c = lane; c < 2 * win3; c += 64) {
            const int p = c >= win3 ? 1 : 0;
            const int rem = c - p * win3;
            const int cx = lo[0] + rem % win, cy = lo[1] + (rem / win) % win, cz = lo[2] + rem / (win * win);
            const int64_t s = (int64_t)p * g.ncell +
                              ((int64_t)wrap_near(cz, g.nz) * g.ny + wrap_near(cy, g.ny)) * g.nx +
                              wrap_near(cx, g.nx);
            const double ux = S.ux[s];
            if (ux > VACANT_TEST) continue;
            const double u[3] = {ux, S.uy[s], S.uz[s]};
            double d[3];
            lat_sep(cx, cy, cz, p, u, x, g.a, d);
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < g.rc2) {
                acc += f_val(sqrt(r2), T);
                atomicOr(&sc.mark[s >> 5], 1u << (s & 31));  // listed in site order by k_mark_emit
            }
        }
        for_runaway_neighbours<kDealt>(x, r, lane, g.rc2, S, sc, g,
                               [&](int, const double *, double r2) { acc += f_val(sqrt(r2), T); });
        acc = wave_sum64(acc);
        if (lane == 0) {
            double Fv;
            bool beyond = false;
            const double d = emb_any<double>(acc, T.emb, T.em, Fv, beyond);
            S.r_rho[r] = acc;
            S.r_fp[r] = d;
            sc.sfp[q] = d;
            S.r_e[2 * r] = Fv;
            if (beyond) atomicAdd(&sc.cnt->range_viol, 1u);
        }
    }
}

// The float32 band pairs of lattice atom s, one team lane per stencil entry (entries
// cell, cell + AFF_TEAM, ...): for each pair whose float32 r^2 fell within RC_BAND_Q of
// rc^2 and on the other side of rc than in float64, iterate f (the float32 window form
// the density pass used, at the window's last node where float32 put r past it).
// Returns this lane's correction of the density (Eq. eam_base: a pair counts iff r < rc).
// The force-pass counterpart, near_pair_fix, follows the same steps.
template <class Body>
__device__ __forceinline__ void for_band_flips(const State &S, const Geom &g, const NearFix32 &nf, int64_t s,
                                               const int c[3], int p, int cell, Body body) {
    const float uix = (float)S.ux[s], uiy = (float)S.uy[s], uiz = (float)S.uz[s];
    for (int k = cell; k < nf.K; k += AFF_TEAM) {
        const NearEntry &e = nf.nt->st[p][k];
        const int64_t j = offset_site(c[0], c[1], c[2], p, e, g.nx, g.ny, g.nz, g.ncell);
        const float dx = ((float)S.ux[j] - uix) + (float)e.ox;
        const float dy = ((float)S.uy[j] - uiy) + (float)e.oy;
        const float dz = ((float)S.uz[j] - uiz) + (float)e.oz;
        const float r2 = pair_r2_f32(dx, dy, dz);
        if (!(fabsf(r2 - nf.rc2) < RC_BAND_Q)) continue;
        float t;
        int sg;
        bool in32;
        if (nf.node_cut) {
            sg = win_seg<true>(win_pos(r2, nf.inv_hq, nf.pcq), nf.nwin, t);
            in32 = sg < nf.nwin;
        } else {
            sg = win_seg<false>(win_pos(r2, nf.inv_hq, nf.pcq), nf.nwin, t);
            in32 = r2 < nf.rc2;
        }
        const bool in64 = pair_in_rc64(S.ux, S.uy, S.uz, s, c[0], c[1], c[2], p, e, g.nx, g.ny, g.nz, g.ncell,
                                       nf.nt->rc2);
        if (in32 == in64) continue;
        const bool past = sg >= nf.nwin;  // float32 r at or past the last node: the node's record at t = 1
        body(j, past ? nf.nwin - 1 : sg, past ? 1.0f : t, in64 ? 1.0 : -1.0, dx, dy, dz, r2);
    }
}

__device__ __forceinline__ double near_rho_fix(const State &S, const Geom &g, const NearFix32 &nf, int64_t s,
                                               const int c[3], int p, int cell) {
    double acc = 0.0;
    for_band_flips(S, g, nf, s, c, p, cell,
                   [&](int64_t, int sg, float t, double sgn, float, float, float, float) {
                       const float2 cf = nf.frec[sg];
                       acc += sgn * (double)(cf.y * t + cf.x);
                   });
    return acc;
}

// Lattice atoms within rc of run-aways: add the run-away terms to rho, refresh F'.
// emb: the embedding network of the learned form (an empty range on other handles).
// q: index into the affected list; cell: this lane's place in its team of AFF_TEAM.
template <typename Real>
__device__ __forceinline__ void affected_rho_one(const State &S, const Scratch &sc, const Geom &g,
                                                 const Tables<double> &T, const Tables<Real> &TL,
                                                 const MlpNet &emb, const NearFix32 &nf, int q, int cell) {
    {
        const int64_t s = sc.affected[q];
        const int p = s >= g.ncell ? 1 : 0;
        const int64_t c = s - p * g.ncell;
        const int cj[3] = {(int)(c % g.nx), (int)((c / g.nx) % g.ny), (int)(c / ((int64_t)g.nx * g.ny))};
        const double u[3] = {S.ux[s], S.uy[s], S.uz[s]};
        double xj[3];
        site_pos(cj[0], cj[1], cj[2], p, g.a, xj);
        for (int k = 0; k < 3; ++k) xj[k] = wrap_coord(xj[k] + u[k], g.L[k]);
        double acc = 0.0;
        for_runaways_around<AFF_TEAM, 4>(xj, cell, sc, g, [&](int, const double *xo) {
            double d[3], r2;
            if (affected_pair(xo, cj, p, u, g, d, r2)) acc += f_val(sqrt(r2), T);
        });
        if (nf.frec) acc += near_rho_fix(S, g, nf, s, cj, p, cell);
        acc = team_sum32(acc);
        if (cell == 0) {
            Real *rho = (Real *)S.rho;
            Real *fp = (Real *)S.fp;
            const Real rj = rho[s] + (Real)acc;
            rho[s] = rj;
            Real Fv;
            bool beyond = false;
            if (mlp_serves(emb, (float)rj)) {
                float ge, dge;
                mlp_eval_lane(emb, (float)rj, ge, dge);
                fp[s] = (Real)dge;
            } else {
                fp[s] = emb_any<Real>(rj, TL.emb, TL.em, Fv, beyond);
            }
            if (beyond) atomicAdd(&sc.cnt->range_viol, 1u);
        }
    }
}

__device__ __forceinline__ int affected_count(const Scratch &sc) {
    const int na = sc.cnt->n_affected;
    return na < sc.affected_cap ? na : (int)sc.affected_cap;
}

template <typename Real>
__device__ __forceinline__ void affected_rho_body(State S, Scratch sc, Geom g, Tables<double> T,
                                                  Tables<Real> TL, MlpNet emb, const NearFix32 &nf) {
    const int na = affected_count(sc);
    const int cell = threadIdx.x & (AFF_TEAM - 1);
    const int nteams = gridDim.x * (AFF_THREADS / AFF_TEAM);
    for (int q = (blockIdx.x * AFF_THREADS + threadIdx.x) / AFF_TEAM; q < na; q += nteams)
        affected_rho_one<Real>(S, sc, g, T, TL, emb, nf, q, cell);
}

template <typename Real>
__global__ __launch_bounds__(AFF_THREADS) void k_affected_rho(State S, Scratch sc, Geom g, Tables<double> T,
                                                              Tables<Real> TL, MlpNet emb, NearFix32 nf) {
    affected_rho_body<Real>(S, sc, g, T, TL, emb, nf);
}


// ---------------------------------------------------------------------------
// forces

template <bool kDealt>
__device__ __forceinline__ void runaway_force_one(const State &S, const Scratch &sc, const Geom &g,
                                                  const Tables<double> &T, int real_is_f32, int energy, int r,
                                                  int lane) {
    const int win = g.win, win3 = win * win * win;
    {
        const double x[3] = {S.r_x[r], S.r_y[r], S.r_z[r]};
        const double fpr = S.r_fp[r];
        const int lo[3] = {window_lo(x[0] * g.inv_a, g.reach), window_lo(x[1] * g.inv_a, g.reach),
                           window_lo(x[2] * g.inv_a, g.reach)};
        double fx = 0.0, fy = 0.0, fz = 0.0, ep = 0.0;
        for (int c = lane; c < 2 * win3; c += 64) {
            const int p = c >= win3 ? 1 : 0;
            const int rem = c - p * win3;
            const int cx = lo[0] + rem % win, cy = lo[1] + (rem / win) % win, cz = lo[2] + rem / (win * win);
            const int64_t s = (int64_t)p * g.ncell +
                              ((int64_t)wrap_near(cz, g.nz) * g.ny + wrap_near(cy, g.ny)) * g.nx +
                              wrap_near(cx, g.nx);
            const double ux = S.ux[s];
            if (ux > VACANT_TEST) continue;
            const double u[3] = {ux, S.uy[s], S.uz[s]};
            double d[3];
            lat_sep(cx, cy, cz, p, u, x, g.a, d);
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < g.rc2) {
                const double rr = sqrt(r2);
                double df, dphi, phi;
                fp_phi(rr, T, df, dphi, phi);
                const double fpj = real_is_f32 ? (double)((const float *)S.fp)[s] : ((const double *)S.fp)[s];
                const double sc_ = ((fpr + fpj) * df + dphi) / rr;
                fx += sc_ * d[0];
                fy += sc_ * d[1];
                fz += sc_ * d[2];
                ep += phi;  // lattice partner has no other record of this pair's energy
            }
        }
        for_runaway_neighbours<kDealt>(x, r, lane, g.rc2, S, sc, g, [&](int o, const double *d, double r2) {
            const double rr = sqrt(r2);
            double df, dphi, phi;
            fp_phi(rr, T, df, dphi, phi);
            const double sc_ = ((fpr + S.r_fp[o]) * df + dphi) / rr;
            fx += sc_ * d[0];
            fy += sc_ * d[1];
            fz += sc_ * d[2];
            ep += 0.5 * phi;
        });
        fx = wave_sum64(fx);
        fy = wave_sum64(fy);
        fz = wave_sum64(fz);
        ep = wave_sum64(ep);
        if (lane == 0) {
            S.r_fx[r] = fx;
            S.r_fy[r] = fy;
            S.r_fz[r] = fz;
            if (energy) S.r_e[2 * r + 1] = ep;
        }
    }
}

// ---------------------------------------------------------------------------
// Run-away sums by coarse cell.
//
// A block takes one coarse cell that holds run-aways (the home cell) and stages in LDS
// what its atoms pair with: the run-aways of the (up to) 27 cells around it, from the
// sorted copies, and the slotted lattice atoms of one lattice window that contains every
// home atom's own search window.  RC_SPLIT lanes serve one home atom: lane k takes the
// staged entries k, k + RC_SPLIT, ... in order, lattice atoms first, then run-aways, and
// the lanes' sums meet in a fixed butterfly.  Each pair's separation is formed as in the
// per-atom form (lat_sep from the atom's own window for a lattice partner, min_image3 of
// the difference for a run-away partner), so the lattice side's reaction terms still see
// the same pair.  A cell whose neighbourhood exceeds the staging capacities is served by
// the per-atom form, one wave per home atom.  Which form serves an atom depends only on
// the state, so results do not depend on how cells are dealt out.
constexpr int RC_THREADS = 256;
constexpr int RC_SPLIT = 16;
constexpr int RC_HOME = RC_THREADS / RC_SPLIT;
constexpr int RC_CAND = 512;  // run-away partners staged per home cell
constexpr int RC_LAT = 448;   // slotted lattice atoms staged per home cell
// Blocks per CU the cell-staged passes are compiled for.  A cell's staging is a few
// dependent memory round trips for about a dozen home atoms, so the passes gain from
// more cells in flight: 5 density blocks (96 VGPRs, 31 KB of LDS each) and 4 force
// blocks (127 VGPRs, 39 KB) instead of the 4 and 3 that 126 and 147 VGPRs and the
// larger capacities (640 / 608) allowed.
constexpr int RC_RHO_BLOCKS = 5;
constexpr int RC_FORCE_BLOCKS = 4;

template <bool FORCE>
struct CellStage {
    double cx[RC_CAND], cy[RC_CAND], cz[RC_CAND];
    double cfp[FORCE ? RC_CAND : 1];  // F' of the run-away partners
    int32_t co[RC_CAND];              // their list indices
    double lx[RC_LAT], ly[RC_LAT], lz[RC_LAT];  // displacements of the lattice partners
    double lfp[FORCE ? RC_LAT : 1];
    int64_t ls[RC_LAT];               // their storage indices
    uint32_t lw[RC_LAT];              // window offsets x | y << 8 | z << 16, parity << 24
    int32_t cstart[27], cpre[28];
    int32_t wcnt[RC_THREADS / 64];
};

// The lattice window of home cell c along one axis: cells [lo, lo + w) (w <= n) contain
// the search window [window_lo(q), window_lo(q) + win) of every q = x / a with x in the
// cell (the coarse cell spans n / nc lattice cells; the margin absorbs rounding of x / a).
__device__ __forceinline__ void cell_window(int c, int n, int nc, const Geom &g, int &lo, int &w) {
    const double span = (double)n / (double)nc;
    lo = window_lo((double)c * span - 1e-3, g.reach);
    const int hi = window_lo((double)(c + 1) * span + 1e-3, g.reach) + g.win;
    w = hi - lo < n ? hi - lo : n;
}

__device__ __forceinline__ double split_sum(double v) {
    // fixed butterfly over the RC_SPLIT lanes of one home atom
    for (int o = RC_SPLIT / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, RC_SPLIT);
    return v;
}

// Stages the home cell whose sorted run-aways start at hs.  Returns false (nothing
// usable staged) when its partners exceed the capacities; every thread of the block
// calls it and gets the same answer.  The loads are grouped so that a cell costs a few
// dependent memory round trips: the window's occupancy words and the neighbour cells'
// stretches together, then every partner's data together.
constexpr int RC_WIN_BATCHES = 4;  // window sites examined per thread per round

template <bool FORCE>
__device__ bool stage_cell(const State &S, const Scratch &sc, const Geom &g, int real_is_f32, int hs,
                           CellStage<FORCE> &st, int &n_cand, int &n_lat, int wlo[3], int ww[3]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t key = sc.skey[hs];
    const int hc[3] = {key % g.nc[0], (key / g.nc[0]) % g.nc[1], key / (g.nc[0] * g.nc[1])};
    const int n3[3] = {g.nx, g.ny, g.nz};
    for (int k = 0; k < 3; ++k) cell_window(hc[k], n3[k], g.nc[k], g, wlo[k], ww[k]);
    const bool wide = ww[0] > 255 || ww[1] > 255 || ww[2] > 255;
    const int w01 = ww[0] * ww[1], w012 = w01 * ww[2];
    const int nwin = wide ? 0 : 2 * w012;

    // round 1 of the window's occupancy words, issued before the cell look-ups
    auto site_of = [&](int w, uint32_t &pack) -> int64_t {
        const int p = w >= w012 ? 1 : 0;
        const int rem = w - p * w012;
        const int ox = rem % ww[0], oy = (rem / ww[0]) % ww[1], oz = rem / w01;
        pack = (uint32_t)ox | ((uint32_t)oy << 8) | ((uint32_t)oz << 16) | ((uint32_t)p << 24);
        return (int64_t)p * g.ncell +
               ((int64_t)wrap_near(wlo[2] + oz, g.nz) * g.ny + wrap_near(wlo[1] + oy, g.ny)) * g.nx +
               wrap_near(wlo[0] + ox, g.nx);
    };
    double ux[RC_WIN_BATCHES];
    int64_t ws[RC_WIN_BATCHES];
    uint32_t wp[RC_WIN_BATCHES];
    auto load_round = [&](int g0) {
#pragma unroll
        for (int b = 0; b < RC_WIN_BATCHES; ++b) {
            const int w = g0 + b * RC_THREADS + tid;
            ux[b] = 2.0 * VACANT_TEST;
            ws[b] = 0;
            wp[b] = 0;
            if (w < nwin) {
                ws[b] = site_of(w, wp[b]);
                ux[b] = S.ux[ws[b]];
            }
        }
    };
    load_round(0);

    if (wave == 0) {
        int cnt = 0;
        if (lane < 27) {
            int cx[3], cy[3], cz[3];
            const int ax = lane % 3, ay = (lane / 3) % 3, az = lane / 9;
            if (ax < axis_cells(hc[0], g.nc[0], cx) && ay < axis_cells(hc[1], g.nc[1], cy) &&
                az < axis_cells(hc[2], g.nc[2], cz)) {
                const int32_t nk = (cz[az] * g.nc[1] + cy[ay]) * g.nc[0] + cx[ax];
                const int c0 = sc.cell_s[nk];
                st.cstart[lane] = c0;
                cnt = sc.cell_s[nk + 1] - c0;
            }
        }
        int incl = cnt;
        for (int o = 1; o < 32; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (lane < 27) st.cpre[lane + 1] = incl;
        if (lane == 0) st.cpre[0] = 0;
    }

    // lattice window, compacted in window order (sublattice, z, y, x)
    int base = 0;
    for (int g0 = 0; g0 < nwin; g0 += RC_WIN_BATCHES * RC_THREADS) {
        if (g0 > 0) load_round(g0);
#pragma unroll
        for (int b = 0; b < RC_WIN_BATCHES; ++b) {
            const bool occ = !(ux[b] > VACANT_TEST);
            const uint64_t m = __ballot(occ);
            if (lane == 0) st.wcnt[wave] = __popcll(m);
            __syncthreads();
            int before = base, total = 0;
            for (int k = 0; k < RC_THREADS / 64; ++k) {
                if (k < wave) before += st.wcnt[k];
                total += st.wcnt[k];
            }
            const int idx = before + __popcll(m & ((1ull << lane) - 1ull));
            if (occ && idx < RC_LAT) {
                st.lx[idx] = ux[b];
                st.ls[idx] = ws[b];
                st.lw[idx] = wp[b];
            }
            base += total;
            __syncthreads();  // wcnt is rewritten by the next batch
        }
        if (base > RC_LAT) break;
    }
    n_lat = base;
    n_cand = st.cpre[27];  // visible: the batches above passed barriers (at least one: nwin > 0)
    if (wide || n_cand > RC_CAND || n_lat > RC_LAT) return false;

    // every partner's data in one round: the lattice atoms' other components (and F'),
    // the run-aways in cell order, each cell's stretch in sorted order
    for (int e = tid; e < n_lat; e += RC_THREADS) {
        const int64_t si = st.ls[e];
        st.ly[e] = S.uy[si];
        st.lz[e] = S.uz[si];
        if (FORCE) st.lfp[e] = real_is_f32 ? (double)((const float *)S.fp)[si] : ((const double *)S.fp)[si];
    }
    for (int e = tid; e < n_cand; e += RC_THREADS) {
        int k = 0;  // the cell holding entry e: how many cells end at or before e (5 steps)
        for (int step = 16; step > 0; step >>= 1)
            if (k + step <= 27 && st.cpre[k + step] <= e) k += step;
        const int q = st.cstart[k] + (e - st.cpre[k]);
        st.cx[e] = sc.srx[q];
        st.cy[e] = sc.sry[q];
        st.cz[e] = sc.srz[q];
        st.co[e] = sc.sidx[q];
        if (FORCE) st.cfp[e] = sc.sfp[q];
    }
    __syncthreads();
    return true;
}

// Lattice partner e of a home atom with search window lo[]: its cell in that window
// (false if outside), as the per-atom form enumerates it.
__device__ __forceinline__ bool staged_site(uint32_t pack, const int wlo[3], const int ww[3], const int lo[3],
                                            const Geom &g, int cc[3], int &p) {
    const int n3[3] = {g.nx, g.ny, g.nz};
    for (int k = 0; k < 3; ++k) {
        int t = wlo[k] + (int)((pack >> (8 * k)) & 0xffu) - lo[k];  // in (-ww, ww), ww <= n
        t = t < 0 ? t + n3[k] : t;
        if (t >= g.win) return false;
        cc[k] = lo[k] + t;
    }
    p = (int)(pack >> 24);
    return true;
}

// Separation of staged lattice partner e from a home atom at x with search window lo
// (false if the partner lies outside that window), and of staged run-away partner e.
template <bool FORCE>
__device__ __forceinline__ bool lat_pair(const CellStage<FORCE> &st, int e, const int wlo[3], const int ww[3],
                                         const int lo[3], const double x[3], const Geom &g, double d[3],
                                         double &r2) {
    int cc[3], p;
    if (!staged_site(st.lw[e], wlo, ww, lo, g, cc, p)) return false;
    const double u[3] = {st.lx[e], st.ly[e], st.lz[e]};
    lat_sep(cc[0], cc[1], cc[2], p, u, x, g.a, d);
    r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    return true;
}

template <bool FORCE>
__device__ __forceinline__ void run_pair(const CellStage<FORCE> &st, int e, const double x[3], const Geom &g,
                                         double d[3], double &r2) {
    d[0] = st.cx[e] - x[0];
    d[1] = st.cy[e] - x[1];
    d[2] = st.cz[e] - x[2];
    min_image3(d, g);
    r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

// A lane's staged entries are e = k + RC_SPLIT i.  The pairs are found first (bit i of
// a mask per kind, at most 64 entries per lane: RC_LAT and RC_CAND are below 64 RC_SPLIT),
// then taken up in groups whose table records are loaded together, lowest i first, so
// the sums keep the entry order.
static_assert(RC_LAT <= 64 * RC_SPLIT && RC_CAND <= 64 * RC_SPLIT, "one 64-bit mask per lane and kind");

// The next (up to) G entries of mask m: e[t] = k + RC_SPLIT * bit; slots past the last
// repeat the first entry and are marked invalid.
template <int G>
__device__ __forceinline__ void take_group(uint64_t &m, int k, int e[G], bool v[G]) {
#pragma unroll
    for (int t = 0; t < G; ++t) {
        v[t] = m != 0;
        e[t] = v[t] ? k + RC_SPLIT * __builtin_ctzll(m) : e[0];
        m &= m - 1;
    }
}

constexpr int RC_RHO_GROUP = 4;    // f records in flight per lane
constexpr int RC_FORCE_GROUP = 1;  // f', phi' and phi records in flight per lane (2 spilled at 4 blocks per CU)

__device__ __forceinline__ void runaway_rho_cell(const State &S, const Scratch &sc, const Geom &g,
                                                 const Tables<double> &T, int hs, CellStage<false> &st) {
    int n_cand = 0, n_lat = 0, wlo[3], ww[3];
    const int nh = sc.cell_s[sc.skey[hs] + 1] - hs;
    if (!stage_cell<false>(S, sc, g, 0, hs, st, n_cand, n_lat, wlo, ww)) {
        const int lane = threadIdx.x & 63;
        for (int j = threadIdx.x >> 6; j < nh; j += RC_THREADS / 64)
            runaway_rho_one<false>(S, sc, g, T, sc.sidx[hs + j], hs + j, lane);
        return;
    }
    const int k = threadIdx.x % RC_SPLIT;
    for (int hb = 0; hb < nh; hb += RC_HOME) {
        const int j = hb + (int)threadIdx.x / RC_SPLIT;
        const bool act = j < nh;
        double acc = 0.0;
        int o = -1;
        if (act) {
            const int q = hs + j;
            o = sc.sidx[q];
            const double x[3] = {sc.srx[q], sc.sry[q], sc.srz[q]};
            const int lo[3] = {window_lo(x[0] * g.inv_a, g.reach), window_lo(x[1] * g.inv_a, g.reach),
                               window_lo(x[2] * g.inv_a, g.reach)};
            uint64_t ml = 0, mc = 0;
            int i = 0;
            for (int e = k; e < n_lat; e += RC_SPLIT, ++i) {
                double d[3], r2;
                if (lat_pair(st, e, wlo, ww, lo, x, g, d, r2) && r2 < g.rc2) ml |= 1ull << i;
            }
            i = 0;
            for (int e = k; e < n_cand; e += RC_SPLIT, ++i) {
                if (st.co[e] == o) continue;
                double d[3], r2;
                run_pair(st, e, x, g, d, r2);
                if (r2 < g.rc2) mc |= 1ull << i;
            }
            while (ml) {
                int e[RC_RHO_GROUP];
                bool v[RC_RHO_GROUP];
                take_group<RC_RHO_GROUP>(ml, k, e, v);
                double f[RC_RHO_GROUP];
#pragma unroll
                for (int t = 0; t < RC_RHO_GROUP; ++t) {
                    double d[3], r2;
                    (void)lat_pair(st, e[t], wlo, ww, lo, x, g, d, r2);
                    f[t] = f_val(sqrt(r2), T);
                }
#pragma unroll
                for (int t = 0; t < RC_RHO_GROUP; ++t)
                    if (v[t]) {
                        acc += f[t];
                        const int64_t s = st.ls[e[t]];
                        atomicOr(&sc.mark[s >> 5], 1u << (s & 31));  // listed in site order by k_mark_emit
                    }
            }
            while (mc) {
                int e[RC_RHO_GROUP];
                bool v[RC_RHO_GROUP];
                take_group<RC_RHO_GROUP>(mc, k, e, v);
                double f[RC_RHO_GROUP];
#pragma unroll
                for (int t = 0; t < RC_RHO_GROUP; ++t) {
                    double d[3], r2;
                    run_pair(st, e[t], x, g, d, r2);
                    f[t] = f_val(sqrt(r2), T);
                }
#pragma unroll
                for (int t = 0; t < RC_RHO_GROUP; ++t)
                    if (v[t]) acc += f[t];
            }
        }
        acc = split_sum(acc);
        if (act && k == 0) {
            double Fv;
            bool beyond = false;
            const double d = emb_any<double>(acc, T.emb, T.em, Fv, beyond);
            S.r_rho[o] = acc;
            S.r_fp[o] = d;
            sc.sfp[hs + j] = d;
            S.r_e[2 * o] = Fv;
            if (beyond) atomicAdd(&sc.cnt->range_viol, 1u);
        }
    }
}

// (f'(r) (F'_i + F'_j) + phi'(r)) / r times the separation, and phi, of one pair.
__device__ __forceinline__ void pair_force(const double d[3], double r2, double fpsum, const Tables<double> &T,
                                           double &fx, double &fy, double &fz, double &phi) {
    const double rr = sqrt(r2);
    double df, dphi;
    fp_phi(rr, T, df, dphi, phi);
    const double sc_ = (fpsum * df + dphi) / rr;
    fx = sc_ * d[0];
    fy = sc_ * d[1];
    fz = sc_ * d[2];
}

__device__ __forceinline__ void runaway_force_cell(const State &S, const Scratch &sc, const Geom &g,
                                                   const Tables<double> &T, int real_is_f32, int energy, int hs,
                                                   CellStage<true> &st) {
    int n_cand = 0, n_lat = 0, wlo[3], ww[3];
    const int nh = sc.cell_s[sc.skey[hs] + 1] - hs;
    if (!stage_cell<true>(S, sc, g, real_is_f32, hs, st, n_cand, n_lat, wlo, ww)) {
        const int lane = threadIdx.x & 63;
        for (int j = threadIdx.x >> 6; j < nh; j += RC_THREADS / 64)
            runaway_force_one<false>(S, sc, g, T, real_is_f32, energy, sc.sidx[hs + j], lane);
        return;
    }
    const int k = threadIdx.x % RC_SPLIT;
    for (int hb = 0; hb < nh; hb += RC_HOME) {
        const int j = hb + (int)threadIdx.x / RC_SPLIT;
        const bool act = j < nh;
        double fx = 0.0, fy = 0.0, fz = 0.0, ep = 0.0;
        int o = -1;
        if (act) {
            const int q = hs + j;
            o = sc.sidx[q];
            const double x[3] = {sc.srx[q], sc.sry[q], sc.srz[q]};
            const double fpr = sc.sfp[q];
            const int lo[3] = {window_lo(x[0] * g.inv_a, g.reach), window_lo(x[1] * g.inv_a, g.reach),
                               window_lo(x[2] * g.inv_a, g.reach)};
            uint64_t ml = 0, mc = 0;
            int i = 0;
            for (int e = k; e < n_lat; e += RC_SPLIT, ++i) {
                double d[3], r2;
                if (lat_pair(st, e, wlo, ww, lo, x, g, d, r2) && r2 < g.rc2) ml |= 1ull << i;
            }
            i = 0;
            for (int e = k; e < n_cand; e += RC_SPLIT, ++i) {
                if (st.co[e] == o) continue;
                double d[3], r2;
                run_pair(st, e, x, g, d, r2);
                if (r2 < g.rc2) mc |= 1ull << i;
            }
            while (ml) {
                int e[RC_FORCE_GROUP];
                bool v[RC_FORCE_GROUP];
                take_group<RC_FORCE_GROUP>(ml, k, e, v);
                double gx[RC_FORCE_GROUP], gy[RC_FORCE_GROUP], gz[RC_FORCE_GROUP], ph[RC_FORCE_GROUP];
#pragma unroll
                for (int t = 0; t < RC_FORCE_GROUP; ++t) {
                    double d[3], r2;
                    (void)lat_pair(st, e[t], wlo, ww, lo, x, g, d, r2);
                    pair_force(d, r2, fpr + st.lfp[e[t]], T, gx[t], gy[t], gz[t], ph[t]);
                }
#pragma unroll
                for (int t = 0; t < RC_FORCE_GROUP; ++t)
                    if (v[t]) {
                        fx += gx[t];
                        fy += gy[t];
                        fz += gz[t];
                        ep += ph[t];  // lattice partner has no other record of this pair's energy
                    }
            }
            while (mc) {
                int e[RC_FORCE_GROUP];
                bool v[RC_FORCE_GROUP];
                take_group<RC_FORCE_GROUP>(mc, k, e, v);
                double gx[RC_FORCE_GROUP], gy[RC_FORCE_GROUP], gz[RC_FORCE_GROUP], ph[RC_FORCE_GROUP];
#pragma unroll
                for (int t = 0; t < RC_FORCE_GROUP; ++t) {
                    double d[3], r2;
                    run_pair(st, e[t], x, g, d, r2);
                    pair_force(d, r2, fpr + st.cfp[e[t]], T, gx[t], gy[t], gz[t], ph[t]);
                }
#pragma unroll
                for (int t = 0; t < RC_FORCE_GROUP; ++t)
                    if (v[t]) {
                        fx += gx[t];
                        fy += gy[t];
                        fz += gz[t];
                        ep += 0.5 * ph[t];
                    }
            }
        }
        fx = split_sum(fx);
        fy = split_sum(fy);
        fz = split_sum(fz);
        ep = split_sum(ep);
        if (act && k == 0) {
            S.r_fx[o] = fx;
            S.r_fy[o] = fy;
            S.r_fz[o] = fz;
            if (energy) S.r_e[2 * o + 1] = ep;
        }
    }
}

// Run-aways of sparse cells: one wave each.
constexpr int LONE_WAVES = 4;

__global__ __launch_bounds__(64 * LONE_WAVES) void k_runaway_rho_lone(State S, Scratch sc, Geom g, Tables<double> T) {
    const int lane = threadIdx.x & 63;
    const int n = sc.cnt->n_lone;
    for (int i = blockIdx.x * LONE_WAVES + (threadIdx.x >> 6); i < n; i += gridDim.x * LONE_WAVES)
    {
        const int q = sc.loneq[i];
        runaway_rho_one<true>(S, sc, g, T, sc.sidx[q], q, lane);
    }
}

__global__ __launch_bounds__(64 * LONE_WAVES) void k_runaway_force_lone(State S, Scratch sc, Geom g,
                                                                        Tables<double> T, int real_is_f32,
                                                                        int energy) {
    const int lane = threadIdx.x & 63;
    const int n = sc.cnt->n_lone;
    for (int i = blockIdx.x * LONE_WAVES + (threadIdx.x >> 6); i < n; i += gridDim.x * LONE_WAVES)
        runaway_force_one<true>(S, sc, g, T, real_is_f32, energy, sc.sidx[sc.loneq[i]], lane);
}

__global__ __launch_bounds__(RC_THREADS, RC_RHO_BLOCKS) void k_runaway_rho_cells(State S, Scratch sc, Geom g, Tables<double> T) {
    __shared__ CellStage<false> st;
    const int n = sc.cnt->n_cells;
    for (int ci = blockIdx.x; ci < n; ci += gridDim.x) {
        __syncthreads();  // the previous cell's staging is no longer read
        runaway_rho_cell(S, sc, g, T, sc.cellq[ci], st);
    }
}

__global__ __launch_bounds__(RC_THREADS, RC_FORCE_BLOCKS) void k_runaway_force_cells(State S, Scratch sc, Geom g, Tables<double> T,
                                                                    int real_is_f32, int energy) {
    __shared__ CellStage<true> st;
    const int n = sc.cnt->n_cells;
    for (int ci = blockIdx.x; ci < n; ci += gridDim.x) {
        __syncthreads();
        runaway_force_cell(S, sc, g, T, real_is_f32, energy, sc.cellq[ci], st);
    }
}


// The force-pass counterpart of near_rho_fix: this lane's corrections of the force and
// of the pair energy (phi from the r-grid records, as the pass takes it).
__device__ __forceinline__ void near_pair_fix(const State &S, const Geom &g, const NearFix32 &nf, int64_t s,
                                              const int c[3], int p, int cell, double &ax, double &ay,
                                              double &az, double &ae) {
    const float *fpa = (const float *)S.fp;
    const float fpi = fpa[s];
    for_band_flips(S, g, nf, s, c, p, cell,
                   [&](int64_t j, int sg, float t, double sgn, float dx, float dy, float dz, float r2) {
                       const float4 rc_ = nf.rec[sg];
                       const float gf = rc_.y * t + rc_.x;  // f'(r) / r
                       const float gp = rc_.w * t + rc_.z;  // phi'(r) / r
                       const float sc_ = (fpi + fpa[j]) * gf + gp;
                       ax += sgn * (double)(sc_ * dx);
                       ay += sgn * (double)(sc_ * dy);
                       az += sgn * (double)(sc_ * dz);
                       const float pr = (__builtin_amdgcn_sqrtf(r2) - nf.fm.x0) * nf.fm.inv_h;
                       const int sr = max(0, min((int)pr, nf.fm.nseg - 1));
                       const float tr = pr - (float)sr;
                       const Q4<float> cp = nf.phi[sr];
                       ae += sgn * 0.5 * (double)(((cp.w * tr + cp.z) * tr + cp.y) * tr + cp.x);
                   });
}

// kick != 0: the force pass already applied the second half-kick with the lattice
// part of F; add the run-away part's kick here and record |v|^2 for the step statistics.
// nf.rec: also correct the float32 gather pass's cut-off decisions (near_pair_fix);
// energy: record the pair-energy correction in aff_e.
template <typename Real>
__device__ __forceinline__ void affected_force_one(const State &S, const Scratch &sc, const Geom &g,
                                                   const Tables<double> &T, int kick, double kf,
                                                   const NearFix32 &nf, int energy, int q, int cell) {
    const double hk = kick ? 0.5 * sc.scal[0] * kf : 0.0;
    {
        const int64_t s = sc.affected[q];
        const int p = s >= g.ncell ? 1 : 0;
        const int64_t c = s - p * g.ncell;
        const int cj[3] = {(int)(c % g.nx), (int)((c / g.nx) % g.ny), (int)(c / ((int64_t)g.nx * g.ny))};
        const double u[3] = {S.ux[s], S.uy[s], S.uz[s]};
        const double fpj = (double)((const Real *)S.fp)[s];
        double xj[3];
        site_pos(cj[0], cj[1], cj[2], p, g.a, xj);
        for (int k = 0; k < 3; ++k) xj[k] = wrap_coord(xj[k] + u[k], g.L[k]);
        double ax = 0.0, ay = 0.0, az = 0.0;
        for_runaways_around<AFF_TEAM, 4>(xj, cell, sc, g, [&](int o, const double *xo) {
            double d[3], r2;  // d = x_j - x_o
            if (!affected_pair(xo, cj, p, u, g, d, r2)) return;
            const double rr = sqrt(r2);
            double df, dphi, phi;
            fp_phi(rr, T, df, dphi, phi);
            const double sc_ = ((fpj + S.r_fp[o]) * df + dphi) / rr;
            ax -= sc_ * d[0];  // separation from j to the run-away is -d
            ay -= sc_ * d[1];
            az -= sc_ * d[2];
        });
        double ae = 0.0;
        if (nf.rec) near_pair_fix(S, g, nf, s, cj, p, cell, ax, ay, az, ae);
        ax = team_sum32(ax);
        ay = team_sum32(ay);
        az = team_sum32(az);
        if (energy) ae = team_sum32(ae);
        if (cell == 0) {
            if (energy) sc.aff_e[q] = ae;
            Real *fxa = (Real *)S.fx;
            Real *fya = (Real *)S.fy;
            Real *fza = (Real *)S.fz;
            fxa[s] = (Real)((double)fxa[s] + ax);
            fya[s] = (Real)((double)fya[s] + ay);
            fza[s] = (Real)((double)fza[s] + az);
            if (kick) {
                const double vx = S.vx[s] + hk * ax, vy = S.vy[s] + hk * ay, vz = S.vz[s] + hk * az;
                S.vx[s] = vx;
                S.vy[s] = vy;
                S.vz[s] = vz;
                sc.aff_v2[q] = vx * vx + vy * vy + vz * vz;
            }
            sc.mark[s >> 5] = 0u;  // every bit of a touched word belongs to an affected site
        }
    }
}

template <typename Real>
__device__ __forceinline__ void affected_force_body(State S, Scratch sc, Geom g, Tables<double> T, int kick,
                                                    double kf, const NearFix32 &nf, int energy) {
    const int na = affected_count(sc);
    const int cell = threadIdx.x & (AFF_TEAM - 1);
    const int nteams = gridDim.x * (AFF_THREADS / AFF_TEAM);
    for (int q = (blockIdx.x * AFF_THREADS + threadIdx.x) / AFF_TEAM; q < na; q += nteams)
        affected_force_one<Real>(S, sc, g, T, kick, kf, nf, energy, q, cell);
}

template <typename Real>
__global__ __launch_bounds__(AFF_THREADS) void k_affected_force(State S, Scratch sc, Geom g, Tables<double> T,
                                                                int kick, double kf, NearFix32 nf, int energy) {
    affected_force_body<Real>(S, sc, g, T, kick, kf, nf, energy);
}


// ---------------------------------------------------------------------------
// Run-away work of a batch as one list.  Run-aways gather in the few boxes whose
// cascades melt them, so a fixed share of blocks per box would leave those boxes to a
// handful of waves.  Instead item q of the list (a run-away, or an affected lattice
// atom) is item q - off[b] of box b, off[b] <= q < off[b + 1], and every wave of the
// grid takes items from the whole list.  Each item is computed exactly as in a
// single-box pass, so results do not depend on how the list is dealt out.

constexpr int FLAT_BLOCKS = 1024;  // off[] (at most BATCH_MAX_BOXES + 1 ints) is staged in LDS

// off[0] = 0, off[b + 1] = off[b] + items of box b; which = 0: coarse cells whose
// run-aways are summed by cell, 1: affected lattice atoms (capped at the list's capacity,
// as the passes over it are), 2: run-aways summed one by one.
__global__ __launch_bounds__(1024) void kb_flat_offsets(const BoxRef *__restrict__ boxes, int nbox, int which,
                                                        int32_t *__restrict__ off) {
    __shared__ int sw[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (threadIdx.x == 0) off[0] = 0;
    int carry = 0;
    for (int base = 0; base < nbox; base += 1024) {
        const int i = base + (int)threadIdx.x;
        int v = 0;
        if (i < nbox)
            v = which == 0 ? boxes[i].sc.cnt->n_cells
                           : (which == 1 ? affected_count(boxes[i].sc) : boxes[i].sc.cnt->n_lone);
        int incl = v;
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        if (lane == 63) sw[w] = incl;
        __syncthreads();
        int before = carry, total = 0;
        for (int k = 0; k < 16; ++k) {
            if (k < w) before += sw[k];
            total += sw[k];
        }
        if (i < nbox) off[i + 1] = before + incl;
        carry += total;
        __syncthreads();  // sw is rewritten by the next chunk
    }
}

// Stages off[0 .. nbox] in LDS; returns the list length.
__device__ __forceinline__ int stage_offsets(int *s_off, const int32_t *__restrict__ off, int nbox) {
    for (int i = threadIdx.x; i <= nbox; i += blockDim.x) s_off[i] = off[i];
    __syncthreads();
    return s_off[nbox];
}

// The box b with off[b] <= q < off[b + 1] (0 <= q < off[nbox]; boxes with no items are
// passed over because their two offsets are equal).
__device__ __forceinline__ int flat_box(const int *s_off, int nbox, int q) {
    int lo = 0, hi = nbox;  // off[lo] <= q < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_off[mid] <= q) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Run-aways of sparse cells, one wave per item, and of crowded cells, one block per
// item, as in the single-box passes.
__global__ __launch_bounds__(64 * LONE_WAVES) void kf_runaway_rho_lone(const BoxRef *__restrict__ boxes, int nbox,
                                                                       const int32_t *off, Tables<double> T) {
    extern __shared__ int s_off[];
    const int total = stage_offsets(s_off, off, nbox);
    const int lane = threadIdx.x & 63;
    for (int q = blockIdx.x * LONE_WAVES + (threadIdx.x >> 6); q < total; q += gridDim.x * LONE_WAVES) {
        const int b = __builtin_amdgcn_readfirstlane(flat_box(s_off, nbox, q));  // one item per wave
        const BoxRef &B = boxes[b];
        const int qs = B.sc.loneq[q - s_off[b]];
        runaway_rho_one<true>(B.S, B.sc, B.g, T, B.sc.sidx[qs], qs, lane);
    }
}

__global__ __launch_bounds__(64 * LONE_WAVES) void kf_runaway_force_lone(const BoxRef *__restrict__ boxes,
                                                                         int nbox, const int32_t *off,
                                                                         Tables<double> T, int energy) {
    extern __shared__ int s_off[];
    const int total = stage_offsets(s_off, off, nbox);
    const int lane = threadIdx.x & 63;
    for (int q = blockIdx.x * LONE_WAVES + (threadIdx.x >> 6); q < total; q += gridDim.x * LONE_WAVES) {
        const int b = __builtin_amdgcn_readfirstlane(flat_box(s_off, nbox, q));
        const BoxRef &B = boxes[b];
        runaway_force_one<true>(B.S, B.sc, B.g, T, 1, energy, B.sc.sidx[B.sc.loneq[q - s_off[b]]], lane);
    }
}

__global__ __launch_bounds__(RC_THREADS, RC_RHO_BLOCKS) void kf_runaway_rho(const BoxRef *__restrict__ boxes, int nbox,
                                                             const int32_t *off, Tables<double> T) {
    extern __shared__ int s_off[];
    __shared__ CellStage<false> st;
    const int total = stage_offsets(s_off, off, nbox);
    for (int q = blockIdx.x; q < total; q += gridDim.x) {
        const int b = flat_box(s_off, nbox, q);
        const BoxRef &B = boxes[b];
        __syncthreads();  // the previous cell's staging is no longer read
        runaway_rho_cell(B.S, B.sc, B.g, T, B.sc.cellq[q - s_off[b]], st);
    }
}

__global__ __launch_bounds__(RC_THREADS, RC_FORCE_BLOCKS) void kf_runaway_force(const BoxRef *__restrict__ boxes, int nbox,
                                                               const int32_t *off, Tables<double> T, int energy) {
    extern __shared__ int s_off[];
    __shared__ CellStage<true> st;
    const int total = stage_offsets(s_off, off, nbox);
    for (int q = blockIdx.x; q < total; q += gridDim.x) {
        const int b = flat_box(s_off, nbox, q);
        const BoxRef &B = boxes[b];
        __syncthreads();
        runaway_force_cell(B.S, B.sc, B.g, T, 1, energy, B.sc.cellq[q - s_off[b]], st);
    }
}

// Affected atoms: one team of AFF_TEAM lanes per item, as in the single-box pass (the
// two teams of a wave may serve different boxes).
__global__ __launch_bounds__(AFF_THREADS) void kf_affected_rho(const BoxRef *__restrict__ boxes, int nbox,
                                                               const int32_t *off, Tables<double> T,
                                                               Tables<float> TL, NearFix32 nf) {
    extern __shared__ int s_off[];
    const int total = stage_offsets(s_off, off, nbox);
    const int cell = threadIdx.x & (AFF_TEAM - 1);
    const int nteams = gridDim.x * (AFF_THREADS / AFF_TEAM);
    for (int q = (blockIdx.x * AFF_THREADS + threadIdx.x) / AFF_TEAM; q < total; q += nteams) {
        const int b = flat_box(s_off, nbox, q);
        const BoxRef &B = boxes[b];
        affected_rho_one<float>(B.S, B.sc, B.g, T, TL, MlpNet{}, nf, q - s_off[b], cell);
    }
}

__global__ __launch_bounds__(AFF_THREADS) void kf_affected_force(const BoxRef *__restrict__ boxes, int nbox,
                                                                 const int32_t *off, Tables<double> T, double kf,
                                                                 NearFix32 nf, int energy) {
    extern __shared__ int s_off[];
    const int total = stage_offsets(s_off, off, nbox);
    const int cell = threadIdx.x & (AFF_TEAM - 1);
    const int nteams = gridDim.x * (AFF_THREADS / AFF_TEAM);
    for (int q = (blockIdx.x * AFF_THREADS + threadIdx.x) / AFF_TEAM; q < total; q += nteams) {
        const int b = flat_box(s_off, nbox, q);
        const BoxRef &B = boxes[b];
        affected_force_one<float>(B.S, B.sc, B.g, T, 1, kf, nf, energy, q - s_off[b], cell);
    }
}

// ---------------------------------------------------------------------------
// The affected list: every lattice atom a run-away atom paired with, in ascending
// site order, compacted from the mark bitmap (count, scan, emit), so every pass
// over it and every sum taken along it runs in a fixed order.

__device__ __forceinline__ int block_exclusive_scan(int v, int *sh_waves, int &total) {
    // 256 lanes = 4 waves
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int n = __shfl_up(incl, o, 64);
        if (lane >= o) incl += n;
    }
    if (lane == 63) sh_waves[w] = incl;
    __syncthreads();
    int off = 0;
    total = 0;
    for (int k = 0; k < MARK_THREADS / 64; ++k) {
        if (k < w) off += sh_waves[k];
        total += sh_waves[k];
    }
    return off + incl - v;
}

// The bitmap is padded with zero words to whole blocks, so no lane tests bounds.
__device__ __forceinline__ void load_mark_words(const Scratch &sc, uint32_t (&m)[MARK_WORDS], int &c) {
    const int64_t w0 = ((int64_t)blockIdx.x * MARK_THREADS + threadIdx.x) * MARK_WORDS;
    const uint4 *p = reinterpret_cast<const uint4 *>(sc.mark + w0);
    const uint4 a = p[0], b = p[1];
    m[0] = a.x, m[1] = a.y, m[2] = a.z, m[3] = a.w;
    m[4] = b.x, m[5] = b.y, m[6] = b.z, m[7] = b.w;
    c = 0;
#pragma unroll
    for (int k = 0; k < MARK_WORDS; ++k) c += __popc(m[k]);
}

__device__ __forceinline__ void mark_count_body(Scratch sc) {
    __shared__ int shw[MARK_THREADS / 64];
    // a batched grid sized for a larger box (marks come from run-aways and, in the
    // float32 gather form, from the density pass's cut-off band: no early exit on n_run)
    if ((int)blockIdx.x >= sc.mark_nblk) return;
    uint32_t m[MARK_WORDS];
    int c, total;
    load_mark_words(sc, m, c);
    block_exclusive_scan(c, shw, total);
    if (threadIdx.x == 0) sc.mark_blk[blockIdx.x] = total;
}

__global__ __launch_bounds__(MARK_THREADS) void k_mark_count(Scratch sc) {
    mark_count_body(sc);
}

__global__ __launch_bounds__(MARK_THREADS) void kb_mark_count(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    mark_count_body(B.sc);
}


__device__ __forceinline__ void mark_scan_body(Scratch sc, int nblk) {
    __shared__ int64_t base_sh;
    __shared__ int wsum[1024 / 64];
    if (threadIdx.x == 0) base_sh = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int c0 = 0; c0 < nblk; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const int v = i < nblk ? sc.mark_blk[i] : 0;
        int incl = v;
        for (int o = 1; o < 64; o <<= 1) {
            const int n = __shfl_up(incl, o, 64);
            if (lane >= o) incl += n;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int64_t off = base_sh;
        int64_t tot = 0;
        for (int k = 0; k < 1024 / 64; ++k) {
            if (k < w) off += wsum[k];
            tot += wsum[k];
        }
        if (i < nblk) sc.mark_off[i] = off + incl - v;
        __syncthreads();
        if (threadIdx.x == 0) base_sh += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t n = base_sh;
        if (n > sc.affected_cap) sc.cnt->overflow = 1;
        sc.cnt->n_affected = (int32_t)(n < sc.affected_cap ? n : sc.affected_cap);
    }
}

__global__ __launch_bounds__(1024) void k_mark_scan(Scratch sc, int nblk) {
    mark_scan_body(sc, nblk);
}

__global__ __launch_bounds__(1024) void kb_mark_scan(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    mark_scan_body(B.sc, B.sc.mark_nblk);
}


__device__ __forceinline__ void mark_emit_body(Scratch sc) {
    __shared__ int shw[MARK_THREADS / 64];
    if ((int)blockIdx.x >= sc.mark_nblk) return;
    uint32_t m[MARK_WORDS];
    int c, total;
    load_mark_words(sc, m, c);
    int64_t pos = sc.mark_off[blockIdx.x] + block_exclusive_scan(c, shw, total);
    if (c == 0) return;
    const int64_t w0 = ((int64_t)blockIdx.x * MARK_THREADS + threadIdx.x) * MARK_WORDS;
    for (int k = 0; k < MARK_WORDS; ++k) {
        uint32_t w = m[k];
        while (w) {
            const int b = __ffs(w) - 1;
            w &= w - 1u;
            if (pos < sc.affected_cap) sc.affected[pos] = (int32_t)((w0 + k) * 32 + b);
            ++pos;
        }
    }
}

__global__ __launch_bounds__(MARK_THREADS) void k_mark_emit(Scratch sc) {
    mark_emit_body(sc);
}

__global__ __launch_bounds__(MARK_THREADS) void kb_mark_emit(const BoxRef *__restrict__ boxes) {
    const BoxRef &B = boxes[blockIdx.y];
    mark_emit_body(B.sc);
}


// ---------------------------------------------------------------------------
// launchers

static Tables<double> t64_of(misa_lattice *h) {
    Tables<double> T;
    T.f = h->t64.f;
    T.force = h->t64.force;
    T.phi = h->t64.phi;
    T.emb = h->t64.emb;
    T.fm = h->t64.fm;
    T.em = h->t64.em;
    return T;
}

static Tables<float> t32_of(misa_lattice *h) {
    Tables<float> T;
    T.f = h->t32.f;
    T.force = h->t32.force;
    T.phi = h->t32.phi;
    T.emb = h->t32.emb;
    T.fm = h->t32.fm;
    T.em = h->t32.em;
    return T;
}

// Blocks of the cell-staged run-away passes on one box: as many as stay resident, since
// the number of occupied cells is known on the device only.
template <typename Kernel>
static int cell_grid(const misa_lattice *h, Kernel k) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, RC_THREADS, 0) != hipSuccess) per_cu = 0;
    return std::max(SMALL_GRID, per_cu * h->n_cu);
}

hipError_t launch_rehash(misa_lattice *h) {
    hipStream_t st = h->stream;
    hipLaunchKernelGGL(k_sort, dim3(1), dim3(SORT_THREADS), 0, st, h->sc.sortbuf, h->sc.cnt, h->rcap, h->sc.l_id,
                       h->sc.scal);
    hipLaunchKernelGGL(k_claim, dim3(SMALL_GRID), dim3(256), 0, st, h->S, h->sc, h->g);
    hipLaunchKernelGGL(k_settle, dim3(SMALL_GRID), dim3(256), 0, st, h->S, h->sc, h->g);
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, st, h->S, h->sc);
    return hipGetLastError();
}

hipError_t launch_runaway_build(misa_lattice *h) {
    hipStream_t st = h->stream;
    const int nb = h->sc.cs_nblk;
    hipLaunchKernelGGL(k_cell_count, dim3(SMALL_GRID), dim3(256), 0, st, h->S, h->sc, h->g);
    hipLaunchKernelGGL(k_cell_sum, dim3(nb), dim3(CS_THREADS), 0, st, h->sc);
    hipLaunchKernelGGL(k_cell_top, dim3(1), dim3(1024), 0, st, h->sc);
    hipLaunchKernelGGL(k_cell_down, dim3(nb), dim3(CS_THREADS), 0, st, h->sc);
    hipLaunchKernelGGL(k_cell_scatter, dim3(SMALL_GRID), dim3(256), 0, st, h->S, h->sc, h->g);
    hipLaunchKernelGGL(k_cell_rank, dim3(SMALL_GRID), dim3(256), 0, st, h->sc);
    hipLaunchKernelGGL(k_cell_order, dim3(SMALL_GRID), dim3(256), 0, st, h->S, h->sc);
    return hipGetLastError();
}

hipError_t launch_runaway_rho(misa_lattice *h) {
    hipStream_t st = h->stream;
    hipLaunchKernelGGL(k_runaway_rho_lone, dim3(SMALL_GRID), dim3(64 * LONE_WAVES), 0, st, h->S, h->sc, h->g,
                       t64_of(h));
    hipLaunchKernelGGL(k_runaway_rho_cells, dim3(cell_grid(h, k_runaway_rho_cells)), dim3(RC_THREADS), 0, st, h->S, h->sc, h->g,
                       t64_of(h));
    hipLaunchKernelGGL(k_mark_count, dim3(h->sc.mark_nblk), dim3(MARK_THREADS), 0, st, h->sc);
    hipLaunchKernelGGL(k_mark_scan, dim3(1), dim3(1024), 0, st, h->sc, h->sc.mark_nblk);
    hipLaunchKernelGGL(k_mark_emit, dim3(h->sc.mark_nblk), dim3(MARK_THREADS), 0, st, h->sc);
    if (h->precision == MISA_FP32)
        hipLaunchKernelGGL(k_affected_rho<float>, dim3(AFF_GRID), dim3(AFF_THREADS), 0, st, h->S, h->sc, h->g, t64_of(h),
                           t32_of(h), h->use_mlp ? h->mlp.net[2] : MlpNet{}, near_fix_of(h));
    else
        hipLaunchKernelGGL(k_affected_rho<double>, dim3(AFF_GRID), dim3(AFF_THREADS), 0, st, h->S, h->sc, h->g,
                           t64_of(h), t64_of(h), MlpNet{}, NearFix32{});
    return hipGetLastError();
}

hipError_t launch_runaway_force(misa_lattice *h, bool energy, bool kick) {
    hipStream_t st = h->stream;
    hipLaunchKernelGGL(k_runaway_force_lone, dim3(SMALL_GRID), dim3(64 * LONE_WAVES), 0, st, h->S, h->sc, h->g,
                       t64_of(h), h->precision == MISA_FP32 ? 1 : 0, energy ? 1 : 0);
    hipLaunchKernelGGL(k_runaway_force_cells, dim3(cell_grid(h, k_runaway_force_cells)), dim3(RC_THREADS), 0, st, h->S, h->sc, h->g,
                       t64_of(h), h->precision == MISA_FP32 ? 1 : 0, energy ? 1 : 0);
    const double kf = ACC_UNIT / h->mass;
    if (h->precision == MISA_FP32)
        hipLaunchKernelGGL(k_affected_force<float>, dim3(AFF_GRID), dim3(AFF_THREADS), 0, st, h->S, h->sc, h->g,
                           t64_of(h), kick ? 1 : 0, kf, near_fix_of(h), energy ? 1 : 0);
    else
        hipLaunchKernelGGL(k_affected_force<double>, dim3(AFF_GRID), dim3(AFF_THREADS), 0, st, h->S, h->sc, h->g,
                           t64_of(h), kick ? 1 : 0, kf, NearFix32{}, energy ? 1 : 0);
    return hipGetLastError();
}

// Batched launches (blockIdx.y = box).  gx_*: blocks per box of the grid-stride kernels.
hipError_t launchb_rehash(hipStream_t st, const BoxRef *boxes, int nbox, int gx_small) {
    hipLaunchKernelGGL(kb_sort, dim3(1, nbox), dim3(SORT_THREADS), 0, st, boxes);
    hipLaunchKernelGGL(kb_claim, dim3(gx_small, nbox), dim3(256), 0, st, boxes);
    hipLaunchKernelGGL(kb_settle, dim3(gx_small, nbox), dim3(256), 0, st, boxes);
    hipLaunchKernelGGL(kb_compact, dim3(1, nbox), dim3(1024), 0, st, boxes);
    return hipGetLastError();
}

// gx_cells: the largest cell-scan block count of the boxes.
hipError_t launchb_runaway_build(hipStream_t st, const BoxRef *boxes, int nbox, int gx_small, int gx_cells) {
    hipLaunchKernelGGL(kb_cell_count, dim3(gx_small, nbox), dim3(256), 0, st, boxes);
    hipLaunchKernelGGL(kb_cell_sum, dim3(gx_cells, nbox), dim3(CS_THREADS), 0, st, boxes);
    hipLaunchKernelGGL(kb_cell_top, dim3(1, nbox), dim3(1024), 0, st, boxes);
    hipLaunchKernelGGL(kb_cell_down, dim3(gx_cells, nbox), dim3(CS_THREADS), 0, st, boxes);
    hipLaunchKernelGGL(kb_cell_scatter, dim3(gx_small, nbox), dim3(256), 0, st, boxes);
    hipLaunchKernelGGL(kb_cell_rank, dim3(gx_small, nbox), dim3(256), 0, st, boxes);
    hipLaunchKernelGGL(kb_cell_order, dim3(gx_small, nbox), dim3(256), 0, st, boxes);
    return hipGetLastError();
}

// Blocks of a grid-stride kernel over the flattened lists that keep every compute unit
// at the kernel's occupancy (its waves are latency-bound chains of scattered loads, so
// the more resident, the better), and at least FLAT_BLOCKS.
template <typename Kernel>
static int fill_grid(const misa_lattice *h0, Kernel k, int threads, size_t lds) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, lds) != hipSuccess) per_cu = 0;
    return std::max(FLAT_BLOCKS, per_cu * h0->n_cu);
}

// off: 3 (nbox + 1) ints for the offsets of the crowded-cell, affected-atom and lone
// run-away lists.  The force half reuses the offsets the density half computed (no count
// changes in between).
hipError_t launchb_runaway_rho(misa_lattice *h0, const BoxRef *boxes, int nbox, int mark_blocks, int32_t *off) {
    hipStream_t st = h0->stream;
    const size_t lds = sizeof(int32_t) * (nbox + 1);
    hipLaunchKernelGGL(kb_flat_offsets, dim3(1), dim3(1024), 0, st, boxes, nbox, 0, off);
    hipLaunchKernelGGL(kb_flat_offsets, dim3(1), dim3(1024), 0, st, boxes, nbox, 2, off + 2 * (nbox + 1));
    hipLaunchKernelGGL(kf_runaway_rho_lone, dim3(fill_grid(h0, kf_runaway_rho_lone, 64 * LONE_WAVES, lds)),
                       dim3(64 * LONE_WAVES), lds, st, boxes, nbox, off + 2 * (nbox + 1), t64_of(h0));
    hipLaunchKernelGGL(kf_runaway_rho, dim3(fill_grid(h0, kf_runaway_rho, RC_THREADS, lds)), dim3(RC_THREADS), lds,
                       st, boxes, nbox, off, t64_of(h0));
    hipLaunchKernelGGL(kb_mark_count, dim3(mark_blocks, nbox), dim3(MARK_THREADS), 0, st, boxes);
    hipLaunchKernelGGL(kb_mark_scan, dim3(1, nbox), dim3(1024), 0, st, boxes);
    hipLaunchKernelGGL(kb_mark_emit, dim3(mark_blocks, nbox), dim3(MARK_THREADS), 0, st, boxes);
    hipLaunchKernelGGL(kb_flat_offsets, dim3(1), dim3(1024), 0, st, boxes, nbox, 1, off + nbox + 1);
    hipLaunchKernelGGL(kf_affected_rho, dim3(fill_grid(h0, kf_affected_rho, AFF_THREADS, lds)), dim3(AFF_THREADS),
                       lds, st, boxes, nbox, off + nbox + 1, t64_of(h0), t32_of(h0), near_fix_of(h0));
    return hipGetLastError();
}

hipError_t launchb_runaway_force(misa_lattice *h0, const BoxRef *boxes, int nbox, bool energy, const int32_t *off) {
    hipStream_t st = h0->stream;
    const size_t lds = sizeof(int32_t) * (nbox + 1);
    hipLaunchKernelGGL(kf_runaway_force_lone, dim3(fill_grid(h0, kf_runaway_force_lone, 64 * LONE_WAVES, lds)),
                       dim3(64 * LONE_WAVES), lds, st, boxes, nbox, off + 2 * (nbox + 1), t64_of(h0),
                       energy ? 1 : 0);
    hipLaunchKernelGGL(kf_runaway_force, dim3(fill_grid(h0, kf_runaway_force, RC_THREADS, lds)), dim3(RC_THREADS),
                       lds, st, boxes, nbox, off, t64_of(h0), energy ? 1 : 0);
    hipLaunchKernelGGL(kf_affected_force, dim3(fill_grid(h0, kf_affected_force, AFF_THREADS, lds)),
                       dim3(AFF_THREADS), lds, st, boxes, nbox, off + nbox + 1, t64_of(h0), ACC_UNIT / h0->mass,
                       near_fix_of(h0), energy ? 1 : 0);
    return hipGetLastError();
}

hipError_t launchb_runaway_clear(hipStream_t st, const BoxRef *boxes, int nbox) {
    hipLaunchKernelGGL(kb_runaway_clear, dim3(1, nbox), dim3(64), 0, st, boxes);
    return hipGetLastError();
}

hipError_t launch_runaway_clear(misa_lattice *h) {
    hipLaunchKernelGGL(k_runaway_clear, dim3(1), dim3(64), 0, h->stream, h->sc);
    return hipGetLastError();
}

}  // namespace misa

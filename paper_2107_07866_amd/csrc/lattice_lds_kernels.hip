// Persistent float32 lattice kernels (rho pass and force pass).
//
// Same gather as the generic tile kernels, reorganised for the table look-ups
// that dominate the pair loop (the same pressure the paper meets on the 64 KiB
// local store, Sec. 4.1): each work-group copies, once, the window of f / phi
// records that pairs of slotted atoms can reach (r >= nearest-site distance -
// 2 delta) into LDS, then loops over 8 x 8 x 8-cell
// tiles, each staged with its periodic halo.  Work-groups are sized to one per
// compute unit; tiles are dealt out so every XCD sweeps one contiguous block of
// tiles (halo re-reads stay in that XCD's L2).  The next tile's displacements are
// fetched into registers while the current tile computes (the GPU counterpart of
// the paper's double-buffered DMA, Sec. 4.3).
//
// The window is re-tabulated from the spline on an equidistant grid in q = r^2,
// with the force records holding f'(r)/r and phi'(r)/r, so a pair costs no square
// root and no reciprocal (each a quarter-rate transcendental).  The records are
// linear in t between the spline's values at the grid nodes, on a grid fine enough
// (6143 segments) that the interpolation error stays near float32 rounding: a pair
// then costs one LDS read of 8 bytes (density) or 16 bytes (force) and one or two
// multiply-adds for the table.
//
// The pair loop is branch-free and unrolled: every stencil candidate runs the
// full arithmetic and out-of-range pairs are dropped by a select (or read a zero
// record), so the LDS reads of several offsets are in flight together instead
// of one dependent chain per offset.  Table indices are clamped into the window:
// a slotted atom is within delta of its site, so an in-range pair can only fall
// below the window after a run-away capacity overflow (reported on its own).
#include "misa_internal.h"

#include <type_traits>

// Multiply-adds fuse only within one expression: every copy of a pair loop (the
// unrolled bodies, the loops with and without the band test of the cut-off) then
// rounds a pair's terms alike, so results do not depend on which copy a stencil
// entry falls into (the tile shapes and the per-tile band test move that boundary).
#pragma clang fp contract(on)

namespace misa {

__device__ __forceinline__ int wrap2(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// Next real item of work-group b at or after iteration it (advances it), or -1.
// Items are dealt so that every XCD sweeps one contiguous block of them.
__device__ __forceinline__ int next_item(int b, int &it, int grid, int n, int n_pad) {
    const int per = n_pad >> 3;  // items per XCD
    for (;; ++it) {
        const int j = (b >> 3) + it * (grid >> 3);  // position inside this XCD's block of items
        if (j >= per) return -1;
        const int id = (b & 7) * per + j;
        if (id < n) return id;
    }
}

// What one tile of a lattice pass needs to know about its box: the box, its tiling
// (tx x ty x tz interior cells, tx ty tz = 512, so 1024 lanes serve both
// sublattices) and the stencil with the LDS offsets of that tile shape.
struct TileGeo {
    int32_t nx, ny, nz, nt0, nt1;
    int32_t tx, ty, tz;             // powers of two
    uint32_t dx, dy, dz;            // ceil(2^32 / (t + 4)) for the staged block's index arithmetic
    int32_t shape;                  // index of the tiling: its stencil is st + shape 2 KMAX
    int64_t ncell;
};

// Tiles of one box: item = tile id; 8 x 8 x 8 tiles, known at compile time (the
// shape fields of TileGeo stay unused).
struct OneBox {
    static constexpr bool kFixed = true;
    static constexpr int kMaxSites = TILE2_SITES;
    int32_t nx, ny, nz, nt0, nt1;
    int64_t ncell;
    PassPtrs P;
    int ntiles, ntiles_pad;
    __device__ __forceinline__ int next(int b, int &it, int grid) const {
        return next_item(b, it, grid, ntiles, ntiles_pad);
    }
    __device__ __forceinline__ int get(int item, TileGeo &G, PassPtrs &Q) const {
        G.nx = nx;
        G.ny = ny;
        G.nz = nz;
        G.nt0 = nt0;
        G.nt1 = nt1;
        G.ncell = ncell;
        Q = P;
        return item;
    }
};

// Tiles of many boxes: item -> (box, tile) from a list built on the host.  With
// kAnyShape every box has its own tile shape (one of the 1024-lane shapes whose
// staged block fits in LDS) and the kernel's stencil argument holds the stencils of
// all shapes; without it every box uses the compile-time 8 x 8 x 8 tiles.
template <bool kAnyShape>
struct ManyBoxesT {
    static constexpr bool kFixed = !kAnyShape;
    static constexpr int kMaxSites = kAnyShape ? TILE2_SITES_MAX : TILE2_SITES;
    const BoxPass *boxes;
    const int2 *items;
    int nitems, nitems_pad;
    __device__ __forceinline__ int next(int b, int &it, int grid) const {
        return next_item(b, it, grid, nitems, nitems_pad);
    }
    __device__ __forceinline__ int get(int item, TileGeo &G, PassPtrs &Q) const {
        const int2 bt = items[item];
        const BoxPass &B = boxes[bt.x];
        G.nx = B.g.nx;
        G.ny = B.g.ny;
        G.nz = B.g.nz;
        G.nt0 = B.g.nt2[0];
        G.nt1 = B.g.nt2[1];
        if (kAnyShape) {
            G.tx = B.g.tshape[0];
            G.ty = B.g.tshape[1];
            G.tz = B.g.tshape[2];
            G.dx = B.g.tdiv[0];
            G.dy = B.g.tdiv[1];
            G.dz = B.g.tdiv[2];
            G.shape = B.shape;
        }
        G.ncell = B.g.ncell;
        Q = B.P;
        return bt.y;
    }
};

// Tile shape of a source: compile-time 8 x 8 x 8 for one box, the box's own otherwise.
// Runtime shapes avoid integer division (tens of instructions on the GPU): the
// interior sides are powers of two (shifts), and an index e < 2^12 of the staged
// block divides by a side p + 4 <= 20 exactly as mulhi(e, ceil(2^32 / p)).
struct Dims {
    int tx, ty, tz, px, py, pz, sites;
    int sx, sy;               // log2 tx, log2 ty
    uint32_t mx, my, mz;      // multiply-high reciprocals of px, py, pz
};
template <class Src>
__device__ __forceinline__ Dims dims_of(const TileGeo &G) {
    Dims d;
    d.tx = Src::kFixed ? T2X : G.tx;
    d.ty = Src::kFixed ? T2Y : G.ty;
    d.tz = Src::kFixed ? T2Z : G.tz;
    d.px = d.tx + 2 * HALO;
    d.py = d.ty + 2 * HALO;
    d.pz = d.tz + 2 * HALO;
    d.sites = 2 * d.px * d.py * d.pz;
    d.sx = __builtin_ctz((unsigned)d.tx);
    d.sy = __builtin_ctz((unsigned)d.ty);
    d.mx = Src::kFixed ? 0u : G.dx;
    d.my = Src::kFixed ? 0u : G.dy;
    d.mz = Src::kFixed ? 0u : G.dz;
    return d;
}

// e / c for a staged-block index e < 2^12 (c one of the block's sides)
template <class Src>
__device__ __forceinline__ int div_side(int e, int c, uint32_t m) {
    return Src::kFixed ? e / c : (int)__umulhi((uint32_t)e, m);
}

// This lane's site in a tile: wave w serves parity w / 8 and the 64 interior sites
// (w % 8) 64 .. + 63 of that parity's tx x ty x tz block (x fastest).  For
// 8 x 8 x 8 tiles that is one z plane per wave.
struct LaneSite {
    int lx, ly, lz, me;
};
__device__ __forceinline__ LaneSite lane_site(const Dims &d, int p, int w, int lane) {
    LaneSite L;
    const int l = (w & 7) * 64 + lane;
    L.lx = l & (d.tx - 1);
    L.ly = (l >> d.sx) & (d.ty - 1);
    L.lz = l >> (d.sx + d.sy);
    L.me = ((p * d.pz + L.lz + HALO) * d.py + L.ly + HALO) * d.px + L.lx + HALO;
    return L;
}

constexpr int TILE2_PER_LANE = (TILE2_SITES_MAX + TILE2_THREADS - 1) / TILE2_THREADS;
static_assert((TILE2_SITES + TILE2_THREADS - 1) / TILE2_THREADS == TILE2_PER_LANE,
              "8 x 8 x 8 tiles and the largest shape take the same registers per lane");

// One lane's share of a tile (interior + halo), held in registers between the
// global fetch and the LDS store.
struct TileRegs {
    double x[TILE2_PER_LANE], y[TILE2_PER_LANE], z[TILE2_PER_LANE];
    float w[TILE2_PER_LANE];
};

template <class Src>
__device__ __forceinline__ void fetch_tile2(TileRegs &R, const double *__restrict__ ux,
                                            const double *__restrict__ uy, const double *__restrict__ uz,
                                            const float *__restrict__ w_src, const TileGeo &g, const Dims &d,
                                            int tid) {
    const int tx = tid % g.nt0;
    const int tyz = tid / g.nt0;
    const int ty = tyz % g.nt1;
    const int tz = tyz / g.nt1;
    const int bx = tx * d.tx - HALO, by = ty * d.ty - HALO, bz = tz * d.tz - HALO;
#pragma unroll
    for (int j = 0; j < TILE2_PER_LANE; ++j) {
        const int e = threadIdx.x + j * TILE2_THREADS;
        if (e < d.sites) {
            int r = div_side<Src>(e, d.px, d.mx);
            const int lx = e - r * d.px;
            const int r2 = div_side<Src>(r, d.py, d.my);
            const int ly = r - r2 * d.py;
            const int p = div_side<Src>(r2, d.pz, d.mz);
            const int lz = r2 - p * d.pz;
            const int gx = wrap2(bx + lx, g.nx), gy = wrap2(by + ly, g.ny), gz = wrap2(bz + lz, g.nz);
            const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
            R.x[j] = ux[idx];
            R.y[j] = uy[idx];
            R.z[j] = uz[idx];
            R.w[j] = w_src ? w_src[idx] : 0.0f;
        }
    }
}

// Stores this lane's share of the tile; returns the largest |u|^2 among the
// occupied sites it stored.
__device__ __forceinline__ float store_tile2(Q4<float> *__restrict__ tile, const TileRegs &R, int sites) {
    float m = 0.0f;
#pragma unroll
    for (int j = 0; j < TILE2_PER_LANE; ++j) {
        const int e = threadIdx.x + j * TILE2_THREADS;
        if (e < sites) {
            Q4<float> q;
            q.x = (float)R.x[j];
            q.y = (float)R.y[j];
            q.z = (float)R.z[j];
            q.w = R.w[j];
            tile[e] = q;
            if (q.x < (float)VACANT_TEST) m = fmaxf(m, q.x * q.x + q.y * q.y + q.z * q.z);
        }
    }
    return m;
}

// Stencil length for this tile.  The stencil is sorted by |offset|; its first kin
// entries lie inside rc, the next one at d_next.  A pair (i, i + o) is closer than
// rc only if |o| < rc + |u_i| + |u_j|, so when every occupied site of the tile and
// its halo has |u| < u_cut = (d_next - rc) / 2 - margin, entries kin .. K - 1 can
// hold no pair within rc and are skipped (u_cut < 0 when no entry lies beyond rc).
// slot: the LDS word of this tile (two words alternate between consecutive tiles).
// klo: entries 0 .. klo - 1 hold no pair within NEAR_MARGIN of rc in this tile
// (thr: this lane's entry of NearTab::thr2), so only entries klo .. need the
// band test of the float32 cut-off decision.
__device__ __forceinline__ int tile_stencil_length(float m, unsigned *slot, unsigned *other, int K, int kin,
                                                   float u_cut2, float thr, int &klo) {
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(slot, __float_as_uint(m));  // |u|^2 >= 0: integer order = float order
    __syncthreads();
    const float umax2 = __uint_as_float(*slot);
    if (threadIdx.x == 0) *other = 0u;  // cleared for the next tile (read after the next barrier pair)
    klo = __builtin_amdgcn_readfirstlane(__popcll(__ballot(umax2 < thr)));
    return __builtin_amdgcn_readfirstlane(umax2 < u_cut2 ? kin : K);
}
__device__ __forceinline__ int tile_stencil_length(float m, unsigned *slot, unsigned *other, int K, int kin,
                                                   float u_cut2) {
    int klo;
    return tile_stencil_length(m, slot, other, K, kin, u_cut2, -1.0f, klo);
}

template <class Src, bool kNodeCut>
__global__ __launch_bounds__(TILE2_THREADS) void k_rho_lds(Src src, const StencilEntry<float> *__restrict__ st,
                                                          int K, int kin, float u_cut2,
                                                          const float2 *__restrict__ fwin, float inv_hq,
                                                          float pcq, int nwin, const Q4<float> *__restrict__ etab,
                                                          TabMeta<float> em, float rc2, const NearTab *__restrict__ nt) {
    __shared__ Q4<float> tile[Src::kMaxSites];
    __shared__ float2 ftab[LDS_TAB_SEGS];  // {f_0, f_1 - f_0} per segment
    __shared__ unsigned umax_slot[2];
    if (threadIdx.x < 2) umax_slot[threadIdx.x] = 0u;
    for (int e = threadIdx.x; e < nwin; e += TILE2_THREADS) ftab[e] = fwin[e];
    if (kNodeCut && threadIdx.x == 0) ftab[nwin] = make_float2(0.0f, 0.0f);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // pcq kept in a vector register for the pair loop: the table position's multiply-add
    // takes one scalar operand (inv_hq), and re-copying pcq would cost an instruction per
    // unrolled iteration
    float pcq_v = pcq;
    asm volatile("" : "+v"(pcq_v));
    // wave-uniform parity: the stencil entries below become scalar loads
    const int p = __builtin_amdgcn_readfirstlane(w >> 3);
    const float thr = nt->thr2[p][lane];
    TileGeo Gf{};  // the fixed shape's lane site and stencil, computed once
    const LaneSite Lf = lane_site(dims_of<Src>(Gf), p, w, lane);
    int it = 0;
    int item = src.next(blockIdx.x, it, gridDim.x);
    TileRegs R;
    if (item >= 0) {
        TileGeo G0;
        PassPtrs P0;
        const int t0 = src.get(item, G0, P0);
        fetch_tile2<Src>(R, P0.ux, P0.uy, P0.uz, nullptr, G0, dims_of<Src>(G0), t0);
    }
    while (item >= 0) {
        TileGeo G;
        PassPtrs P;
        const int tid = src.get(item, G, P);
        const Dims d = dims_of<Src>(G);
        const LaneSite L = Src::kFixed ? Lf : lane_site(d, p, w, lane);
        // wave-uniform shape and parity: the stencil entries are scalar loads from st
        const int shp = Src::kFixed ? 0 : __builtin_amdgcn_readfirstlane(G.shape);
        const StencilEntry<float> *sp = st + (shp * 2 + p) * KMAX;
        __syncthreads();  // previous tile fully consumed (and the table copied)
        const float m = store_tile2(tile, R, d.sites);
        int klo;
        const int Kt =
            tile_stencil_length(m, &umax_slot[it & 1], &umax_slot[(it + 1) & 1], K, kin, u_cut2, thr, klo);
        ++it;
        const int nxt = src.next(blockIdx.x, it, gridDim.x);
        if (nxt >= 0) {
            TileGeo Gn;
            PassPtrs Pn;
            const int ntid = src.get(nxt, Gn, Pn);
            fetch_tile2<Src>(R, Pn.ux, Pn.uy, Pn.uz, nullptr, Gn, dims_of<Src>(Gn), ntid);  // in flight during this tile
        }
        const int tx = tid % G.nt0;
        const int tyz = tid / G.nt0;
        const int gx = tx * d.tx + L.lx, gy = (tyz % G.nt1) * d.ty + L.ly, gz = (tyz / G.nt1) * d.tz + L.lz;
        if (gx < G.nx && gy < G.ny && gz < G.nz) {
            const int me = L.me;
            const Q4<float> ui = tile[me];
            float acc = 0.0f;
            // f(r_ij) of entry k added to acc; returns r^2 - rc^2
            auto term = [&](int k) -> float {
                const StencilEntry<float> e = sp[k];
                const Q4<float> uj = tile[me + e.lds];
                const float dx = (uj.x - ui.x) + e.ox;
                const float dy = (uj.y - ui.y) + e.oy;
                const float dz = (uj.z - ui.z) + e.oz;
                const float r2 = pair_r2_f32(dx, dy, dz);
                float t;
                const int s = win_seg<kNodeCut>(win_pos(r2, inv_hq, pcq_v), nwin, t);  // q = r^2 grid
                const float2 c = ftab[s];
                const float vr = c.y * t + c.x;
                acc += (kNodeCut || r2 < rc2) ? vr : 0.0f;
                return r2 - rc2;
            };
            // Entries klo .. also track the pair closest to rc^2.  A pair whose float32
            // r^2 lies within RC_BAND_Q of rc^2 may fall on the other side of rc than in
            // float64: such an atom joins the list of atoms that run-aways touch, whose
            // fix-ups correct its density and force.  (Two loop variables, and the band
            // test as a running minimum in a vector register: with a shared variable or
            // a lane-mask flag the unrolled loops lost the overlap of their LDS reads.)
            float dmin = 1.0f;
#pragma unroll 4
            for (int k = 0; k < klo; ++k) (void)term(k);
#pragma unroll 4
            for (int k2 = klo; k2 < Kt; ++k2) dmin = fminf(dmin, fabsf(term(k2)));
            const int64_t idx = (int64_t)p * G.ncell + ((int64_t)gz * G.ny + gy) * G.nx + gx;
            if (dmin < RC_BAND_Q) atomicOr(&P.mark[idx >> 5], 1u << (idx & 31));
            float fpv = 0.0f;
            bool beyond = false;
            if (ui.x > (float)VACANT_TEST) {
                acc = 0.0f;
            } else if (acc > em.x_last) {
                beyond = true;
                fpv = em.d_last;
            } else {
                const float q = (acc - em.x0) * em.inv_h;
                int kk = (int)q;
                kk = kk < em.nseg - 1 ? kk : em.nseg - 1;
                kk = kk > 0 ? kk : 0;
                const float t = q - (float)kk;
                const Q4<float> d = etab[2 * kk + 1];
                fpv = (d.z * t + d.y) * t + d.x;
            }
            P.rho[idx] = acc;
            P.fp[idx] = fpv;
            if (beyond) atomicAdd(P.range_viol, 1u);
        }
        item = nxt;
    }
}

__device__ __forceinline__ double wave_sum_l(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max_l(double v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Fused second half-kick of velocity Verlet: v += (dt/2) C F / m right after F is
// known, plus per-tile {max |v|^2, sum |v|^2} over atoms that no run-away atom
// touches (those get their run-away terms, kick and statistics in the fixup pass).
template <class Src, bool kEnergy, bool kNodeCut, bool kKick>
__global__ __launch_bounds__(TILE2_THREADS) void k_force_lds(Src src, const StencilEntry<float> *__restrict__ st,
                                                            int K, int kin, float u_cut2,
                                                            const float4 *__restrict__ fwin, float inv_hq,
                                                            float pcq, int nwin, Tables<float> T, float rc2,
                                                            double kf) {
    __shared__ Q4<float> tile[Src::kMaxSites];
    __shared__ unsigned umax_slot[2];
    if (threadIdx.x < 2) umax_slot[threadIdx.x] = 0u;
    __shared__ float4 fab[LDS_TAB_SEGS];  // {gf_0, gf_1 - gf_0, gp_0, gp_1 - gp_0} per segment
    __shared__ double red[4][TILE2_THREADS / 64];
    for (int e = threadIdx.x; e < nwin; e += TILE2_THREADS) fab[e] = fwin[e];
    if (kNodeCut && threadIdx.x == 0) fab[nwin] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // pcq kept in a vector register for the pair loop: the table position's multiply-add
    // takes one scalar operand (inv_hq), and re-copying pcq would cost an instruction per
    // unrolled iteration
    float pcq_v = pcq;
    asm volatile("" : "+v"(pcq_v));
    const int p = __builtin_amdgcn_readfirstlane(w >> 3);
    TileGeo Gf{};  // the fixed shape's lane site and stencil, computed once
    const LaneSite Lf = lane_site(dims_of<Src>(Gf), p, w, lane);
    const int nlast = T.fm.nseg - 1;
    int it = 0;
    int item = src.next(blockIdx.x, it, gridDim.x);
    TileRegs R;
    if (item >= 0) {
        TileGeo G0;
        PassPtrs P0;
        const int t0 = src.get(item, G0, P0);
        fetch_tile2<Src>(R, P0.ux, P0.uy, P0.uz, P0.fp, G0, dims_of<Src>(G0), t0);
    }
    while (item >= 0) {
        TileGeo G;
        PassPtrs P;
        const int tid = src.get(item, G, P);
        const Dims d = dims_of<Src>(G);
        const LaneSite L = Src::kFixed ? Lf : lane_site(d, p, w, lane);
        // wave-uniform shape and parity: the stencil entries are scalar loads from st
        const int shp = Src::kFixed ? 0 : __builtin_amdgcn_readfirstlane(G.shape);
        const StencilEntry<float> *sp = st + (shp * 2 + p) * KMAX;
        __syncthreads();
        const float m = store_tile2(tile, R, d.sites);
        const int Kt = tile_stencil_length(m, &umax_slot[it & 1], &umax_slot[(it + 1) & 1], K, kin, u_cut2);
        ++it;
        const int nxt = src.next(blockIdx.x, it, gridDim.x);
        if (nxt >= 0) {
            TileGeo Gn;
            PassPtrs Pn;
            const int ntid = src.get(nxt, Gn, Pn);
            fetch_tile2<Src>(R, Pn.ux, Pn.uy, Pn.uz, Pn.fp, Gn, dims_of<Src>(Gn), ntid);  // in flight during this tile
        }
        const double hk = kKick ? 0.5 * P.scal[0] * kf : 0.0;
        const int tx = tid % G.nt0;
        const int tyz = tid / G.nt0;
        const int gx = tx * d.tx + L.lx, gy = (tyz % G.nt1) * d.ty + L.ly, gz = (tyz / G.nt1) * d.tz + L.lz;
        const bool active = gx < G.nx && gy < G.ny && gz < G.nz;
        const int64_t idx = (int64_t)p * G.ncell + ((int64_t)gz * G.ny + gy) * G.nx + gx;
        double e_emb = 0.0, e_pair = 0.0, kvm = 0.0, kvs = 0.0;
        double v0x = 0.0, v0y = 0.0, v0z = 0.0;
        uint32_t mw = 0u;
        if (kKick && active) {  // issued now, consumed after the pair loop
            v0x = P.vx[idx];
            v0y = P.vy[idx];
            v0z = P.vz[idx];
            mw = P.mark[idx >> 5];
        }
        if (active) {
            const int me = L.me;
            const Q4<float> ui = tile[me];
            float ax = 0.0f, ay = 0.0f, az = 0.0f, ep = 0.0f;
            // A pair whose float32 r^2 lies within RC_BAND_Q of rc^2 may fall on the other
            // side of rc than in float64: the density pass lists such atoms with the atoms
            // run-aways touch, and the fix-up of that list corrects their forces.
#pragma unroll 2
            for (int k = 0; k < Kt; ++k) {
                const StencilEntry<float> e = sp[k];
                const Q4<float> uj = tile[me + e.lds];
                const float dx = (uj.x - ui.x) + e.ox;
                const float dy = (uj.y - ui.y) + e.oy;
                const float dz = (uj.z - ui.z) + e.oz;
                const float r2 = pair_r2_f32(dx, dy, dz);
                float t;
                const int s = win_seg<kNodeCut>(win_pos(r2, inv_hq, pcq_v), nwin, t);  // q = r^2 grid
                const float4 a = fab[s];
                const float gf = a.y * t + a.x;  // f'(r) / r
                const float gp = a.w * t + a.z;  // phi'(r) / r
                float sc = (ui.w + uj.w) * gf + gp;
                if (!kNodeCut) sc = r2 < rc2 ? sc : 0.0f;
                ax += sc * dx;
                ay += sc * dy;
                az += sc * dz;
                if (kEnergy) {  // last step only: phi(r) from the r-grid records
                    const float pr = (__builtin_amdgcn_sqrtf(r2) - T.fm.x0) * T.fm.inv_h;
                    const int sg = max(0, min((int)pr, nlast));
                    const float tr = pr - (float)sg;
                    const Q4<float> cp = T.phi[sg];
                    const float v = ((cp.w * tr + cp.z) * tr + cp.y) * tr + cp.x;
                    ep += (kNodeCut ? s < nwin : r2 < rc2) ? v : 0.0f;  // same pair set as the force
                }
            }
            const bool vac = ui.x > (float)VACANT_TEST;
            if (vac) ax = ay = az = 0.0f;
            P.fx[idx] = ax;
            P.fy[idx] = ay;
            P.fz[idx] = az;
            if (kKick && !vac) {
                const double vx = v0x + hk * (double)ax;
                const double vy = v0y + hk * (double)ay;
                const double vz = v0z + hk * (double)az;
                P.vx[idx] = vx;
                P.vy[idx] = vy;
                P.vz[idx] = vz;
                if (!((mw >> (idx & 31)) & 1u)) {
                    kvm = vx * vx + vy * vy + vz * vz;
                    kvs = kvm;
                }
            }
            if (kEnergy && !vac) {
                const float rr = P.rho[idx];
                float Fv;
                if (rr > T.em.x_last) {
                    Fv = T.em.y_last + T.em.d_last * (rr - T.em.x_last);
                } else {
                    const float q = (rr - T.em.x0) * T.em.inv_h;
                    int kk = (int)q;
                    kk = kk < T.em.nseg - 1 ? kk : T.em.nseg - 1;
                    kk = kk > 0 ? kk : 0;
                    const float t = q - (float)kk;
                    const Q4<float> c = T.emb[2 * kk];
                    Fv = ((c.w * t + c.z) * t + c.y) * t + c.x;
                }
                e_emb = (double)Fv;
                e_pair = 0.5 * (double)ep;
            }
        }
        if (kEnergy || kKick) {
            if (kEnergy) {
                e_emb = wave_sum_l(e_emb);
                e_pair = wave_sum_l(e_pair);
            }
            if (kKick) {
                kvm = wave_max_l(kvm);
                kvs = wave_sum_l(kvs);
            }
            if (lane == 0) {
                red[0][w] = e_emb;
                red[1][w] = e_pair;
                red[2][w] = kvm;
                red[3][w] = kvs;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double s0 = 0.0, s1 = 0.0, m2 = 0.0, s3 = 0.0;
                for (int q = 0; q < TILE2_THREADS / 64; ++q) {
                    s0 += red[0][q];
                    s1 += red[1][q];
                    m2 = fmax(m2, red[2][q]);
                    s3 += red[3][q];
                }
                if (kEnergy) {
                    P.part[2 * tid] = s0;
                    P.part[2 * tid + 1] = s1;
                }
                if (kKick) {
                    P.part_kick[2 * tid] = m2;
                    P.part_kick[2 * tid + 1] = s3;
                }
            }
        }
        item = nxt;
    }
}

bool lds_path(const misa_lattice *h) {
    return h->precision == MISA_FP32 && !h->use_mlp && h->lds32.usable && h->persistent_grid > 0;
}

NearFix32 near_fix_of(const misa_lattice *h) {
    NearFix32 nf;
    if (!lds_path(h) || half_path(h)) return nf;  // the half-stencil passes decide in float64 themselves
    nf.frec = h->lds32.lf;
    nf.rec = h->lds32.lg;
    nf.nt = h->near_g;
    nf.phi = h->t32.phi;
    nf.fm = h->t32.fm;
    nf.inv_hq = h->lds32.inv_hq;
    nf.pcq = h->lds32.pcq;
    nf.rc2 = (float)h->g.rc2;
    nf.nwin = h->lds32.nwin;
    nf.node_cut = h->lds32.node_cut ? 1 : 0;
    nf.K = h->K;
    return nf;
}

PassPtrs pass_ptrs(misa_lattice *h) {
    PassPtrs P;
    P.ux = h->S.ux;
    P.uy = h->S.uy;
    P.uz = h->S.uz;
    P.rho = (float *)h->S.rho;
    P.fp = (float *)h->S.fp;
    P.fx = (float *)h->S.fx;
    P.fy = (float *)h->S.fy;
    P.fz = (float *)h->S.fz;
    P.vx = h->S.vx;
    P.vy = h->S.vy;
    P.vz = h->S.vz;
    P.mark = h->sc.mark;
    P.scal = h->sc.scal;
    P.part = h->sc.part;
    P.part_kick = h->sc.part_kick;
    P.range_viol = &h->sc.cnt->range_viol;
    return P;
}

static OneBox one_box(misa_lattice *h) {
    OneBox o;
    const Geom &g = h->g;
    o.nx = g.nx;
    o.ny = g.ny;
    o.nz = g.nz;
    o.nt0 = g.nt2[0];
    o.nt1 = g.nt2[1];
    o.ncell = g.ncell;
    o.P = pass_ptrs(h);
    o.ntiles = g.ntiles2;
    o.ntiles_pad = g.ntiles2_pad;
    return o;
}

// ---------------------------------------------------------------------------
// Float64 density pass on the same persistent scheme.  Beside an 8 x 8 x 8 tile of
// float64 displacements (x and y as one 16-byte word, z apart: 81 KiB) sit RWIN64_MAX
// float64 spline records of f (32 bytes: the segment's cubic in t) as bands around the
// stencil's shell distances, with a zero record for pairs at or past the cut-off
// (BandWin64); a pair outside its entry's band reads the table record from global memory.

// Stores this lane's share of the tile; returns the largest |u|^2 among the occupied
// sites it stored (in float32, as the stencil-length test takes it).
__device__ __forceinline__ float store_tile64(double2 *__restrict__ txy, double *__restrict__ tz,
                                              const TileRegs &R, int sites) {
    float m = 0.0f;
#pragma unroll
    for (int j = 0; j < TILE2_PER_LANE; ++j) {
        const int e = threadIdx.x + j * TILE2_THREADS;
        if (e < sites) {
            txy[e] = make_double2(R.x[j], R.y[j]);
            tz[e] = R.z[j];
            if (R.x[j] < VACANT_TEST) m = fmaxf(m, (float)(R.x[j] * R.x[j] + R.y[j] * R.y[j] + R.z[j] * R.z[j]));
        }
    }
    return m;
}

// rho_i = sum_j f(r_ij) over the stencil, then F'(rho_i) (Sec. 2.2 steps 1-2), float64.
// nodes: nn nodes of f from source node k0 on; fm: the source table's grid.
// recs, nrec: the LDS records ({c0, c1}, {c2, c3} each) in LDS order; band: per parity
// and stencil entry, the segments held and where; ftab: the table's records.
template <bool kNodeCut>
__global__ __launch_bounds__(TILE2_THREADS) void k_rho_lds64(OneBox src, const StencilEntry<double> *__restrict__ st,
                                                            int K, int kin, float u_cut2,
                                                            const double2 *__restrict__ recs, int nrec,
                                                            const int4 *__restrict__ band,
                                                            const Q4<double> *__restrict__ ftab, TabMeta<double> fm,
                                                            const Q4<double> *__restrict__ etab, TabMeta<double> em,
                                                            double rc2) {
    __shared__ double2 txy[TILE2_SITES];
    __shared__ double tz[TILE2_SITES];
    __shared__ double2 rw[2 * RWIN64_MAX];
    __shared__ unsigned umax_slot[2];
    if (threadIdx.x < 2) umax_slot[threadIdx.x] = 0u;
    for (int e = threadIdx.x; e < 2 * nrec; e += TILE2_THREADS) rw[e] = recs[e];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p = __builtin_amdgcn_readfirstlane(w >> 3);  // wave-uniform parity: scalar stencil loads
    TileGeo Gf{};
    const Dims d = dims_of<OneBox>(Gf);
    const LaneSite L = lane_site(d, p, w, lane);
    const StencilEntry<double> *sp = st + p * KMAX;
    const int4 *bp = band + p * KMAX;
    const int nlast = fm.nseg - 1;
    // pp = (r - x0) / h, capped at nseg (kNodeCut: the zero record) or at the last node
    const double pc0 = -fm.x0 * fm.inv_h;
    const double dtop = (double)fm.nseg;
    int it = 0;
    int item = src.next(blockIdx.x, it, gridDim.x);
    TileRegs R;
    if (item >= 0) {
        TileGeo G0;
        PassPtrs P0;
        const int t0 = src.get(item, G0, P0);
        fetch_tile2<OneBox>(R, P0.ux, P0.uy, P0.uz, nullptr, G0, d, t0);
    }
    while (item >= 0) {
        TileGeo G;
        PassPtrs P;
        const int tid = src.get(item, G, P);
        __syncthreads();  // previous tile fully consumed (and the window copied)
        const float m = store_tile64(txy, tz, R, d.sites);
        const int Kt = tile_stencil_length(m, &umax_slot[it & 1], &umax_slot[(it + 1) & 1], K, kin, u_cut2);
        ++it;
        const int nxt = src.next(blockIdx.x, it, gridDim.x);
        if (nxt >= 0) {
            TileGeo Gn;
            PassPtrs Pn;
            const int ntid = src.get(nxt, Gn, Pn);
            fetch_tile2<OneBox>(R, Pn.ux, Pn.uy, Pn.uz, nullptr, Gn, d, ntid);  // in flight during this tile
        }
        const int tx = tid % G.nt0;
        const int tyz = tid / G.nt0;
        const int gx = tx * d.tx + L.lx, gy = (tyz % G.nt1) * d.ty + L.ly, gz = (tyz / G.nt1) * d.tz + L.lz;
        if (gx < G.nx && gy < G.ny && gz < G.nz) {
            const int me = L.me;
            const double2 pi = txy[me];
            const double zi = tz[me];
            double acc = 0.0;
#pragma unroll 2
            for (int k = 0; k < Kt; ++k) {
                const StencilEntry<double> e = sp[k];
                const double2 pj = txy[me + e.lds];
                const double dx = (pj.x - pi.x) + e.ox;
                const double dy = (pj.y - pi.y) + e.oy;
                const double dz = (tz[me + e.lds] - zi) + e.oz;
                const double r2 = dx * dx + dy * dy + dz * dz;
                // table segment s and offset t; with kNodeCut pairs at or past the cut-off
                // (the last node) take s = nseg, whose record is zero
                const double pp = fmin(fma(sqrt_nr1(r2), fm.inv_h, pc0), dtop);
                const int s = max((int)pp, 0);
                const double t = pp - (double)s;
                // this entry's band of LDS records (read unconditionally, see k_force_lds64),
                // else the table's record in global memory (zeros past the last segment)
                const int4 bw = bp[k];
                const int l = s - bw.x;
                const bool inw = (unsigned)l < (unsigned)bw.y;
                const int lw = bw.z + (inw ? l : 0);
                double2 a = rw[2 * lw], b = rw[2 * lw + 1];
                if (!inw) {
                    const double *g4 = &ftab[min(s, nlast)].x;
                    const double z = s <= nlast ? 1.0 : 0.0;
                    a = make_double2(z * g4[0], z * g4[1]);
                    b = make_double2(z * g4[2], z * g4[3]);
                }
                const double v = ((b.y * t + b.x) * t + a.y) * t + a.x;
                acc += (kNodeCut || r2 < rc2) ? v : 0.0;
            }
            const int64_t idx = (int64_t)p * G.ncell + ((int64_t)gz * G.ny + gy) * G.nx + gx;
            double fpv = 0.0;
            bool beyond = false;
            if (pi.x > VACANT_TEST) {
                acc = 0.0;
            } else {
                double Fv;
                fpv = emb_eval<double>(acc, etab, em, Fv, beyond);
            }
            ((double *)P.rho)[idx] = acc;  // float64 arrays on a float64 handle
            ((double *)P.fp)[idx] = fpv;
            if (beyond) atomicAdd(P.range_viol, 1u);
        }
        item = nxt;
    }
}

static Tables<double> t64_tab(const misa_lattice *h) {
    Tables<double> T;
    T.f = h->t64.f;
    T.force = h->t64.force;
    T.phi = h->t64.phi;
    T.emb = h->t64.emb;
    T.fm = h->t64.fm;
    T.em = h->t64.em;
    T.force6 = h->t64.force6;
    return T;
}

// Float64 force pass on the same persistent scheme.  The tile holds {x, y} and
// {z, F'} per site (32 bytes, 110.6 KiB for 8 x 8 x 8 cells), which leaves room for
// FWIN64_MAX dense force records (48 bytes each: f' and phi' as quadratics in t) and a
// zero record.  With 5000-point tables these are bands of the table around the five BCC
// neighbour shells within rc (BandWin64): a pair outside its stencil entry's band, as in
// a cascade, gathers its record from global memory; the branch is nearly always uniform
// across a wave, whose lanes share one stencil offset.  Per-tile partials use the
// 8 x 8 x 8 tiling.
struct TileRegs64 {
    double x[TILE2_PER_LANE], y[TILE2_PER_LANE], z[TILE2_PER_LANE], w[TILE2_PER_LANE];
};

__device__ __forceinline__ void fetch_tile64(TileRegs64 &R, const PassPtrs &P, const TileGeo &g, const Dims &d,
                                             int tid) {
    const double *__restrict__ fp = (const double *)P.fp;  // float64 arrays on a float64 handle
    const int tx = tid % g.nt0;
    const int tyz = tid / g.nt0;
    const int ty = tyz % g.nt1;
    const int tz = tyz / g.nt1;
    const int bx = tx * d.tx - HALO, by = ty * d.ty - HALO, bz = tz * d.tz - HALO;
#pragma unroll
    for (int j = 0; j < TILE2_PER_LANE; ++j) {
        const int e = threadIdx.x + j * TILE2_THREADS;
        if (e < d.sites) {
            const int r = e / d.px;
            const int lx = e - r * d.px;
            const int r2 = r / d.py;
            const int ly = r - r2 * d.py;
            const int p = r2 / d.pz;
            const int lz = r2 - p * d.pz;
            const int gx = wrap2(bx + lx, g.nx), gy = wrap2(by + ly, g.ny), gz = wrap2(bz + lz, g.nz);
            const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
            R.x[j] = P.ux[idx];
            R.y[j] = P.uy[idx];
            R.z[j] = P.uz[idx];
            R.w[j] = fp[idx];
        }
    }
}

__device__ __forceinline__ float store_tile64w(double2 *__restrict__ txy, double2 *__restrict__ tzw,
                                               const TileRegs64 &R, int sites) {
    float m = 0.0f;
#pragma unroll
    for (int j = 0; j < TILE2_PER_LANE; ++j) {
        const int e = threadIdx.x + j * TILE2_THREADS;
        if (e < sites) {
            txy[e] = make_double2(R.x[j], R.y[j]);
            tzw[e] = make_double2(R.z[j], R.w[j]);
            if (R.x[j] < VACANT_TEST) m = fmaxf(m, (float)(R.x[j] * R.x[j] + R.y[j] * R.y[j] + R.z[j] * R.z[j]));
        }
    }
    return m;
}

// F_i = sum_j [(F'_i + F'_j) f'(r) + phi'(r)] (x_j - x_i) / r  (Eq. eam_force_ij), float64,
// with the fused second half-kick and per-tile partials as in k_force_lds.
// recs, nrec: the LDS records in LDS order; band: per parity and stencil entry, the
// segments held and where (BandWin64).
template <bool kEnergy, bool kKick, bool kNodeCut>
__global__ __launch_bounds__(TILE2_THREADS) void k_force_lds64(OneBox src, const StencilEntry<double> *__restrict__ st,
                                                              int K, int kin, float u_cut2, Tables<double> T,
                                                              const double2 *__restrict__ recs, int nrec,
                                                              const int4 *__restrict__ band, double rc2, double kf) {
    __shared__ double2 txy[TILE2_SITES];
    __shared__ double2 tzw[TILE2_SITES];
    __shared__ double2 fw[3 * (FWIN64_MAX + 1)];
    __shared__ double red[4][TILE2_THREADS / 64];
    __shared__ unsigned umax_slot[2];
    if (threadIdx.x < 2) umax_slot[threadIdx.x] = 0u;
    const double2 *__restrict__ f6 = reinterpret_cast<const double2 *>(T.force6);
    for (int e = threadIdx.x; e < 3 * nrec; e += TILE2_THREADS) fw[e] = recs[e];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p = __builtin_amdgcn_readfirstlane(w >> 3);
    TileGeo Gf{};
    const Dims d = dims_of<OneBox>(Gf);
    const LaneSite L = lane_site(d, p, w, lane);
    const StencilEntry<double> *sp = st + p * KMAX;
    const int4 *bp = band + p * KMAX;
    const int nlast = T.fm.nseg - 1;
    // pp = (r - x0) / h, capped at nseg (kNodeCut: the zero record) or at the last node
    const double pc0 = -T.fm.x0 * T.fm.inv_h;
    const double dtop = kNodeCut ? (double)T.fm.nseg : (double)nlast + 1.0;
    int it = 0;
    int item = src.next(blockIdx.x, it, gridDim.x);
    TileRegs64 R;
    if (item >= 0) {
        TileGeo G0;
        PassPtrs P0;
        const int t0 = src.get(item, G0, P0);
        fetch_tile64(R, P0, G0, d, t0);
    }
    while (item >= 0) {
        TileGeo G;
        PassPtrs P;
        const int tid = src.get(item, G, P);
        __syncthreads();  // previous tile fully consumed (and the window copied)
        const float m = store_tile64w(txy, tzw, R, d.sites);
        const int Kt = tile_stencil_length(m, &umax_slot[it & 1], &umax_slot[(it + 1) & 1], K, kin, u_cut2);
        ++it;
        const int nxt = src.next(blockIdx.x, it, gridDim.x);
        if (nxt >= 0) {
            TileGeo Gn;
            PassPtrs Pn;
            const int ntid = src.get(nxt, Gn, Pn);
            fetch_tile64(R, Pn, Gn, d, ntid);  // in flight during this tile
        }
        const double hk = kKick ? 0.5 * P.scal[0] * kf : 0.0;
        const int tx = tid % G.nt0;
        const int tyz = tid / G.nt0;
        const int gx = tx * d.tx + L.lx, gy = (tyz % G.nt1) * d.ty + L.ly, gz = (tyz / G.nt1) * d.tz + L.lz;
        const bool active = gx < G.nx && gy < G.ny && gz < G.nz;
        const int64_t idx = (int64_t)p * G.ncell + ((int64_t)gz * G.ny + gy) * G.nx + gx;
        double e_emb = 0.0, e_pair = 0.0, kvm = 0.0, kvs = 0.0;
        if (active) {
            const int me = L.me;
            const double2 pi = txy[me];
            const double2 zwi = tzw[me];
            double ax = 0.0, ay = 0.0, az = 0.0, ep = 0.0;
#pragma unroll 2
            for (int k = 0; k < Kt; ++k) {
                const StencilEntry<double> e = sp[k];
                const double2 pj = txy[me + e.lds];
                const double2 zwj = tzw[me + e.lds];
                const double dx = (pj.x - pi.x) + e.ox;
                const double dy = (pj.y - pi.y) + e.oy;
                const double dz = (zwj.x - zwi.x) + e.oz;
                const double r2 = dx * dx + dy * dy + dz * dz;
                double r, rinv;
                sqrt_rsqrt_nr1(r2, r, rinv);
                // table segment s and offset t; with kNodeCut pairs at or past the cut-off
                // (the last node) take s = nseg, whose LDS record is zero
                const double pp = fmin(fma(r, T.fm.inv_h, pc0), dtop);
                const int s = max((int)pp, 0);
                const double t = pp - (double)s;
                // this entry's band of LDS records, else global memory (zeros past the last
                // segment: pairs at or past the cut-off)
                const int4 bw = bp[k];
                const int l = s - bw.x;
                const bool inw = (unsigned)l < (unsigned)bw.y;
                // {f'0, f'1}, {f'2, phi'0}, {phi'1, phi'2}: read from LDS unconditionally (a
                // select between the two sources would turn every read into a generic load
                // through the vector memory path), replaced from global memory outside the band
                const int lw = bw.z + (inw ? l : 0);
                double2 q0 = fw[3 * lw], q1 = fw[3 * lw + 1], q2 = fw[3 * lw + 2];
                if (!inw) {  // read as scalars: keeps the compiler from merging it with the LDS read
                    const double *g6 = T.force6 + 6 * min(s, nlast);
                    const double z = s <= nlast ? 1.0 : 0.0;
                    q0 = make_double2(z * g6[0], z * g6[1]);
                    q1 = make_double2(z * g6[2], z * g6[3]);
                    q2 = make_double2(z * g6[4], z * g6[5]);
                }
                const double dfr = (q1.x * t + q0.y) * t + q0.x;
                const double dph = (q2.y * t + q2.x) * t + q1.y;
                double sc = ((zwi.y + zwj.y) * dfr + dph) * rinv;
                if (!kNodeCut) sc = r2 < rc2 ? sc : 0.0;
                ax += sc * dx;
                ay += sc * dy;
                az += sc * dz;
                if (kEnergy) {  // last step only
                    const bool in = kNodeCut ? s < nlast + 1 : r2 < rc2;
                    const Q4<double> c = T.phi[min(s, nlast)];
                    const double v = ((c.w * t + c.z) * t + c.y) * t + c.x;
                    ep += in ? v : 0.0;
                }
            }
            const bool vac = pi.x > VACANT_TEST;
            if (vac) ax = ay = az = 0.0;
            double *fxo = (double *)P.fx;  // float64 arrays on a float64 handle
            double *fyo = (double *)P.fy;
            double *fzo = (double *)P.fz;
            fxo[idx] = ax;
            fyo[idx] = ay;
            fzo[idx] = az;
            if (kKick && !vac) {
                const double v0x = P.vx[idx], v0y = P.vy[idx], v0z = P.vz[idx];
                const uint32_t mw = P.mark[idx >> 5];
                const double vx = v0x + hk * ax;
                const double vy = v0y + hk * ay;
                const double vz = v0z + hk * az;
                P.vx[idx] = vx;
                P.vy[idx] = vy;
                P.vz[idx] = vz;
                if (!((mw >> (idx & 31)) & 1u)) {
                    kvm = vx * vx + vy * vy + vz * vz;
                    kvs = kvm;
                }
            }
            if (kEnergy && !vac) {
                double Fv;
                bool beyond = false;
                emb_eval<double>(((const double *)P.rho)[idx], T.emb, T.em, Fv, beyond);
                e_emb = Fv;
                e_pair = 0.5 * ep;
            }
        }
        if (kEnergy || kKick) {
            if (kEnergy) {
                e_emb = wave_sum_l(e_emb);
                e_pair = wave_sum_l(e_pair);
            }
            if (kKick) {
                kvm = wave_max_l(kvm);
                kvs = wave_sum_l(kvs);
            }
            if (lane == 0) {
                red[0][w] = e_emb;
                red[1][w] = e_pair;
                red[2][w] = kvm;
                red[3][w] = kvs;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                double s0 = 0.0, s1 = 0.0, m2 = 0.0, s3 = 0.0;
                for (int q = 0; q < TILE2_THREADS / 64; ++q) {
                    s0 += red[0][q];
                    s1 += red[1][q];
                    m2 = fmax(m2, red[2][q]);
                    s3 += red[3][q];
                }
                if (kEnergy) {
                    P.part[2 * tid] = s0;
                    P.part[2 * tid + 1] = s1;
                }
                if (kKick) {
                    P.part_kick[2 * tid] = m2;
                    P.part_kick[2 * tid + 1] = s3;
                }
            }
        }
        item = nxt;
    }
}

bool lds64f_path(const misa_lattice *h) {
    return h->precision == MISA_FP64 && !h->use_mlp && h->persistent_grid > 0 && h->g.nsites > 0 &&
           h->fwin64.nrec > 0;
}

template <bool kEnergy, bool kKick>
static void force_lds64_variant(misa_lattice *h) {
    // the tables' last node at rc: pairs past it read the zero record instead of a select
    const bool node_cut = std::fabs(h->t64.fm.x_last - h->g.rc) <= 1e-12 * h->g.rc;
    auto kern = node_cut ? k_force_lds64<kEnergy, kKick, true> : k_force_lds64<kEnergy, kKick, false>;
    hipLaunchKernelGGL(kern, dim3(h->persistent_grid), dim3(TILE2_THREADS), 0, h->stream, one_box(h), h->st64p, h->K,
                       h->K_in, h->u_cut2, t64_tab(h), h->fwin64.recs, h->fwin64.nrec, h->fwin64.band, h->g.rc2,
                       ACC_UNIT / h->mass);
}

hipError_t launch_force_lds64(misa_lattice *h, bool energy, bool kick) {
    if (energy && kick) force_lds64_variant<true, true>(h);
    else if (energy) force_lds64_variant<true, false>(h);
    else if (kick) force_lds64_variant<false, true>(h);
    else force_lds64_variant<false, false>(h);
    return hipGetLastError();
}

bool lds64_path(const misa_lattice *h) {
    return h->precision == MISA_FP64 && !h->use_mlp && h->rwin64.nrec > 0 && h->persistent_grid > 0;
}

hipError_t launch_rho_lds64(misa_lattice *h) {
    OneBox o = one_box(h);
    const bool node_cut = std::fabs(h->t64.fm.x_last - h->g.rc) <= 1e-12 * h->g.rc;
    auto kern = node_cut ? k_rho_lds64<true> : k_rho_lds64<false>;
    hipLaunchKernelGGL(kern, dim3(h->persistent_grid), dim3(TILE2_THREADS), 0, h->stream, o, h->st64p, h->K, h->K_in,
                       h->u_cut2, h->rwin64.recs, h->rwin64.nrec, h->rwin64.band, h->t64.f, h->t64.fm, h->t64.emb,
                       h->t64.em, h->g.rc2);
    return hipGetLastError();
}

static Tables<float> t32_tab(const misa_lattice *h) {
    Tables<float> T;
    T.f = h->t32.f;
    T.force = h->t32.force;
    T.phi = h->t32.phi;
    T.emb = h->t32.emb;
    T.fm = h->t32.fm;
    T.em = h->t32.em;
    return T;
}

// h: the handle whose stencil and tables serve (every box of a batch shares them).
template <class Src>
static hipError_t rho_lds_src(misa_lattice *h, const Src &src, int grid, const StencilEntry<float> *st) {
    auto kern = h->lds32.node_cut ? k_rho_lds<Src, true> : k_rho_lds<Src, false>;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(TILE2_THREADS), 0, h->stream, src, st, h->K, h->K_in,
                       h->u_cut2, h->lds32.lf, h->lds32.inv_hq, h->lds32.pcq, h->lds32.nwin, h->t32.emb, h->t32.em,
                       (float)h->g.rc2, near_args(h, false));
    return hipGetLastError();
}

template <class Src, bool kEnergy, bool kKick>
static void force_lds_variant(misa_lattice *h, const Src &src, int grid, const StencilEntry<float> *st) {
    auto kern = h->lds32.node_cut ? k_force_lds<Src, kEnergy, true, kKick> : k_force_lds<Src, kEnergy, false, kKick>;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(TILE2_THREADS), 0, h->stream, src, st, h->K, h->K_in,
                       h->u_cut2, h->lds32.lg, h->lds32.inv_hq, h->lds32.pcq, h->lds32.nwin, t32_tab(h),
                       (float)h->g.rc2, ACC_UNIT / h->mass);
}

template <class Src>
static hipError_t force_lds_src(misa_lattice *h, const Src &src, int grid, bool energy, bool kick,
                                const StencilEntry<float> *st) {
    if (energy && kick) force_lds_variant<Src, true, true>(h, src, grid, st);
    else if (energy) force_lds_variant<Src, true, false>(h, src, grid, st);
    else if (kick) force_lds_variant<Src, false, true>(h, src, grid, st);
    else force_lds_variant<Src, false, false>(h, src, grid, st);
    return hipGetLastError();
}

hipError_t launch_rho_lds(misa_lattice *h) { return rho_lds_src(h, one_box(h), h->persistent_grid, h->st32p); }

hipError_t launch_force_lds(misa_lattice *h, bool energy, bool kick) {
    return force_lds_src(h, one_box(h), h->persistent_grid, energy, kick, h->st32p);
}

hipError_t launch_rho_lds_batch(misa_lattice *h0, const BoxPass *boxes, const int2 *items, int nitems,
                                const StencilEntry<float> *st_shapes, bool any_shape) {
    if (any_shape) {
        ManyBoxesT<true> m{boxes, items, nitems, (nitems + 7) / 8 * 8};
        return rho_lds_src(h0, m, h0->persistent_grid, st_shapes);
    }
    ManyBoxesT<false> m{boxes, items, nitems, (nitems + 7) / 8 * 8};
    return rho_lds_src(h0, m, h0->persistent_grid, st_shapes);
}

hipError_t launch_force_lds_batch(misa_lattice *h0, const BoxPass *boxes, const int2 *items, int nitems,
                                  bool energy, bool kick, const StencilEntry<float> *st_shapes, bool any_shape) {
    if (any_shape) {
        ManyBoxesT<true> m{boxes, items, nitems, (nitems + 7) / 8 * 8};
        return force_lds_src(h0, m, h0->persistent_grid, energy, kick, st_shapes);
    }
    ManyBoxesT<false> m{boxes, items, nitems, (nitems + 7) / 8 * 8};
    return force_lds_src(h0, m, h0->persistent_grid, energy, kick, st_shapes);
}

}  // namespace misa

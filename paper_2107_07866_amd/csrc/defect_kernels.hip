// Direct defect analysis from the lattice store (Wigner-Seitz count).
//
// The paper names direct defect analysis as a feature of MISA-MD (Sec. 1) and
// counts the defects a cascade leaves (Sec. 5.1).  The Lattice List makes the
// Wigner-Seitz count almost free: a slotted atom lies within delta of its site,
// so it sits in that site's cell; only the run-away atoms need the nearest-site
// rule.  A site is a vacancy if its slot is empty and no run-away atom is
// nearest to it; every atom beyond the first in a cell is an interstitial.
#include "misa_internal.h"

namespace misa {

constexpr int DEF_THREADS = 256;

__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t *sh) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t t = 0;
    for (int k = 0; k < DEF_THREADS / 64; ++k) t += sh[k];
    return t;
}

// out[0] += empty slots (integer atomics: the total does not depend on the order)
__global__ __launch_bounds__(DEF_THREADS) void k_count_empty(State S, Geom g, unsigned long long *out) {
    __shared__ int64_t sh[DEF_THREADS / 64];
    int64_t c = 0;
    for (int64_t s = (int64_t)blockIdx.x * DEF_THREADS + threadIdx.x; s < g.nsites;
         s += (int64_t)gridDim.x * DEF_THREADS)
        c += S.atom[s] == VACANT_ID ? 1 : 0;
    const int64_t t = block_sum_i64(c, sh);
    if (threadIdx.x == 0 && t) atomicAdd(out, (unsigned long long)t);
}

// Nearest site of every run-away atom as a sort key (site << 32 | list position).
__global__ void k_runaway_site_keys(State S, Scratch sc, Geom g) {
    const int n = sc.cnt->n_run;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const double x[3] = {S.r_x[r], S.r_y[r], S.r_z[r]};
        double u[3], u2;
        const int64_t s = hash_site(x, g, u, &u2);
        sc.sortbuf[r] = ((uint64_t)s << 32) | (uint32_t)r;
    }
}

// One work-group: sort the keys (bitonic; in LDS when they fit), then walk the runs
// of equal sites.  out[1] += run-away atoms in cells whose slot is occupied or that
// hold more than one of them (interstitials); out[2] += empty slots they fill.
constexpr int DEF_SORT_LDS = 8192;
__global__ __launch_bounds__(1024) void k_runaway_cells(State S, Scratch sc, unsigned long long *out) {
    __shared__ uint64_t sh[DEF_SORT_LDS];
    __shared__ unsigned long long acc[2];
    const int n = sc.cnt->n_run;
    if (threadIdx.x < 2) acc[threadIdx.x] = 0;
    int P = 1;
    while (P < n) P <<= 1;
    const bool in_lds = P <= DEF_SORT_LDS;
    uint64_t *A = in_lds ? sh : sc.sortbuf;  // sortbuf holds next_pow2(capacity) entries
    for (int i = threadIdx.x; i < P; i += 1024) {
        if (in_lds)
            sh[i] = i < n ? sc.sortbuf[i] : ~0ull;
        else if (i >= n)
            sc.sortbuf[i] = ~0ull;
    }
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += 1024) {
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
    unsigned long long inter = 0, filled = 0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        const uint32_t site = (uint32_t)(A[i] >> 32);
        if (i > 0 && (uint32_t)(A[i - 1] >> 32) == site) continue;  // not the start of a run
        int len = 1;
        while (i + len < n && (uint32_t)(A[i + len] >> 32) == site) ++len;
        const bool occupied = S.atom[site] != VACANT_ID;
        inter += occupied ? len : len - 1;
        filled += occupied ? 0 : 1;
    }
    atomicAdd(&acc[0], inter);
    atomicAdd(&acc[1], filled);
    __syncthreads();
    if (threadIdx.x == 0) {
        out[1] += acc[0];
        out[2] += acc[1];
    }
}

// out (device, 3 counters, zeroed by the caller): empty slots, interstitials, filled empty slots.
hipError_t launch_defects(misa_lattice *h, unsigned long long *out) {
    const Geom &g = h->g;
    const int64_t b = std::min<int64_t>((g.nsites + DEF_THREADS - 1) / DEF_THREADS, 4096);
    hipLaunchKernelGGL(k_count_empty, dim3(b > 0 ? b : 1), dim3(DEF_THREADS), 0, h->stream, h->S, g, out);
    hipLaunchKernelGGL(k_runaway_site_keys, dim3(SMALL_GRID), dim3(256), 0, h->stream, h->S, h->sc, g);
    hipLaunchKernelGGL(k_runaway_cells, dim3(1), dim3(1024), 0, h->stream, h->S, h->sc, out);
    return hipGetLastError();
}

}  // namespace misa

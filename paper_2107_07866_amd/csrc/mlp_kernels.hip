// Learned form: surrogate networks for f, phi and F.
//
// (1) Lattice passes.  The rho and force passes of the float32 form with every
//     table look-up of a lattice pair replaced by a network evaluation.  A wave
//     holds 64 sites and so, per stencil offset, 64 pair distances; the 32 x 32
//     middle layer of those 64 evaluations runs on the matrix cores as
//     Z2^T = W2 H1^T in two 32-column blocks (v_mfma_f32_32x32x8 bf16, float32
//     accumulation).  W2 is the A operand, held in registers for the whole kernel;
//     lanes l and l + 32 share a column and each computes the half of the first
//     layer that its B-operand slots hold, so no transposition is needed.  The
//     bfloat16 B operands carry each activation as a sum of two bfloat16 terms.
//     Inputs outside a network's range take the float32 table instead.
// (2) Training.  Per-sample float32 forward and backward passes of one network
//     (the backward pass goes through the input tangent, since the loss involves
//     g'), per-block partial gradients combined in a fixed order, and Adam.
// (3) Force matching.  Forces of sampled atoms from their pair lists with the
//     f and phi networks, and the per-pair coefficients of the force loss.
#include "misa_internal.h"

#include "mlp_device.h"
#include "mlp_wave.h"

namespace misa {

__device__ __forceinline__ int wrapm(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

__device__ __forceinline__ void load_tile_f(Q4<float> *__restrict__ tile, const double *__restrict__ ux,
                                            const double *__restrict__ uy, const double *__restrict__ uz,
                                            const float *__restrict__ w_src, const Geom &g, int bx, int by,
                                            int bz) {
    for (int e = threadIdx.x; e < TILE_SITES; e += TILE_THREADS) {
        const int lx = e % PX;
        int r = e / PX;
        const int ly = r % PY;
        r /= PY;
        const int lz = r % PZ;
        const int p = r / PZ;
        const int gx = wrapm(bx + lx, g.nx), gy = wrapm(by + ly, g.ny), gz = wrapm(bz + lz, g.nz);
        const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
        Q4<float> q;
        q.x = (float)ux[idx];
        q.y = (float)uy[idx];
        q.z = (float)uz[idx];
        q.w = w_src ? w_src[idx] : 0.0f;
        tile[e] = q;
    }
}

struct MlpSet {
    MlpNet net[3];
    const uint16_t *w2b[3];  // W2 of each network as bfloat16 bits
};

// rho_i = sum_j f(r_ij) and F'(rho_i) with the networks.  Every lane of a wave runs
// the pair loop (the matrix-core evaluation needs the whole wave); lanes outside the
// box compute on wrapped data and store nothing.  The f network runs with its
// tangent, and f'(r) of every candidate goes to dfbuf (candidate k of site i at
// k nsites + i), so that the force pass only runs the phi network.
__global__ __launch_bounds__(TILE_THREADS) void k_rho_mlp(const double *__restrict__ ux,
                                                          const double *__restrict__ uy,
                                                          const double *__restrict__ uz, float *__restrict__ rho,
                                                          float *__restrict__ fp,
                                                          const StencilEntry<float> *__restrict__ st, int K,
                                                          Tables<float> T, MlpSet M, Geom g,
                                                          uint32_t *__restrict__ range_viol,
                                                          float *__restrict__ dfbuf, const NearTab *__restrict__ nt) {
    __shared__ Q4<float> tile[TILE_SITES];
    __shared__ MlpLds Lf, Le;
    const int tid = tile_of_block(blockIdx.x, g);
    if (tid >= g.ntiles) return;  // whole work-group leaves together
    const int tx = tid % g.ntx;
    const int tyz = tid / g.ntx;
    const int ty = tyz % g.nty;
    const int tz = tyz / g.nty;
    load_tile_f(tile, ux, uy, uz, nullptr, g, tx * TX - HALO, ty * TY - HALO, tz * TZ - HALO);
    fill_lds(Lf, M.net[0].p);
    fill_lds(Le, M.net[2].p);
    bf16x4_t Af[4], Ae[4];
    load_a(Af, M.w2b[0]);
    load_a(Ae, M.w2b[2]);
    __syncthreads();

    const MlpNet nf = M.net[0], ne = M.net[2];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p = __builtin_amdgcn_readfirstlane(w / TZ);
    const int lz = w % TZ, lx = lane % TX, ly = lane / TX;
    const int gx = tx * TX + lx, gy = ty * TY + ly, gz = tz * TZ + lz;
    const bool active = gx < g.nx && gy < g.ny && gz < g.nz;
    const int me = ((p * PZ + lz + HALO) * PY + ly + HALO) * PX + lx + HALO;
    const Q4<float> ui = tile[me];
    const float rc2 = (float)g.rc2;
    const StencilEntry<float> *sp = st + p * KMAX;
    const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
    const float kfd = nf.y_scale * nf.s;
    float acc = 0.0f;
    for (int k = 0; k < K; ++k) {
        const StencilEntry<float> e = sp[k];
        const Q4<float> uj = tile[me + e.lds];
        const float dx = (uj.x - ui.x) + e.ox;
        const float dy = (uj.y - ui.y) + e.oy;
        const float dz = (uj.z - ui.z) + e.oz;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float r = r2 * rinv;  // as the force pass forms it, so both passes see the same r
        float y, dyt;
        mlp_wave<true>(Lf, Af, net_t(nf, r), y, dyt);
        float dfr = 0.0f;
        bool in = r2 < rc2;
        if (active && fabsf(r2 - rc2) < RC_BAND_Q)  // cut-off decided again in float64 (NearTab)
            in = pair_in_rc64(ux, uy, uz, idx, gx, gy, gz, p, nt->st[p][k], g.nx, g.ny, g.nz, g.ncell, nt->rc2);
        if (in) {
            float v = nf.y_shift + nf.y_scale * y;
            dfr = kfd * dyt;
            if (!mlp_serves(nf, r)) {
                int s;
                float t;
                seg32(r, T.fm, s, t);
                const Q4<float> c = T.f[s];
                v = ((c.w * t + c.z) * t + c.y) * t + c.x;
                const Q4<float> a = T.force[2 * s];
                dfr = (a.z * t + a.y) * t + a.x;
            }
            acc += v;
        }
        if (active) dfbuf[(int64_t)k * g.nsites + idx] = dfr;
    }
    const bool vac = ui.x > (float)VACANT_TEST;
    if (vac) acc = 0.0f;
    float ye, de;
    mlp_wave<true>(Le, Ae, net_t(ne, acc), ye, de);
    float fpv = ne.y_scale * ne.s * de;
    bool beyond = false;
    if (!mlp_serves(ne, acc)) {
        float Fv;
        fpv = emb_tab(acc, T, Fv, beyond);
    }
    if (vac) fpv = 0.0f;
    if (active) {
        rho[idx] = acc;
        fp[idx] = fpv;
        if (beyond) atomicAdd(range_viol, 1u);
    }
}

__device__ __forceinline__ double wave_sum_m(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// F_i = sum_j [(F'_i + F'_j) f'(r) + phi'(r)] (x_j - x_i) / r with the networks;
// with kEnergy, per-tile sums of F(rho_i) and 1/2 sum_j phi(r_ij).
template <bool kEnergy>
__global__ __launch_bounds__(TILE_THREADS) void k_force_mlp(
    const double *__restrict__ ux, const double *__restrict__ uy, const double *__restrict__ uz,
    const float *__restrict__ fp, const float *__restrict__ rho, float *__restrict__ fx, float *__restrict__ fy,
    float *__restrict__ fz, const StencilEntry<float> *__restrict__ st, int K, Tables<float> T, MlpSet M, Geom g,
    double *__restrict__ part, const float *__restrict__ dfbuf, const NearTab *__restrict__ nt) {
    __shared__ Q4<float> tile[TILE_SITES];
    __shared__ MlpLds Lp, Le;
    __shared__ double red[2][TILE_THREADS / 64];
    const int tid = tile_of_block(blockIdx.x, g);
    if (tid >= g.ntiles) return;
    const int tx = tid % g.ntx;
    const int tyz = tid / g.ntx;
    const int ty = tyz % g.nty;
    const int tz = tyz / g.nty;
    load_tile_f(tile, ux, uy, uz, fp, g, tx * TX - HALO, ty * TY - HALO, tz * TZ - HALO);
    fill_lds(Lp, M.net[1].p);
    if (kEnergy) fill_lds(Le, M.net[2].p);
    bf16x4_t Ap[4];
    load_a(Ap, M.w2b[1]);
    __syncthreads();

    const MlpNet np = M.net[1];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int p = __builtin_amdgcn_readfirstlane(w / TZ);
    const int lz = w % TZ, lx = lane % TX, ly = lane / TX;
    const int gx = tx * TX + lx, gy = ty * TY + ly, gz = tz * TZ + lz;
    const bool active = gx < g.nx && gy < g.ny && gz < g.nz;
    const int me = ((p * PZ + lz + HALO) * PY + ly + HALO) * PX + lx + HALO;
    const Q4<float> ui = tile[me];
    const float rc2 = (float)g.rc2;
    const StencilEntry<float> *sp = st + p * KMAX;
    const float kp = np.y_scale * np.s;
    const int64_t idx = (int64_t)p * g.ncell + ((int64_t)gz * g.ny + gy) * g.nx + gx;
    float ax = 0.0f, ay = 0.0f, az = 0.0f, ep = 0.0f;
    for (int k = 0; k < K; ++k) {
        const StencilEntry<float> e = sp[k];
        const Q4<float> uj = tile[me + e.lds];
        const float dx = (uj.x - ui.x) + e.ox;
        const float dy = (uj.y - ui.y) + e.oy;
        const float dz = (uj.z - ui.z) + e.oz;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float rinv = __builtin_amdgcn_rsqf(r2);
        const float r = r2 * rinv;
        const float dfr = active ? dfbuf[(int64_t)k * g.nsites + idx] : 0.0f;  // f'(r) from the rho pass
        float yp, dp;
        mlp_wave<true>(Lp, Ap, net_t(np, r), yp, dp);
        bool in = r2 < rc2;
        if (active && fabsf(r2 - rc2) < RC_BAND_Q)  // cut-off decided again in float64 (NearTab)
            in = pair_in_rc64(ux, uy, uz, idx, gx, gy, gz, p, nt->st[p][k], g.nx, g.ny, g.nz, g.ncell, nt->rc2);
        if (in) {
            float dph = kp * dp, ph = np.y_shift + np.y_scale * yp;
            if (!mlp_serves(np, r)) {
                int s;
                float t;
                seg32(r, T.fm, s, t);
                const Q4<float> a = T.force[2 * s], b = T.force[2 * s + 1];
                dph = (b.y * t + b.x) * t + a.w;
                const Q4<float> c = T.phi[s];
                ph = ((c.w * t + c.z) * t + c.y) * t + c.x;
            }
            const float sc = ((ui.w + uj.w) * dfr + dph) * rinv;
            ax += sc * dx;
            ay += sc * dy;
            az += sc * dz;
            if (kEnergy) ep += ph;
        }
    }
    const bool vac = ui.x > (float)VACANT_TEST;
    if (vac) ax = ay = az = 0.0f;
    if (active) {
        fx[idx] = ax;
        fy[idx] = ay;
        fz[idx] = az;
    }
    if (kEnergy) {
        const MlpNet ne = M.net[2];
        bf16x4_t Ae[4];
        load_a(Ae, M.w2b[2]);
        const float rr = active ? rho[idx] : 0.0f;
        float ye, unused;
        mlp_wave<false>(Le, Ae, net_t(ne, rr), ye, unused);
        float Fv = ne.y_shift + ne.y_scale * ye;
        if (!mlp_serves(ne, rr)) {
            bool beyond = false;
            emb_tab(rr, T, Fv, beyond);
        }
        double e_emb = (active && !vac) ? (double)Fv : 0.0;
        double e_pair = (active && !vac) ? 0.5 * (double)ep : 0.0;
        e_emb = wave_sum_m(e_emb);
        e_pair = wave_sum_m(e_pair);
        if (lane == 0) {
            red[0][w] = e_emb;
            red[1][w] = e_pair;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s0 = 0.0, s1 = 0.0;
            for (int q = 0; q < TILE_THREADS / 64; ++q) {
                s0 += red[0][q];
                s1 += red[1][q];
            }
            part[2 * tid] = s0;
            part[2 * tid + 1] = s1;
        }
    }
}

static MlpSet mlp_set_of(const misa_lattice *h) {
    MlpSet M;
    for (int f = 0; f < 3; ++f) {
        M.net[f] = h->mlp.net[f];
        M.w2b[f] = h->mlp.w2b[f];
    }
    return M;
}

static Tables<float> t32_tables(const misa_lattice *h) {
    Tables<float> T;
    T.f = h->t32.f;
    T.force = h->t32.force;
    T.phi = h->t32.phi;
    T.emb = h->t32.emb;
    T.fm = h->t32.fm;
    T.em = h->t32.em;
    return T;
}

hipError_t launch_rho_mlp(misa_lattice *h) {
    if (!h->pairbuf) return hipErrorInvalidValue;  // made by misa_set_mlp
    const Geom &g = h->g;
    hipLaunchKernelGGL(k_rho_mlp, dim3(g.ntiles_pad), dim3(TILE_THREADS), 0, h->stream, h->S.ux, h->S.uy, h->S.uz,
                       (float *)h->S.rho, (float *)h->S.fp, h->st32, h->K, t32_tables(h), mlp_set_of(h), g,
                       &h->sc.cnt->range_viol, h->pairbuf, near_args(h, false));
    return hipGetLastError();
}

hipError_t launch_force_mlp(misa_lattice *h, bool energy) {
    if (!h->pairbuf) return hipErrorInvalidValue;
    const Geom &g = h->g;
    auto kern = energy ? k_force_mlp<true> : k_force_mlp<false>;
    hipLaunchKernelGGL(kern, dim3(g.ntiles_pad), dim3(TILE_THREADS), 0, h->stream, h->S.ux, h->S.uy, h->S.uz,
                       (const float *)h->S.fp, (const float *)h->S.rho, (float *)h->S.fx, (float *)h->S.fy,
                       (float *)h->S.fz, h->st32, h->K, t32_tables(h), mlp_set_of(h), g, h->sc.part, h->pairbuf,
                       near_args(h, false));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Evaluation entry points of the trainer (the two forward paths).

__global__ void k_eval_lane(MlpNet m, const double *__restrict__ x, int64_t n, double *__restrict__ y,
                            double *__restrict__ dy) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float g, dg;
        mlp_eval_lane(m, (float)x[i], g, dg);
        y[i] = g;
        dy[i] = dg;
    }
}

// Matrix-core path: 64 points per wave; padding lanes repeat the last point.
__global__ __launch_bounds__(256) void k_eval_mfma(MlpNet m, const uint16_t *__restrict__ w2b,
                                                   const double *__restrict__ x, int64_t n, double *__restrict__ y,
                                                   double *__restrict__ dy) {
    __shared__ MlpLds L;
    fill_lds(L, m.p);
    bf16x4_t A[4];
    load_a(A, w2b);
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += stride) {  // uniform over the block
        const int64_t i = base + threadIdx.x;
        const float xi = (float)x[i < n ? i : n - 1];
        float yy, dd;
        mlp_wave<true>(L, A, (xi - m.c) * m.s, yy, dd);
        if (i < n) {
            y[i] = m.y_shift + m.y_scale * yy;
            dy[i] = m.y_scale * m.s * dd;
        }
    }
}

hipError_t launch_mlp_eval(hipStream_t st, int path, const MlpNet &m, const uint16_t *w2b, const double *x,
                           int64_t n, double *y, double *dy) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    if (path == 0)
        hipLaunchKernelGGL(k_eval_lane, dim3(blocks), dim3(256), 0, st, m, x, n, y, dy);
    else
        hipLaunchKernelGGL(k_eval_mfma, dim3(blocks), dim3(256), 0, st, m, w2b, x, n, y, dy);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Training: per-sample forward and backward passes, one sample per lane,
// GRAD_SAMPLES samples per block; per-block partial gradients.

constexpr int GS = MLP_H + 1;  // padded LDS row

__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    // Steele, Lea and Flood, "Fast splittable pseudorandom number generators" (2014)
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Partial gradient of block blk (samples blk GRAD_SAMPLES ..) into J.part[blk], and
// its Sobolev loss into J.loss_part[blk].  GRAD_SPLIT consecutive lanes serve one
// sample, each taking GRAD_UNITS of the hidden units of both layers (sums over a
// sample's units: a fixed butterfly over its lanes).
__device__ __forceinline__ float split_sum(float v) {
    for (int o = 1; o < GRAD_SPLIT; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void grad_block(const GradJob &J, int blk) {
    // weights and per-sample vectors in LDS (rows padded against bank conflicts)
    __shared__ float P[MLP_NP];
    __shared__ float sh1[GRAD_SAMPLES][GS], sd1[GRAD_SAMPLES][GS], sa1[GRAD_SAMPLES][GS];
    __shared__ float su[GRAD_SAMPLES][GS], sv[GRAD_SAMPLES][GS], sq[GRAD_SAMPLES][GS];
    __shared__ float sp1[GRAD_SAMPLES][GS], sz1[GRAD_SAMPLES][GS];
    __shared__ float scv[GRAD_SAMPLES];
    __shared__ double sloss[GRAD_SAMPLES];
    const int tid = threadIdx.x;
    const int b = tid / GRAD_SPLIT, u0 = (tid % GRAD_SPLIT) * GRAD_UNITS;  // sample, first unit of this lane
    for (int j = tid; j < MLP_NP; j += GRAD_THREADS) P[j] = J.p[j];
    const int64_t i = (int64_t)blk * GRAD_SAMPLES + b;
    const bool sob = J.cval == nullptr;
    const int64_t count = sob ? J.batch : J.n;
    const bool live = i < count;
    int64_t idx = i;
    if (sob)
        idx = live ? (int64_t)(splitmix64(J.seed ^ splitmix64(J.step * 0x100000001b3ull + (uint64_t)i)) %
                               (uint64_t)J.n)
                   : 0;
    else if (!live)
        idx = 0;
    const float t = ((float)J.x[idx] - J.c) * J.s;
    __syncthreads();
    // forward with tangents: layer 1
    for (int kk = 0; kk < GRAD_UNITS; ++kk) {
        const int k = u0 + kk;
        const float w = P[OFF_W1 + k];
        const float z = w * t + P[OFF_B1 + k];
        const float sg = sigm(z);
        const float h = z * sg;
        const float a = sg + h * (1.0f - sg);
        sh1[b][k] = h;
        sa1[b][k] = a;
        sd1[b][k] = a * w;
    }
    __syncthreads();
    // layer 2 and the output
    float y = 0.0f, dyt = 0.0f;
    for (int nn = 0; nn < GRAD_UNITS; ++nn) {
        const int n = u0 + nn;
        const float *w2 = P + OFF_W2 + n * MLP_H;
        float z = P[OFF_B2 + n], dz = 0.0f;
#pragma unroll 8
        for (int k = 0; k < MLP_H; ++k) {
            z += w2[k] * sh1[b][k];
            dz += w2[k] * sd1[b][k];
        }
        const float sg = sigm(z);
        const float h2 = z * sg;
        const float a2 = sg + h2 * (1.0f - sg);
        y += P[OFF_W3 + n] * h2;
        dyt += P[OFF_W3 + n] * a2 * dz;
        su[b][n] = z;   // z2 until the reverse pass
        sv[b][n] = dz;  // dz2 until the reverse pass
    }
    y = split_sum(y) + P[OFF_B3];
    dyt = split_sum(dyt);
    float cv, cd;
    double loss = 0.0;
    if (sob) {
        const float yn = (float)((J.y[idx] - (double)J.y_shift) / (double)J.y_scale);
        const float dn = (float)(J.dy[idx] / ((double)J.y_scale * (double)J.s));
        const float ey = y - yn, ed = dyt - dn;
        const float inv = 1.0f / (float)count;
        cv = live ? 2.0f * ey * inv : 0.0f;
        cd = live ? 2.0f * J.lam * ed * inv : 0.0f;
        loss = live ? (double)(ey * ey + J.lam * ed * ed) : 0.0;
    } else {
        cv = live ? (float)J.cval[idx] : 0.0f;
        cd = live ? (float)J.cder[idx] : 0.0f;
    }
    // reverse through layer 2 (this lane's output units)
    for (int nn = 0; nn < GRAD_UNITS; ++nn) {
        const int n = u0 + nn;
        const float z = su[b][n], dz = sv[b][n];
        const float sg = sigm(z);
        const float h2 = z * sg;
        const float a2 = sg + h2 * (1.0f - sg);
        const float s2 = sg * (1.0f - sg) * (2.0f + z * (1.0f - 2.0f * sg));  // silu''
        const float w3 = P[OFF_W3 + n];
        sq[b][n] = cv * h2 + cd * a2 * dz;         // d/dw3
        su[b][n] = cv * w3 * a2 + cd * w3 * dz * s2;  // d/dz2
        sv[b][n] = cd * w3 * a2;                   // d/d(dz2)
    }
    __syncthreads();
    // reverse through layer 1 (this lane's hidden units)
    for (int kk = 0; kk < GRAD_UNITS; ++kk) {
        const int k = u0 + kk;
        float gh = 0.0f, gd = 0.0f;
#pragma unroll 8
        for (int n = 0; n < MLP_H; ++n) {
            const float w = P[OFF_W2 + n * MLP_H + k];
            gh += w * su[b][n];
            gd += w * sv[b][n];
        }
        const float w1 = P[OFF_W1 + k];
        const float z = w1 * t + P[OFF_B1 + k];
        const float sg = sigm(z);
        const float s1 = sg * (1.0f - sg) * (2.0f + z * (1.0f - 2.0f * sg));
        const float a1 = sa1[b][k];
        const float gz1 = gh * a1 + gd * w1 * s1;
        sp1[b][k] = gd * a1 + gz1 * t;  // d/dW1
        sz1[b][k] = gz1;                // d/db1
    }
    if (u0 == 0) {
        scv[b] = cv;
        sloss[b] = loss;
    }
    __syncthreads();
    // block sums in a fixed order
    float *out = J.part + (int64_t)blk * MLP_NP;
    {
        constexpr int PER = MLP_H * MLP_H / GRAD_THREADS;  // entries of W2 per thread
        const int n = tid / (MLP_H / PER), k0 = (tid % (MLP_H / PER)) * PER;
        for (int j = 0; j < PER; ++j) {
            const int k = k0 + j;
            float s = 0.0f;
#pragma unroll 8
            for (int q = 0; q < GRAD_SAMPLES; ++q) s += su[q][n] * sh1[q][k] + sv[q][n] * sd1[q][k];
            out[OFF_W2 + n * MLP_H + k] = s;
        }
    }
    if (tid < MLP_H) {
        float g1 = 0.0f, gb1 = 0.0f, gb2 = 0.0f, gw3 = 0.0f;
        for (int q = 0; q < GRAD_SAMPLES; ++q) {
            g1 += sp1[q][tid];
            gb1 += sz1[q][tid];
            gb2 += su[q][tid];
            gw3 += sq[q][tid];
        }
        out[OFF_W1 + tid] = g1;
        out[OFF_B1 + tid] = gb1;
        out[OFF_B2 + tid] = gb2;
        out[OFF_W3 + tid] = gw3;
    }
    if (tid == MLP_H) {
        float g3 = 0.0f;
        for (int q = 0; q < GRAD_SAMPLES; ++q) g3 += scv[q];
        out[OFF_B3] = g3;
    }
    if (tid == MLP_H + 1 && J.loss_part) {
        double l = 0.0;
        for (int q = 0; q < GRAD_SAMPLES; ++q) l += sloss[q];
        J.loss_part[blk] = l;
    }
}

__global__ __launch_bounds__(GRAD_THREADS) void k_grad(GradJob J) { grad_block(J, blockIdx.x); }

// Adam on element j of a network's float32 master weights (q: the bfloat16 rounding).
__device__ __forceinline__ void adam_one(int j, double g, float *__restrict__ w, float *__restrict__ m,
                                         float *__restrict__ v, float *__restrict__ q, double lr, double bc1,
                                         double bc2) {
    const double mj = 0.9 * (double)m[j] + 0.1 * g;
    const double vj = 0.999 * (double)v[j] + 0.001 * g * g;
    m[j] = (float)mj;
    v[j] = (float)vj;
    const double step = lr * (mj / bc1) / (sqrt(vj / bc2) + 1e-8);
    const float wj = (float)((double)w[j] - step);
    w[j] = wj;
    q[j] = bf16_float(bf16_bits(wj));
}

// One fit iteration of up to three networks in one launch (blockIdx.y = network):
// every block writes its partial gradient; the block that finishes last for its
// network sums the partials in block order (float64, as k_grad_sum) and takes the
// Adam step (as k_adam), so an iteration is one launch and the GPU never waits on
// the host between the gradient and the update.  Counting the finished blocks is
// the only cross-block step; nothing waits on another block.
__global__ __launch_bounds__(GRAD_THREADS) void k_fit_step(FitSteps F) {
    const FitStep &S = F.s[blockIdx.y];
    if (S.nblk1 == 0 || (int)blockIdx.x < S.nblk1)
        grad_block(S.J, blockIdx.x);
    else
        grad_block(S.J2, blockIdx.x - S.nblk1);  // its partials follow J's: J2.part = J.part + nblk1 MLP_NP
    __shared__ int last;
    __threadfence();  // this block's partial gradient and loss, before the count
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(S.ticket, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    // agent-scope acquire: the other blocks' partials are read from L2 (this block has
    // not read them before, and the fence invalidates its L1)
    __threadfence();
    const float *part = S.J.part;
    for (int j = threadIdx.x; j < MLP_NP; j += GRAD_THREADS) {
        double g = 0.0;
        // all partials of element j in flight at once; summed in block order
#pragma unroll 64
        for (int q = 0; q < (int)gridDim.x; ++q) g += (double)part[(int64_t)q * MLP_NP + j];
        adam_one(j, g, S.w, S.m, S.v, S.q, F.lr, S.bc1, S.bc2);
    }
    if (threadIdx.x == 0) {
        if (S.slot >= 0) {
            const double *lp = S.J.loss_part;
            double l = 0.0;
            for (int q = 0; q < (int)gridDim.x; ++q) l += lp[q];
            S.loss_hist[S.slot] = l;
        }
        *S.ticket = 0;  // for the next iteration (a later launch on the same stream)
    }
}

// grad[j] = sum over blocks of part[blk][j] (fixed order), float64.
__global__ void k_grad_sum(const float *__restrict__ part, int nblk, double *__restrict__ grad) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < MLP_NP; j += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int q = 0; q < nblk; ++q) s += (double)part[(int64_t)q * MLP_NP + j];
        grad[j] = s;
    }
}

// Adam on the float32 master weights; q receives them rounded to bfloat16.
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const double *__restrict__ grad, float *__restrict__ q, double lr, double bc1, double bc2) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < MLP_NP; j += gridDim.x * blockDim.x)
        adam_one(j, grad[j], w, m, v, q, lr, bc1, bc2);
}

__global__ void k_round_weights(const float *__restrict__ w, float *__restrict__ q, uint16_t *__restrict__ w2b) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < MLP_NP; j += gridDim.x * blockDim.x) {
        const uint32_t b = bf16_bits(w[j]);
        q[j] = bf16_float(b);
        if (w2b && j >= OFF_W2 && j < OFF_W2 + MLP_H * MLP_H) w2b[j - OFF_W2] = (uint16_t)b;
    }
}

hipError_t launch_fit_step(hipStream_t st, const FitSteps &F, int nblk) {
    hipLaunchKernelGGL(k_fit_step, dim3(nblk, F.nnet), dim3(GRAD_THREADS), 0, st, F);
    return hipGetLastError();
}

hipError_t launch_grad(hipStream_t st, const GradJob &J, int nblk) {
    hipLaunchKernelGGL(k_grad, dim3(nblk), dim3(GRAD_THREADS), 0, st, J);
    return hipGetLastError();
}

hipError_t launch_grad_sum(hipStream_t st, const float *part, int nblk, double *grad) {
    hipLaunchKernelGGL(k_grad_sum, dim3((MLP_NP + 255) / 256), dim3(256), 0, st, part, nblk, grad);
    return hipGetLastError();
}

hipError_t launch_adam(hipStream_t st, float *w, float *m, float *v, const double *grad, float *q, double lr,
                       int64_t step) {
    const double bc1 = 1.0 - pow(0.9, (double)step), bc2 = 1.0 - pow(0.999, (double)step);
    hipLaunchKernelGGL(k_adam, dim3((MLP_NP + 255) / 256), dim3(256), 0, st, w, m, v, grad, q, lr, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_round_weights(hipStream_t st, const float *w, float *q, uint16_t *w2b) {
    hipLaunchKernelGGL(k_round_weights, dim3((MLP_NP + 255) / 256), dim3(256), 0, st, w, q, w2b);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Force matching

// One wave per sampled atom; lanes take slots lane and lane + 64.
__global__ __launch_bounds__(64) void k_fm(FmJob J) {
    const int q = blockIdx.x;
    if (q >= J.nb) return;
    const int e = J.envs[q];
    const int lane = threadIdx.x;
    const double fi = J.fpi[e];
    double F[3] = {0.0, 0.0, 0.0};
    float dfv[2] = {0.f, 0.f}, dpv[2] = {0.f, 0.f};
    for (int u = 0; u < 2; ++u) {
        const int slot = lane + 64 * u;
        if (slot >= MISA_FM_SLOTS) break;
        const int64_t o = (int64_t)e * MISA_FM_SLOTS + slot;
        const double r = J.r[o];
        J.x_out[(int64_t)q * MISA_FM_SLOTS + slot] = r;
        if (r <= 0.0) continue;
        float g, dg;
        mlp_eval_lane(J.nf, (float)r, g, dg);
        dfv[u] = dg;
        mlp_eval_lane(J.np, (float)r, g, dg);
        dpv[u] = dg;
        const double s = (fi + J.fpj[o]) * (double)dfv[u] + (double)dpv[u];
        for (int c = 0; c < 3; ++c) F[c] += s * J.dhat[3 * o + c];
    }
    for (int c = 0; c < 3; ++c) F[c] = wave_sum_m(F[c]);
    double res[3];
    for (int c = 0; c < 3; ++c) res[c] = F[c] - J.fref[3 * (int64_t)e + c];
    if (lane == 0) J.loss_part[q] = (res[0] * res[0] + res[1] * res[1] + res[2] * res[2]) * J.inv_norm;
    const double kf = (double)J.nf.y_scale * (double)J.nf.s, kp = (double)J.np.y_scale * (double)J.np.s;
    for (int u = 0; u < 2; ++u) {
        const int slot = lane + 64 * u;
        if (slot >= MISA_FM_SLOTS) break;
        const int64_t o = (int64_t)e * MISA_FM_SLOTS + slot;
        const int64_t w = (int64_t)q * MISA_FM_SLOTS + slot;
        const double r = J.r[o];
        double pf = 0.0, pp = 0.0;
        if (r > 0.0) {
            const double proj =
                2.0 * J.inv_norm * (res[0] * J.dhat[3 * o] + res[1] * J.dhat[3 * o + 1] + res[2] * J.dhat[3 * o + 2]);
            pf = proj * (fi + J.fpj[o]) * kf;
            pp = proj * kp;
        }
        J.cf[w] = pf;
        J.cp[w] = pp;
    }
}

// Mini-batch of sampled atoms; a batch as large as the data takes every atom once, in order.
__global__ void k_fm_draw(int32_t *envs, int nb, int64_t n_env, uint64_t seed, uint64_t step) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += gridDim.x * blockDim.x)
        envs[i] = nb == n_env ? i
                              : (int32_t)(splitmix64(seed ^ splitmix64(step * 0x100000001b3ull + (uint64_t)i)) %
                                          (uint64_t)n_env);
}

__global__ void k_fm_norm(const double *__restrict__ fref, int64_t n, double *__restrict__ out) {
    __shared__ double red[1024 / 64];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < 3 * n; i += 1024) s += fref[i] * fref[i];
    s = wave_sum_m(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < 1024 / 64; ++q) t += red[q];
        out[0] = t / (double)n;
    }
}

hipError_t launch_fm(hipStream_t st, const FmJob &J, uint64_t seed, uint64_t step, int32_t *envs) {
    hipLaunchKernelGGL(k_fm_draw, dim3((J.nb + 255) / 256), dim3(256), 0, st, envs, J.nb, J.n_env, seed, step);
    hipLaunchKernelGGL(k_fm, dim3(J.nb), dim3(64), 0, st, J);
    return hipGetLastError();
}

hipError_t launch_fm_norm(hipStream_t st, const double *fref, int64_t n, double *out) {
    hipLaunchKernelGGL(k_fm_norm, dim3(1), dim3(1024), 0, st, fref, n, out);
    return hipGetLastError();
}

// Sum of nb doubles (fixed order) into out[slot].
__global__ void k_sum_into(const double *__restrict__ a, int n, double *__restrict__ out, int slot) {
    __shared__ double red[256 / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += a[i];
    s = wave_sum_m(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[slot] = red[0] + red[1] + red[2] + red[3];
}

hipError_t launch_sum_into(hipStream_t st, const double *a, int n, double *out, int slot) {
    hipLaunchKernelGGL(k_sum_into, dim3(1), dim3(256), 0, st, a, n, out, slot);
    return hipGetLastError();
}

}  // namespace misa

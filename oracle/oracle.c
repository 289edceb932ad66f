/*
 * oracle.c -- plain, slow, obviously correct FP64 CPU oracle for the EAM
 * lattice molecular-dynamics hot path of MISA-MD (Chu, Li et al.,
 * "MD Simulation of Hundred-Billion-Metal-Atom Cascade Collision on Sunway
 * Taihulight").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the GPU library.
 *
 * What it computes, and where the paper defines it:
 *   - EAM energy  E_i = F(sum_{j!=i} f(r_ij)) + 1/2 sum_{j!=i} phi(r_ij)
 *     (Sec. 2.2, Eq. eam_base; single species, so rho_beta = f).
 *   - EAM pair force (Sec. 2.2, Eq. eam_force_ij) and the five-step procedure
 *     listed under it: rho_i, F'(rho_i), phi', f', then F_i summed over all
 *     neighbours j within the cut-off.
 *   - Potential functions from equidistant tables interpolated per segment by
 *     a cubic S_k(x) with derivative S_k'(x) (Sec. 4.1).  The paper does not
 *     fix how the segment coefficients come from the samples; this oracle
 *     takes the local reading: cubic Hermite segments whose node slopes are
 *     fourth-order central differences of the samples (one-sided / second-order
 *     at the two nodes nearest each end), linear extrapolation beyond the last
 *     node.
 *   - The MD time loop of Sec. 2.1 (Fig. 1), read as kick-drift-kick velocity
 *     Verlet, with the adaptive step dt = min(dt_max, dx_max / max_i |v_i|)
 *     evaluated at the start of each step (the paper names adaptive time steps
 *     as a feature of MISA-MD without giving the rule).
 *   - The learned form: a small SiLU network per potential function in place
 *     of its table inside the network's input range, the table outside it
 *     (an extension beyond the paper, whose functions always come from tables).
 *   - Lattice ids of BCC sites (Sec. 3, Hash Initialization: the worked 2-D
 *     example and the 3-D index equation), the neighbour offset index
 *     (Sec. 3, Neighbor Offset Index initialization), the nearest-site hash
 *     (Sec. 3: the hash maps an atom to its nearest lattice site) and the
 *     hash update of Algorithm 2 (atoms leave the array when they drift off
 *     their site; clash atoms return to empty sites).
 *
 * Readings taken where the paper is silent (all restated in the design notes):
 *   - cut-off test r^2 < rc^2 (strict); minimum image on a periodic box;
 *   - F'(0) := 0 analytically for an atom with no neighbours;
 *   - an atom stays in its lattice slot only while |x - site| <= delta, so a
 *     neighbour stencil of radius rc + 2 delta is exact; ties for one empty
 *     slot go to the lowest atom id;
 *   - the nearest site is chosen between the per-axis-rounded corner site and
 *     the per-axis floor + 1/2 body-centre site, the corner winning exact ties.
 *
 * Build:  gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared
 *              -o liboracle.so oracle.c -lm
 * (-ffp-contract=off keeps every product rounded on its own, so integer
 *  decisions taken from floating point are reproducible.)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* 1 eV/(Angstrom amu) in Angstrom/fs^2, from e = 1.602176634e-19 C (exact SI)
 * and 1 amu = 1.66053906660e-27 kg (CODATA 2018). */
#define ORC_ACC ((1.602176634e-19 / 1.66053906660e-27) * 1e-10)

enum { ORC_ANALYTIC = 0, ORC_ANALYTIC_SF = 1, ORC_TABLE = 2, ORC_MLP = 3 };

/* Width of the hidden layers of the surrogate networks. */
#define ORC_MLP_H 32

/* A surrogate network for one potential function (the learned form): inputs in
 * [x_lo, x_hi] map to t = (x - c) s with c = (x_lo + x_hi) / 2, s = 2 / (x_hi - x_lo);
 * two SiLU layers of ORC_MLP_H units and a linear output y give
 * g(x) = y_shift + y_scale y(t).  p holds W1[H], b1[H], W2[H][H] (row = output
 * unit), b2[H], w3[H], b3 in that order. */
typedef struct {
    double x_lo, x_hi, y_shift, y_scale;
    const double *p;
} orc_mlp;

/* One tabulated function: n samples y_k at x_k = x0 + k h, plus node slopes m
 * (in units of the sample spacing) filled by orc_spline_slopes. */
typedef struct {
    double x0, h;
    int64_t n;
    const double *y;
    const double *m;
} orc_table;

typedef struct {
    int32_t mode;       /* ORC_ANALYTIC, ORC_ANALYTIC_SF, ORC_TABLE or ORC_MLP */
    int32_t pad_;
    double rc;          /* cut-off radius */
    /* analytic form: f(r) = exp(-f_beta (r/f_re - 1));
       phi(r) = m_d [exp(-2 m_alpha (r - m_r0)) - 2 exp(-m_alpha (r - m_r0))];
       F(rho) = -emb_a sqrt(rho) */
    double f_beta, f_re, m_d, m_alpha, m_r0, emb_a;
    orc_table f, phi, emb;
    /* ORC_MLP: the networks inside their ranges, the tables above outside them */
    orc_mlp mf, mphi, memb;
} orc_potential;

/* ------------------------------------------------------------------ */
/* Spline (Sec. 4.1: per-segment cubic and its derivative)             */
/* ------------------------------------------------------------------ */

/* Node slopes in units of h: fourth-order central differences inside,
 * second-order central differences at nodes 1 and n-2, one-sided first
 * differences at the two end nodes. */
void orc_spline_slopes(const double *y, int64_t n, double *m)
{
    if (n < 5) {
        for (int64_t k = 0; k < n; ++k) m[k] = 0.0;
        return;
    }
    m[0] = y[1] - y[0];
    m[1] = (y[2] - y[0]) / 2.0;
    for (int64_t k = 2; k <= n - 3; ++k)
        m[k] = (y[k - 2] - 8.0 * y[k - 1] + 8.0 * y[k + 1] - y[k + 2]) / 12.0;
    m[n - 2] = (y[n - 1] - y[n - 3]) / 2.0;
    m[n - 1] = y[n - 1] - y[n - 2];
}

/* Value and d/dx of the interpolant at x.  Returns 1 when x lies beyond the
 * last node (linear extrapolation used), 0 otherwise. */
int orc_spline_eval(const orc_table *T, double x, double *val, double *der)
{
    double p = (x - T->x0) / T->h;
    int64_t last = T->n - 1;
    if (p > (double)last) {
        double t = p - (double)last;
        *val = T->y[last] + T->m[last] * t;
        *der = T->m[last] / T->h;
        return 1;
    }
    int64_t k = (int64_t)floor(p);
    if (k < 0) k = 0;
    if (k > T->n - 2) k = T->n - 2;
    double t = p - (double)k;
    double y0 = T->y[k], y1 = T->y[k + 1];
    double m0 = T->m[k], m1 = T->m[k + 1];
    /* cubic Hermite on [x_k, x_k+1] in the local variable t in [0, 1] */
    double c0 = y0;
    double c1 = m0;
    double c2 = 3.0 * (y1 - y0) - 2.0 * m0 - m1;
    double c3 = m0 + m1 - 2.0 * (y1 - y0);
    *val = ((c3 * t + c2) * t + c1) * t + c0;
    *der = ((3.0 * c3 * t + 2.0 * c2) * t + c1) / T->h;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Potential functions                                                  */
/* ------------------------------------------------------------------ */

static void an_f(const orc_potential *P, double r, double *v, double *d)
{
    double e = exp(-P->f_beta * (r / P->f_re - 1.0));
    *v = e;
    *d = -(P->f_beta / P->f_re) * e;
}

static void an_phi(const orc_potential *P, double r, double *v, double *d)
{
    double e1 = exp(-2.0 * P->m_alpha * (r - P->m_r0));
    double e2 = exp(-P->m_alpha * (r - P->m_r0));
    *v = P->m_d * (e1 - 2.0 * e2);
    *d = P->m_d * (-2.0 * P->m_alpha * e1 + 2.0 * P->m_alpha * e2);
}

/* Value and d/dx of a surrogate network, straight from its definition. */
void orc_mlp_eval(const orc_mlp *M, double x, double *v, double *d)
{
    const int H = ORC_MLP_H;
    const double *W1 = M->p, *b1 = W1 + H, *W2 = b1 + H, *b2 = W2 + H * H, *w3 = b2 + H;
    const double b3 = w3[H];
    const double c = 0.5 * (M->x_lo + M->x_hi), s = 2.0 / (M->x_hi - M->x_lo);
    const double t = (x - c) * s;
    double h1[ORC_MLP_H], dh1[ORC_MLP_H];   /* layer-1 outputs and their d/dt */
    for (int k = 0; k < H; ++k) {
        double z = W1[k] * t + b1[k];
        double sg = 1.0 / (1.0 + exp(-z));
        h1[k] = z * sg;
        dh1[k] = (sg + z * sg * (1.0 - sg)) * W1[k];
    }
    double y = b3, dy = 0.0;
    for (int n = 0; n < H; ++n) {
        double z = b2[n], dz = 0.0;
        for (int k = 0; k < H; ++k) {
            z += W2[n * H + k] * h1[k];
            dz += W2[n * H + k] * dh1[k];
        }
        double sg = 1.0 / (1.0 + exp(-z));
        y += w3[n] * z * sg;
        dy += w3[n] * (sg + z * sg * (1.0 - sg)) * dz;
    }
    *v = M->y_shift + M->y_scale * y;
    *d = M->y_scale * s * dy;
}

static int in_range(const orc_mlp *M, double x) { return x >= M->x_lo && x <= M->x_hi; }

/* electron density contribution f(r) and f'(r) */
void orc_pot_f(const orc_potential *P, double r, double *v, double *d)
{
    if (P->mode == ORC_MLP && in_range(&P->mf, r)) {
        orc_mlp_eval(&P->mf, r, v, d);
        return;
    }
    if (P->mode == ORC_TABLE || P->mode == ORC_MLP) {
        orc_spline_eval(&P->f, r, v, d);
        return;
    }
    an_f(P, r, v, d);
    if (P->mode == ORC_ANALYTIC_SF) {
        double vc, dc;
        an_f(P, P->rc, &vc, &dc);
        *v = *v - vc - (r - P->rc) * dc;
        *d = *d - dc;
    }
}

/* pair potential phi(r) and phi'(r) */
void orc_pot_phi(const orc_potential *P, double r, double *v, double *d)
{
    if (P->mode == ORC_MLP && in_range(&P->mphi, r)) {
        orc_mlp_eval(&P->mphi, r, v, d);
        return;
    }
    if (P->mode == ORC_TABLE || P->mode == ORC_MLP) {
        orc_spline_eval(&P->phi, r, v, d);
        return;
    }
    an_phi(P, r, v, d);
    if (P->mode == ORC_ANALYTIC_SF) {
        double vc, dc;
        an_phi(P, P->rc, &vc, &dc);
        *v = *v - vc - (r - P->rc) * dc;
        *d = *d - dc;
    }
}

/* embedding energy F(rho) and F'(rho); returns 1 if rho was beyond the table */
int orc_pot_emb(const orc_potential *P, double rho, double *v, double *d)
{
    if (P->mode == ORC_MLP && in_range(&P->memb, rho)) {
        orc_mlp_eval(&P->memb, rho, v, d);
        return 0;
    }
    if (P->mode == ORC_TABLE || P->mode == ORC_MLP)
        return orc_spline_eval(&P->emb, rho, v, d);
    if (rho <= 0.0) {
        *v = 0.0;
        *d = 0.0;
        return 0;
    }
    double s = sqrt(rho);
    *v = -P->emb_a * s;
    *d = -P->emb_a / (2.0 * s);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Brute-force O(N^2) EAM (Sec. 2.2, Eq. eam_base and Eq. eam_force_ij) */
/* ------------------------------------------------------------------ */

static inline void min_image(double d[3], const double L[3])
{
    for (int a = 0; a < 3; ++a) d[a] -= L[a] * nearbyint(d[a] / L[a]);
}

/*
 * rho[i]  = sum_{j != i, r_ij < rc} f(r_ij)                     (step 1)
 * fp[i]   = F'(rho_i)                                           (step 2)
 * F[i]    = sum_{j != i} s_ij (x_j - x_i) / r_ij,
 *           s_ij = (F'_i + F'_j) f'(r_ij) + phi'(r_ij)          (steps 3-5)
 * energies[0] = sum_i F(rho_i); energies[1] = 1/2 sum_i sum_{j!=i} phi(r_ij)
 * npairs[i] = number of j with r_ij < rc (optional)
 * Any output pointer may be NULL except rho and fp (scratch if not wanted).
 */
int orc_eam_brute(const orc_potential *P, const double *x, int64_t N, const double L[3],
                  double *rho, double *fp, double *F, double *energies, int64_t *npairs)
{
    const double rc2 = P->rc * P->rc;
    double *emb_e = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *pair_e = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    if (!emb_e || !pair_e) {
        free(emb_e);
        free(pair_e);
        return -1;
    }
    int64_t extrap = 0;

#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; ++i) {
        double acc = 0.0;
        int64_t cnt = 0;
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
            min_image(d, L);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rc2) {
                double fv, fd;
                orc_pot_f(P, sqrt(r2), &fv, &fd);
                acc += fv;
                ++cnt;
            }
        }
        rho[i] = acc;
        if (npairs) npairs[i] = cnt;
    }

    for (int64_t i = 0; i < N; ++i) {
        double v, d;
        extrap += orc_pot_emb(P, rho[i], &v, &d);
        emb_e[i] = v;
        fp[i] = d;
    }

#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < N; ++i) {
        double fx = 0.0, fy = 0.0, fz = 0.0, ep = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
            min_image(d, L);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rc2) {
                double r = sqrt(r2);
                double fv, fd, pv, pd;
                orc_pot_f(P, r, &fv, &fd);
                orc_pot_phi(P, r, &pv, &pd);
                double s = (fp[i] + fp[j]) * fd + pd;
                fx += s * d[0] / r;
                fy += s * d[1] / r;
                fz += s * d[2] / r;
                ep += 0.5 * pv;
            }
        }
        if (F) {
            F[3 * i] = fx;
            F[3 * i + 1] = fy;
            F[3 * i + 2] = fz;
        }
        pair_e[i] = ep;
    }

    if (energies) {
        double ee = 0.0, pe = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            ee += emb_e[i];
            pe += pair_e[i];
        }
        energies[0] = ee;
        energies[1] = pe;
    }
    free(emb_e);
    free(pair_e);
    return (int)(extrap > 0 ? 1 : 0);
}

/* ------------------------------------------------------------------ */
/* Exact cell-binned variant: same pair set, O(N) work                  */
/* ------------------------------------------------------------------ */

typedef struct {
    int nc[3];
    double cs[3];
    int64_t *start; /* ncell + 1 */
    int64_t *atoms; /* N, grouped by cell */
} cell_list;

static int64_t cell_of(const double *xi, const double L[3], const cell_list *C, int c3[3])
{
    for (int a = 0; a < 3; ++a) {
        double w = xi[a] - L[a] * floor(xi[a] / L[a]);
        int c = (int)(w / C->cs[a]);
        if (c >= C->nc[a]) c = C->nc[a] - 1;
        if (c < 0) c = 0;
        c3[a] = c;
    }
    return ((int64_t)c3[2] * C->nc[1] + c3[1]) * C->nc[0] + c3[0];
}

static int build_cells(const double *x, int64_t N, const double L[3], double rc, cell_list *C)
{
    for (int a = 0; a < 3; ++a) {
        int n = (int)floor(L[a] / rc);
        if (n < 1) n = 1;
        C->nc[a] = n;
        C->cs[a] = L[a] / n;
    }
    int64_t ncell = (int64_t)C->nc[0] * C->nc[1] * C->nc[2];
    C->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    C->atoms = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    if (!C->start || !C->atoms || !cid) {
        free(C->start);
        free(C->atoms);
        free(cid);
        return -1;
    }
    for (int64_t i = 0; i < N; ++i) {
        int c3[3];
        cid[i] = cell_of(x + 3 * i, L, C, c3);
        C->start[cid[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) C->start[c + 1] += C->start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ncell > 0 ? ncell : 1));
    memcpy(fill, C->start, sizeof(int64_t) * (size_t)ncell);
    for (int64_t i = 0; i < N; ++i) C->atoms[fill[cid[i]]++] = i; /* ascending atom id within a cell */
    free(fill);
    free(cid);
    return 0;
}

static void free_cells(cell_list *C)
{
    free(C->start);
    free(C->atoms);
}

/* distinct neighbour cell indices along one axis (1, 2 or 3 of them) */
static int axis_neighbours(int c, int n, int out[3])
{
    if (n == 1) {
        out[0] = 0;
        return 1;
    }
    if (n == 2) {
        out[0] = 0;
        out[1] = 1;
        return 2;
    }
    out[0] = (c + n - 1) % n;
    out[1] = c;
    out[2] = (c + 1) % n;
    return 3;
}

/* Neighbours j != i of atom i with r_ij < rc, found through the cell list:
 * ids, minimum-image separations x_j - x_i and squared distances. */
typedef struct {
    int64_t n, cap;
    int64_t *j;
    double *d;  /* 3 per neighbour */
    double *r2;
} nbr_buf;

static void nbr_push(nbr_buf *b, int64_t j, const double d[3], double r2)
{
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 256;
        b->j = (int64_t *)realloc(b->j, sizeof(int64_t) * (size_t)b->cap);
        b->d = (double *)realloc(b->d, sizeof(double) * 3 * (size_t)b->cap);
        b->r2 = (double *)realloc(b->r2, sizeof(double) * (size_t)b->cap);
    }
    b->j[b->n] = j;
    b->d[3 * b->n] = d[0];
    b->d[3 * b->n + 1] = d[1];
    b->d[3 * b->n + 2] = d[2];
    b->r2[b->n] = r2;
    b->n++;
}

static void nbr_free(nbr_buf *b)
{
    free(b->j);
    free(b->d);
    free(b->r2);
}

static void cell_neighbours(const cell_list *C, const double *x, const double L[3], int64_t i, double rc2,
                            nbr_buf *out)
{
    int c3[3], nxs[3], nys[3], nzs[3];
    out->n = 0;
    cell_of(x + 3 * i, L, C, c3);
    int kx = axis_neighbours(c3[0], C->nc[0], nxs);
    int ky = axis_neighbours(c3[1], C->nc[1], nys);
    int kz = axis_neighbours(c3[2], C->nc[2], nzs);
    for (int az = 0; az < kz; ++az)
        for (int ay = 0; ay < ky; ++ay)
            for (int ax = 0; ax < kx; ++ax) {
                int64_t cc = ((int64_t)nzs[az] * C->nc[1] + nys[ay]) * C->nc[0] + nxs[ax];
                for (int64_t q = C->start[cc]; q < C->start[cc + 1]; ++q) {
                    int64_t j = C->atoms[q];
                    if (j == i) continue;
                    double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
                    min_image(d, L);
                    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    if (r2 < rc2) nbr_push(out, j, d, r2);
                }
            }
}

/* Same outputs as orc_eam_brute; the pair set is identical because every
 * cell is at least rc wide and neighbour cells are deduplicated. */
int orc_eam_cells(const orc_potential *P, const double *x, int64_t N, const double L[3],
                  double *rho, double *fp, double *F, double *energies, int64_t *npairs)
{
    const double rc2 = P->rc * P->rc;
    cell_list C;
    if (build_cells(x, N, L, P->rc, &C)) return -1;
    double *emb_e = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *pair_e = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    int64_t extrap = 0;

#pragma omp parallel
    {
        nbr_buf nb = {0, 0, NULL, NULL, NULL};
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < N; ++i) {
            cell_neighbours(&C, x, L, i, rc2, &nb);
            double acc = 0.0;
            for (int64_t q = 0; q < nb.n; ++q) {
                double fv, fd;
                orc_pot_f(P, sqrt(nb.r2[q]), &fv, &fd);
                acc += fv;
            }
            rho[i] = acc;
            if (npairs) npairs[i] = nb.n;
        }
        nbr_free(&nb);
    }
    for (int64_t i = 0; i < N; ++i) {
        double v, d;
        extrap += orc_pot_emb(P, rho[i], &v, &d);
        emb_e[i] = v;
        fp[i] = d;
    }
#pragma omp parallel
    {
        nbr_buf nb = {0, 0, NULL, NULL, NULL};
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < N; ++i) {
            cell_neighbours(&C, x, L, i, rc2, &nb);
            double fx = 0.0, fy = 0.0, fz = 0.0, ep = 0.0;
            for (int64_t q = 0; q < nb.n; ++q) {
                int64_t j = nb.j[q];
                const double *d = nb.d + 3 * q;
                double r = sqrt(nb.r2[q]);
                double fv, fd, pv, pd;
                orc_pot_f(P, r, &fv, &fd);
                orc_pot_phi(P, r, &pv, &pd);
                double s = (fp[i] + fp[j]) * fd + pd;
                fx += s * d[0] / r;
                fy += s * d[1] / r;
                fz += s * d[2] / r;
                ep += 0.5 * pv;
            }
            if (F) {
                F[3 * i] = fx;
                F[3 * i + 1] = fy;
                F[3 * i + 2] = fz;
            }
            pair_e[i] = ep;
        }
        nbr_free(&nb);
    }
    if (energies) {
        double ee = 0.0, pe = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            ee += emb_e[i];
            pe += pair_e[i];
        }
        energies[0] = ee;
        energies[1] = pe;
    }
    free(emb_e);
    free(pair_e);
    free_cells(&C);
    return (int)(extrap > 0 ? 1 : 0);
}

/* Neighbour ids of atom i (r_ij < rc), ascending, via brute force (cells = 0)
 * or the cell list (cells = 1).  Returns the count (written up to cap). */
int64_t orc_neighbours(const double *x, int64_t N, const double L[3], double rc, int64_t i,
                       int cells, int64_t *out, int64_t cap)
{
    const double rc2 = rc * rc;
    int64_t cnt = 0;
    if (!cells) {
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) continue;
            double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
            min_image(d, L);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rc2) {
                if (cnt < cap) out[cnt] = j;
                ++cnt;
            }
        }
        return cnt;
    }
    cell_list C;
    if (build_cells(x, N, L, rc, &C)) return -1;
    nbr_buf nb = {0, 0, NULL, NULL, NULL};
    cell_neighbours(&C, x, L, i, rc2, &nb);
    for (int64_t q = 0; q < nb.n; ++q) {
        if (cnt < cap) out[cnt] = nb.j[q];
        ++cnt;
    }
    nbr_free(&nb);
    free_cells(&C);
    /* ascending order (insertion sort of the written part) */
    int64_t w = cnt < cap ? cnt : cap;
    for (int64_t a = 1; a < w; ++a) {
        int64_t key = out[a], b = a - 1;
        while (b >= 0 && out[b] > key) {
            out[b + 1] = out[b];
            --b;
        }
        out[b + 1] = key;
    }
    return cnt;
}

/*
 * Forces, densities and embedding derivatives for a sample of M atoms of a
 * large system, without evaluating the whole system: rho is computed for the
 * sample and for every neighbour of a sampled atom (their F' enters the
 * sampled forces), then F for the sampled atoms.  Exact (cell-binned pair set).
 * npairs_s (optional) receives the number of neighbours within rc of each
 * sampled atom.
 */
int orc_eam_sampled(const orc_potential *P, const double *x, int64_t N, const double L[3],
                    const int64_t *sample, int64_t M, double *rho_s, double *fp_s, double *F_s,
                    int64_t *npairs_s)
{
    const double rc2 = P->rc * P->rc;
    cell_list C;
    if (build_cells(x, N, L, P->rc, &C)) return -1;
    /* slot index of each needed atom, -1 if not needed */
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    int64_t *need = NULL;
    int64_t nneed = 0, cap = M * 80 + 16;
    need = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    if (!slot || !need) {
        free(slot);
        free(need);
        free_cells(&C);
        return -1;
    }
    for (int64_t i = 0; i < N; ++i) slot[i] = -1;
    nbr_buf nb = {0, 0, NULL, NULL, NULL};
    for (int64_t s = 0; s < M; ++s) {
        int64_t i = sample[s];
        cell_neighbours(&C, x, L, i, rc2, &nb);
        for (int64_t q = -1; q < nb.n; ++q) {
            int64_t j = q < 0 ? i : nb.j[q];
            if (slot[j] >= 0) continue;
            if (nneed == cap) {
                cap *= 2;
                need = (int64_t *)realloc(need, sizeof(int64_t) * (size_t)cap);
            }
            slot[j] = nneed;
            need[nneed++] = j;
        }
    }
    nbr_free(&nb);
    double *rho_n = (double *)malloc(sizeof(double) * (size_t)(nneed > 0 ? nneed : 1));
    double *fp_n = (double *)malloc(sizeof(double) * (size_t)(nneed > 0 ? nneed : 1));
#pragma omp parallel
    {
        nbr_buf b = {0, 0, NULL, NULL, NULL};
#pragma omp for schedule(dynamic, 64)
        for (int64_t q = 0; q < nneed; ++q) {
            cell_neighbours(&C, x, L, need[q], rc2, &b);
            double acc = 0.0;
            for (int64_t k = 0; k < b.n; ++k) {
                double fv, fd;
                orc_pot_f(P, sqrt(b.r2[k]), &fv, &fd);
                acc += fv;
            }
            rho_n[q] = acc;
            double v, d;
            orc_pot_emb(P, acc, &v, &d);
            fp_n[q] = d;
        }
#pragma omp for schedule(dynamic, 16)
        for (int64_t s = 0; s < M; ++s) {
            int64_t i = sample[s];
            cell_neighbours(&C, x, L, i, rc2, &b);
            double fpi = fp_n[slot[i]];
            double fx = 0.0, fy = 0.0, fz = 0.0;
            for (int64_t k = 0; k < b.n; ++k) {
                int64_t j = b.j[k];
                const double *d = b.d + 3 * k;
                double r = sqrt(b.r2[k]);
                double fv, fd, pv, pd;
                orc_pot_f(P, r, &fv, &fd);
                orc_pot_phi(P, r, &pv, &pd);
                double sij = (fpi + fp_n[slot[j]]) * fd + pd;
                fx += sij * d[0] / r;
                fy += sij * d[1] / r;
                fz += sij * d[2] / r;
            }
            rho_s[s] = rho_n[slot[i]];
            fp_s[s] = fpi;
            if (npairs_s) npairs_s[s] = b.n;
            F_s[3 * s] = fx;
            F_s[3 * s + 1] = fy;
            F_s[3 * s + 2] = fz;
        }
        nbr_free(&b);
    }
    free(rho_n);
    free(fp_n);
    free(slot);
    free(need);
    free_cells(&C);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Time integration (Sec. 2.1, Fig. 1, read as kick-drift-kick Verlet)  */
/* ------------------------------------------------------------------ */

double orc_kinetic(const double *v, int64_t N, double mass)
{
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2];
    return 0.5 * mass * s / ORC_ACC;
}

double orc_acc_unit(void) { return ORC_ACC; }

/*
 * nsteps of velocity Verlet on (x, v), in place.  F (N*3) holds the force at
 * the current x on entry when have_force != 0, and on exit always.
 * Each step:  dt = dx_max > 0 ? min(dt_max, dx_max / max|v|) : dt_max
 *             v += (dt/2) C F / m;  x += dt v;  F = F(x);  v += (dt/2) C F / m.
 * log (optional, nsteps * 5): [dt, E_kin, E_emb, E_pair, max|v| at step start].
 * cells != 0 uses the exact cell-binned force evaluation.
 */
int orc_run(const orc_potential *P, double *x, double *v, double *F, int64_t N, const double L[3],
            double mass, int64_t nsteps, double dt_max, double dx_max, int cells, int have_force,
            double *log)
{
    double *rho = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *fp = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double en[2] = {0.0, 0.0};
    if (!rho || !fp) {
        free(rho);
        free(fp);
        return -1;
    }
    if (!have_force) {
        if (cells)
            orc_eam_cells(P, x, N, L, rho, fp, F, en, NULL);
        else
            orc_eam_brute(P, x, N, L, rho, fp, F, en, NULL);
    }
    const double kf = ORC_ACC / mass;
    for (int64_t s = 0; s < nsteps; ++s) {
        double vmax2 = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double q = v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2];
            if (q > vmax2) vmax2 = q;
        }
        double vmax = sqrt(vmax2);
        double dt = dt_max;
        if (dx_max > 0.0 && vmax > 0.0 && dx_max / vmax < dt_max) dt = dx_max / vmax;
        double hk = 0.5 * dt * kf;
        for (int64_t i = 0; i < 3 * N; ++i) {
            v[i] += hk * F[i];
            x[i] += dt * v[i];
        }
        if (cells)
            orc_eam_cells(P, x, N, L, rho, fp, F, en, NULL);
        else
            orc_eam_brute(P, x, N, L, rho, fp, F, en, NULL);
        for (int64_t i = 0; i < 3 * N; ++i) v[i] += hk * F[i];
        if (log) {
            log[5 * s + 0] = dt;
            log[5 * s + 1] = orc_kinetic(v, N, mass);
            log[5 * s + 2] = en[0];
            log[5 * s + 3] = en[1];
            log[5 * s + 4] = vmax;
        }
    }
    free(rho);
    free(fp);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Lattice list, offsets and hash (Sec. 3, Algorithms 1 and 2)          */
/* ------------------------------------------------------------------ */

/* lattice id of site (X, Y, Z): X runs over 2 box_x half-cell columns,
 * odd X are body centres (Sec. 3, Hash Initialization). */
int64_t orc_lattice_id(int64_t box_x, int64_t box_y, int64_t X, int64_t Y, int64_t Z)
{
    return 2 * box_x * box_y * Z + 2 * box_x * Y + X;
}

void orc_lattice_coords(int64_t box_x, int64_t box_y, int64_t id, int64_t *X, int64_t *Y, int64_t *Z)
{
    int64_t row = 2 * box_x;
    *X = id % row;
    *Y = (id / row) % box_y;
    *Z = id / (row * box_y);
}

/* Cartesian position of site (X, Y, Z) for lattice constant a. */
void orc_site_position(double a, int64_t X, int64_t Y, int64_t Z, double pos[3])
{
    double half = (double)(X & 1) * 0.5;
    pos[0] = (double)X * 0.5 * a;
    pos[1] = ((double)Y + half) * a;
    pos[2] = ((double)Z + half) * a;
}

/* Neighbor Offset Index: every (dX, dY, dZ) != 0 whose site lies strictly
 * closer than R to a site of the given parity (X even = 0, odd = 1), by
 * enumeration over a cube.  Order: dZ, then dY, then dX ascending.
 * Returns the count (written up to cap triples). */
int64_t orc_stencil(double a, double R, int parity, int64_t *out, int64_t cap)
{
    int64_t w = (int64_t)ceil(R / a) + 1;
    int64_t X0 = parity ? 1 : 0;
    double p0[3];
    orc_site_position(a, X0 + 4 * w, w, w, p0); /* shift so coordinates stay non-negative */
    int64_t cnt = 0;
    for (int64_t dz = -w; dz <= w; ++dz)
        for (int64_t dy = -w; dy <= w; ++dy)
            for (int64_t dx = -2 * w; dx <= 2 * w; ++dx) {
                if (dx == 0 && dy == 0 && dz == 0) continue;
                double p1[3];
                orc_site_position(a, X0 + 4 * w + dx, w + dy, w + dz, p1);
                double d0 = p1[0] - p0[0], d1 = p1[1] - p0[1], d2 = p1[2] - p0[2];
                if (d0 * d0 + d1 * d1 + d2 * d2 < R * R) {
                    if (cnt < cap) {
                        out[3 * cnt] = dx;
                        out[3 * cnt + 1] = dy;
                        out[3 * cnt + 2] = dz;
                    }
                    ++cnt;
                }
            }
    return cnt;
}

/* Nearest site by exhaustive search over every site of the periodic box
 * (minimum-image distance).  Returns the lattice id; *dist2 = squared distance. */
int64_t orc_nearest_site_brute(int64_t nx, int64_t ny, int64_t nz, double a, const double x[3], double *dist2)
{
    const double L[3] = {nx * a, ny * a, nz * a};
    int64_t best = -1;
    double bd = INFINITY;
    for (int64_t Z = 0; Z < nz; ++Z)
        for (int64_t Y = 0; Y < ny; ++Y)
            for (int64_t X = 0; X < 2 * nx; ++X) {
                double p[3];
                orc_site_position(a, X, Y, Z, p);
                double d[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
                min_image(d, L);
                double q = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (q < bd) {
                    bd = q;
                    best = orc_lattice_id(nx, ny, X, Y, Z);
                }
            }
    if (dist2) *dist2 = bd;
    return best;
}

/*
 * The hash: nearest site by rule.  The position is wrapped into the box;
 * the nearest corner site rounds each coordinate (in units of a) to the
 * nearest integer (ties to even), the nearest body-centre site takes
 * floor + 1/2; the closer of the two wins, the corner on an exact tie.
 * u receives x - site (Cartesian), *u2 = |u|^2 (summed x, y, z in order).
 */
int64_t orc_hash(int64_t nx, int64_t ny, int64_t nz, double a, const double x[3], double u[3], double *u2)
{
    const int64_t n[3] = {nx, ny, nz};
    const double inv_a = 1.0 / a;
    double xw[3], uc[3], ub[3];
    int64_t ic[3], ib[3];
    for (int k = 0; k < 3; ++k) {
        double Lk = (double)n[k] * a;
        xw[k] = x[k] - Lk * floor(x[k] / Lk);
        double q = xw[k] * inv_a;
        double c = nearbyint(q);
        double b = floor(q) + 0.5;
        uc[k] = xw[k] - c * a;
        ub[k] = xw[k] - b * a;
        ic[k] = (int64_t)c;
        ib[k] = (int64_t)floor(q);
    }
    double dc = uc[0] * uc[0] + uc[1] * uc[1] + uc[2] * uc[2];
    double db = ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2];
    int centre = db < dc;
    int64_t c3[3];
    for (int k = 0; k < 3; ++k) {
        int64_t c = centre ? ib[k] : ic[k];
        c %= n[k];
        if (c < 0) c += n[k];
        c3[k] = c;
        u[k] = centre ? ub[k] : uc[k];
    }
    *u2 = centre ? db : dc;
    return orc_lattice_id(nx, ny, 2 * c3[0] + centre, c3[1], c3[2]);
}

/*
 * Wigner-Seitz defect count: every atom belongs to the cell of its nearest
 * lattice site (the hash rule below, which is the nearest site); a site whose
 * cell holds no atom is a vacancy, every atom beyond the first in a cell an
 * interstitial.  occ (may be NULL) receives the per-site atom count, indexed
 * by lattice id.  out[0] = vacancies, out[1] = interstitials.  The paper names
 * direct defect analysis as a feature (Sec. 1) and counts defects of a cascade
 * (Sec. 5.1) without fixing the method; this is the textbook one.
 */
int orc_wigner_seitz(int64_t nx, int64_t ny, int64_t nz, double a, const double *x, int64_t n, int64_t out[2],
                     int32_t *occ)
{
    const int64_t ns = 2 * nx * ny * nz;
    int32_t *o = occ ? occ : (int32_t *)malloc(sizeof(int32_t) * (size_t)ns);
    if (!o) return -1;
    for (int64_t s = 0; s < ns; ++s) o[s] = 0;
    for (int64_t i = 0; i < n; ++i) {
        double u[3], u2;
        o[orc_hash(nx, ny, nz, a, x + 3 * i, u, &u2)] += 1;
    }
    int64_t vac = 0, inter = 0;
    for (int64_t s = 0; s < ns; ++s) {
        if (o[s] == 0) ++vac;
        if (o[s] > 1) inter += o[s] - 1;
    }
    out[0] = vac;
    out[1] = inter;
    if (!occ) free(o);
    return 0;
}


/*
 * Fresh placement of N atoms into the lattice list: an atom is a slot
 * candidate when |x - nearest site| <= delta; among candidates of one site
 * the lowest atom id takes the slot.  slot[i] = lattice id or -1 (clash /
 * run-away atom).
 */
void orc_place(int64_t nx, int64_t ny, int64_t nz, double a, double delta, const double *x, int64_t N,
               int64_t *slot)
{
    int64_t nsites = 2 * nx * ny * nz;
    unsigned char *taken = (unsigned char *)calloc((size_t)nsites, 1);
    const double d2 = delta * delta;
    for (int64_t i = 0; i < N; ++i) { /* ascending id: first claimant = lowest id */
        double u[3], u2;
        int64_t s = orc_hash(nx, ny, nz, a, x + 3 * i, u, &u2);
        if (u2 <= d2 && !taken[s]) {
            taken[s] = 1;
            slot[i] = s;
        } else {
            slot[i] = -1;
        }
    }
    free(taken);
}

/*
 * Hash update (Algorithm 2 with the slot tolerance delta): first every atom in
 * a slot whose displacement from that slot's site exceeds delta leaves it;
 * then every atom outside the array, in ascending id, takes the slot of its
 * nearest site if that slot is empty and it lies within delta of the site.
 */
void orc_rehash(int64_t nx, int64_t ny, int64_t nz, double a, double delta, const double *x, int64_t N,
                int64_t *slot)
{
    int64_t nsites = 2 * nx * ny * nz;
    unsigned char *taken = (unsigned char *)calloc((size_t)nsites, 1);
    const double d2 = delta * delta;
    const double L[3] = {nx * a, ny * a, nz * a};
    for (int64_t i = 0; i < N; ++i) {
        if (slot[i] < 0) continue;
        int64_t X, Y, Z;
        orc_lattice_coords(nx, ny, slot[i], &X, &Y, &Z);
        double p[3];
        orc_site_position(a, X, Y, Z, p);
        double d[3] = {x[3 * i] - p[0], x[3 * i + 1] - p[1], x[3 * i + 2] - p[2]};
        min_image(d, L);
        if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] > d2)
            slot[i] = -1;
        else
            taken[slot[i]] = 1;
    }
    for (int64_t i = 0; i < N; ++i) {
        if (slot[i] >= 0) continue;
        double u[3], u2;
        int64_t s = orc_hash(nx, ny, nz, a, x + 3 * i, u, &u2);
        if (u2 <= d2 && !taken[s]) {
            taken[s] = 1;
            slot[i] = s;
        }
    }
    free(taken);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

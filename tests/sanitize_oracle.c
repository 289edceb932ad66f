/* Exercises every entry point of oracle.c on small inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py).
 * It checks no numbers (the pins do that); a sanitizer report or a non-zero exit
 * fails the test. */
#include "../oracle/oracle.c"

#include <stdio.h>

static double lcg(uint64_t *s) {
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) / 9007199254740992.0;
}

int main(void) {
    uint64_t seed = 12345;
    const double a = 2.855, rc = 5.0, delta = 0.6;
    const int64_t n = 5, N = 2 * n * n * n;
    const double L[3] = {n * a, n * a, n * a};
    double *x = malloc(sizeof(double) * 3 * (N + 1)), *v = malloc(sizeof(double) * 3 * (N + 1));
    double *F = malloc(sizeof(double) * 3 * (N + 1)), *rho = malloc(sizeof(double) * (N + 1));
    double *fp = malloc(sizeof(double) * (N + 1));
    int64_t *np_ = malloc(sizeof(int64_t) * (N + 1)), *slot = malloc(sizeof(int64_t) * (N + 1));
    for (int64_t i = 0; i < N; ++i) {
        const int64_t p = i / (n * n * n), c = i % (n * n * n);
        const double site[3] = {(c % n + 0.5 * p) * a, (c / n % n + 0.5 * p) * a, (c / (n * n) + 0.5 * p) * a};
        for (int k = 0; k < 3; ++k) {
            x[3 * i + k] = site[k] + 0.1 * (lcg(&seed) - 0.5);
            v[3 * i + k] = 0.01 * (lcg(&seed) - 0.5);
        }
    }
    /* an interstitial */
    x[3 * N] = 2.5 * a + 0.03;
    x[3 * N + 1] = 2.0 * a;
    x[3 * N + 2] = 1.0 * a;
    v[3 * N] = v[3 * N + 1] = v[3 * N + 2] = 0.0;

    /* tables sampled from the analytic form */
    enum { NT = 400 };
    static double fy[NT], py[NT], ey[NT], fm[NT], pm[NT], em[NT];
    orc_potential P;
    memset(&P, 0, sizeof(P));
    P.mode = ORC_ANALYTIC;
    P.rc = rc;
    P.f_beta = 3.0;
    P.f_re = 2.47;
    P.m_d = 0.4;
    P.m_alpha = 1.6;
    P.m_r0 = 2.5;
    P.emb_a = 1.0;
    const double hr = rc / (NT - 1), he = 61.8 / (NT - 1);
    for (int k = 0; k < NT; ++k) {
        double d;
        orc_pot_f(&P, k * hr, &fy[k], &d);
        orc_pot_phi(&P, k * hr, &py[k], &d);
        orc_pot_emb(&P, k * he, &ey[k], &d);
    }
    orc_spline_slopes(fy, NT, fm);
    orc_spline_slopes(py, NT, pm);
    orc_spline_slopes(ey, NT, em);
    orc_potential T = P;
    T.mode = ORC_TABLE;
    T.f = (orc_table){0.0, hr, NT, fy, fm};
    T.phi = (orc_table){0.0, hr, NT, py, pm};
    T.emb = (orc_table){0.0, he, NT, ey, em};
    /* a small network for the learned mode */
    static double wp[ORC_MLP_H * (ORC_MLP_H + 4) + 1];
    for (size_t k = 0; k < sizeof(wp) / sizeof(wp[0]); ++k) wp[k] = 0.2 * (lcg(&seed) - 0.5);
    orc_potential Mp = T;
    Mp.mode = ORC_MLP;
    Mp.mf = (orc_mlp){1.6, rc, 0.0, 1.0, wp};
    Mp.mphi = (orc_mlp){1.6, rc, 0.0, 1.0, wp};
    Mp.memb = (orc_mlp){4.0, 36.0, 0.0, 1.0, wp};

    double en[2], val, der;
    int rc_ = 0;
    const orc_potential *pots[3] = {&P, &T, &Mp};
    for (int q = 0; q < 3; ++q) {
        rc_ |= orc_eam_brute(pots[q], x, N + 1, L, rho, fp, F, en, np_) < 0;
        rc_ |= orc_eam_cells(pots[q], x, N + 1, L, rho, fp, F, en, np_) < 0;
    }
    const int64_t sample[4] = {0, 7, N - 1, N};
    rc_ |= orc_eam_sampled(&T, x, N + 1, L, sample, 4, rho, fp, F, np_) < 0;
    int64_t nb[256];
    rc_ |= orc_neighbours(x, N + 1, L, rc, 3, 1, nb, 256) < 0;
    rc_ |= orc_neighbours(x, N + 1, L, rc, 3, 0, nb, 256) < 0;
    orc_spline_eval(&T.f, 7.5, &val, &der); /* beyond the last node */
    orc_spline_eval(&T.f, -0.1, &val, &der);
    double log_[5 * 4];
    rc_ |= orc_run(&T, x, v, F, N + 1, L, 55.845, 4, 1.0, 0.05, 1, 0, log_) < 0;
    (void)orc_kinetic(v, N + 1, 55.845);
    int64_t X, Y, Z;
    orc_lattice_coords(2 * n, n, orc_lattice_id(2 * n, n, 3, 4, 1), &X, &Y, &Z);
    double pos[3], u[3], u2, d2;
    orc_site_position(a, X, Y, Z, pos);
    int64_t st[3 * 128];
    rc_ |= orc_stencil(a, rc + 2 * delta, 0, st, 128) < 0;
    rc_ |= orc_stencil(a, rc + 2 * delta, 1, st, 128) < 0;
    for (int64_t i = 0; i <= N; ++i) {
        (void)orc_nearest_site_brute(n, n, n, a, &x[3 * i], &d2);
        (void)orc_hash(n, n, n, a, &x[3 * i], u, &u2);
    }
    int64_t ws[2];
    rc_ |= orc_wigner_seitz(n, n, n, a, x, N + 1, ws, NULL) < 0;
    orc_place(n, n, n, a, delta, x, N + 1, slot);
    orc_rehash(n, n, n, a, delta, x, N + 1, slot);
    printf("sanitized oracle run: %s\n", rc_ ? "allocation failure" : "ok");
    free(x);
    free(v);
    free(F);
    free(rho);
    free(fp);
    free(np_);
    free(slot);
    return rc_;
}

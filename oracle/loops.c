/*
 * Loop form of the 3D SBP-SAT FDTD leapfrog step, one block, fp64.
 *
 * TEST INFRASTRUCTURE ONLY (the oracle): used by the tests, by the
 * smoke check and by the CPU-baseline leg of the benchmark.  It shares no
 * code with the HIP library.
 *
 * What it computes (paper references by section / equation):
 *  - grids of Table T1: Ex (x-,y+,z+), Ey (x+,y-,z+), Ez (x+,y+,z-),
 *    Hx (x+,y-,z-), Hy (x-,y+,z-), Hz (x-,y-,z+); "+" has n+1 nodes, "-" n+2;
 *  - E7-E12 written row by row (E24, Algorithms 1-2): the interior rows are
 *    the two-point Yee difference, the first and last rows are the Appendix
 *    closures of D+ (two rows per end) and D- (three rows per end);
 *  - the SAT penalties folded into those rows (equivalent to E13-E15 with
 *    E18 and E19-E21 with E23): a PEC face flips the sign of the boundary E
 *    value in the first/last D- row of the H equations; a PMC face flips the
 *    sign of the boundary H value in the first/last D+ row of the E
 *    equations;
 *  - an absorbing face (not in the paper): the PMC row change plus a damping
 *    2/(eta h) on the tangential E nodes of the face;
 *  - leapfrog (Section V) with E^{n+1} = Ca E^n + Cb (curl H^{n+1/2} + J),
 *    Ca = (1-b)/(1+b), Cb = (dt/eps)/(1+b), b = dt (sigma + sigma_abc)/(2 eps);
 *  - energy W^n (E16 with the leapfrog pairing of H).
 * Node materials: mean of the per-cell values over the cells whose closed
 * box contains the node.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NC 6
enum { EX, EY, EZ, HX, HY, HZ };
enum { F_PEC = 0, F_PMC = 1, F_ABC = 2 };

static const double MU0 = 4e-7 * 3.14159265358979323846;
static const double C0 = 299792458.0;

/* grid type per component and axis: 1 = "+" (n+1 nodes), 0 = "-" (n+2) */
static const int PLUS[NC][3] = {
    {0, 1, 1}, {1, 0, 1}, {1, 1, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

/* E7-E12: target <- sign * D^axis(source) */
typedef struct { int src, axis, sign; } term;
static const term CURL[NC][2] = {
    {{HZ, 1, +1}, {HY, 2, -1}}, {{HX, 2, +1}, {HZ, 0, -1}}, {{HY, 0, +1}, {HX, 1, -1}},
    {{EY, 2, +1}, {EZ, 1, -1}}, {{EZ, 0, +1}, {EX, 2, -1}}, {{EX, 1, +1}, {EY, 0, -1}}};

typedef struct {
    int n[3];
    double h[3];
    const double *eps_r, *mu_r, *sigma; /* per cell, x fastest, NULL = 1,1,0 */
    int faces[6];                       /* -x,+x,-y,+y,-z,+z */
    double dt;
    int nsrc;
    const int *src_comp, *src_node;     /* node: 3 ints per source */
    const int *src_wave;                /* 0 gauss, 1 modulated gauss */
    const double *src_par;              /* tw, t0, f0, amp per source */
    int nprobe;
    const int *probe_comp, *probe_node;
    long step0;                         /* index of the first step (time origin) */
} oracle_cfg;

static int dim(int c, int a, const int n[3]) { return PLUS[c][a] ? n[a] + 1 : n[a] + 2; }

/* Appendix row r of h*D+ (from "-" data to "+" node r); flip = PMC/absorbing */
static int dplus_row(int n, int r, int flip_lo, int flip_hi, int idx[3], double c[3]) {
    if (r == 0) {
        idx[0] = 0; idx[1] = 1; idx[2] = 2;
        c[0] = flip_lo ? 1.0 : -1.0; c[1] = 0.5; c[2] = 0.5;
        return 3;
    }
    if (r == 1) {
        idx[0] = 0; idx[1] = 1; idx[2] = 2;
        c[0] = -0.5; c[1] = -0.25; c[2] = 0.75;
        return 3;
    }
    if (r == n - 1) {
        idx[0] = n - 1; idx[1] = n; idx[2] = n + 1;
        c[0] = -0.75; c[1] = 0.25; c[2] = 0.5;
        return 3;
    }
    if (r == n) {
        idx[0] = n - 1; idx[1] = n; idx[2] = n + 1;
        c[0] = -0.5; c[1] = -0.5; c[2] = flip_hi ? -1.0 : 1.0;
        return 3;
    }
    idx[0] = r; idx[1] = r + 1;
    c[0] = -1.0; c[1] = 1.0;
    return 2;
}

/* Appendix row r of h*D- (from "+" data to "-" node r); flip = PEC */
static int dminus_row(int n, int r, int flip_lo, int flip_hi, int idx[3], double c[3]) {
    if (r == 0) {
        idx[0] = 0; idx[1] = 1;
        c[0] = flip_lo ? 1.0 : -1.0; c[1] = 1.0;
        return 2;
    }
    if (r == 1) {
        idx[0] = 0; idx[1] = 1;
        c[0] = -1.0; c[1] = 1.0;
        return 2;
    }
    if (r == 2) {
        idx[0] = 0; idx[1] = 1; idx[2] = 2;
        c[0] = -0.2; c[1] = -0.6; c[2] = 0.8;
        return 3;
    }
    if (r == n - 1) {
        idx[0] = n - 2; idx[1] = n - 1; idx[2] = n;
        c[0] = -0.8; c[1] = 0.6; c[2] = 0.2;
        return 3;
    }
    if (r == n || r == n + 1) {
        idx[0] = n - 1; idx[1] = n;
        c[0] = -1.0; c[1] = (r == n + 1 && flip_hi) ? -1.0 : 1.0;
        return 2;
    }
    idx[0] = r - 1; idx[1] = r;
    c[0] = -1.0; c[1] = 1.0;
    return 2;
}

static double weight(int plus, int n, int r, double h) {
    if (plus) return (r == 0 || r == n) ? 0.5 * h : h;
    if (r == 0 || r == n + 1) return 0.5 * h;
    if (r == 1 || r == n) return 0.25 * h;
    if (r == 2 || r == n - 1) return 1.25 * h;
    return h;
}

/* cells containing node r of an axis: lo..hi inclusive */
static void cell_range(int plus, int n, int r, int *lo, int *hi) {
    if (plus) {
        *lo = r - 1 < 0 ? 0 : r - 1;
        *hi = r > n - 1 ? n - 1 : r;
    } else {
        int c = r == 0 ? 0 : (r == n + 1 ? n - 1 : r - 1);
        *lo = *hi = c;
    }
}

static double node_mean(const double *cells, double dflt, int c, const int n[3], int i, int j, int k) {
    if (!cells) return dflt;
    int lo[3], hi[3], r[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) cell_range(PLUS[c][a], n[a], r[a], &lo[a], &hi[a]);
    double acc = 0.0;
    int cnt = 0;
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
                acc += cells[(size_t)x + (size_t)n[0] * ((size_t)y + (size_t)n[1] * z)];
                ++cnt;
            }
    return acc / cnt;
}

static double wave(int kind, double t, const double *p) {
    double g = exp(-4.0 * 3.14159265358979323846 * (t - p[1]) * (t - p[1]) / (p[0] * p[0]));
    return kind == 1 ? sin(2.0 * 3.14159265358979323846 * p[2] * t) * g : g;
}

/* Runs nsteps leapfrog steps in place on f[6]; energy[s] = W^{step0+s};
 * probes[p*nsteps + s] = sample of E^{n+1}.  Returns 0 on success. */
int oracle_run(const oracle_cfg *cfg, double *f0, double *f1, double *f2, double *f3,
               double *f4, double *f5, long nsteps, double *energy, double *probes, int nthreads) {
    double *f[NC] = {f0, f1, f2, f3, f4, f5};
    const int *n = cfg->n;
    for (int a = 0; a < 3; ++a)
        if (n[a] < 4) return -1;
    const double eps0 = 1.0 / (MU0 * C0 * C0);
    const double dt = cfg->dt;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    /* per-node coefficients */
    double *ca[3], *cb[3], *we[3], *db[3], *wh[3];
    size_t sz[NC];
    for (int c = 0; c < NC; ++c) sz[c] = (size_t)dim(c, 0, n) * dim(c, 1, n) * dim(c, 2, n);
    for (int c = 0; c < 3; ++c) {
        ca[c] = malloc(sz[c] * sizeof(double));
        cb[c] = malloc(sz[c] * sizeof(double));
        we[c] = malloc(sz[c] * sizeof(double));
        db[c] = malloc(sz[c + 3] * sizeof(double));
        wh[c] = malloc(sz[c + 3] * sizeof(double));
    }
    for (int c = 0; c < 3; ++c) {
        int sx = dim(c, 0, n), sy = dim(c, 1, n), szz = dim(c, 2, n);
        for (int k = 0; k < szz; ++k)
            for (int j = 0; j < sy; ++j)
                for (int i = 0; i < sx; ++i) {
                    size_t o = (size_t)i + (size_t)sx * ((size_t)j + (size_t)sy * k);
                    double eps = eps0 * node_mean(cfg->eps_r, 1.0, c, n, i, j, k);
                    double mu = MU0 * node_mean(cfg->mu_r, 1.0, c, n, i, j, k);
                    double sig = node_mean(cfg->sigma, 0.0, c, n, i, j, k);
                    double eta = sqrt(mu / eps);
                    int r[3] = {i, j, k};
                    for (int a = 0; a < 3; ++a) {
                        if (a == c) continue; /* normal component */
                        if (r[a] == 0 && cfg->faces[2 * a] == F_ABC) sig += 2.0 / (eta * cfg->h[a]);
                        if (r[a] == n[a] && cfg->faces[2 * a + 1] == F_ABC) sig += 2.0 / (eta * cfg->h[a]);
                    }
                    double b = dt * sig / (2.0 * eps);
                    ca[c][o] = (1.0 - b) / (1.0 + b);
                    cb[c][o] = (dt / eps) / (1.0 + b);
                    we[c][o] = eps * weight(PLUS[c][0], n[0], i, cfg->h[0]) *
                               weight(PLUS[c][1], n[1], j, cfg->h[1]) * weight(PLUS[c][2], n[2], k, cfg->h[2]);
                }
        int hc = c + 3;
        sx = dim(hc, 0, n); sy = dim(hc, 1, n); szz = dim(hc, 2, n);
        for (int k = 0; k < szz; ++k)
            for (int j = 0; j < sy; ++j)
                for (int i = 0; i < sx; ++i) {
                    size_t o = (size_t)i + (size_t)sx * ((size_t)j + (size_t)sy * k);
                    double mu = MU0 * node_mean(cfg->mu_r, 1.0, hc, n, i, j, k);
                    db[c][o] = dt / mu;
                    wh[c][o] = mu * weight(PLUS[hc][0], n[0], i, cfg->h[0]) *
                               weight(PLUS[hc][1], n[1], j, cfg->h[1]) * weight(PLUS[hc][2], n[2], k, cfg->h[2]);
                }
    }
    double *hold = malloc((sz[3] > sz[4] ? (sz[3] > sz[5] ? sz[3] : sz[5]) : (sz[4] > sz[5] ? sz[4] : sz[5])) *
                          sizeof(double) * 3);
    double *hprev[3] = {hold, hold + sz[3], hold + sz[3] + sz[4]};

    for (long s = 0; s < nsteps; ++s) {
        long nstep = cfg->step0 + s;
        double w_h = 0.0, w_e = 0.0;
        /* ---------------- H^{n+1/2} = H^{n-1/2} + dt/mu * sum sign D-(E) */
        for (int hc = HX; hc <= HZ; ++hc) {
            int sx = dim(hc, 0, n), sy = dim(hc, 1, n), szz = dim(hc, 2, n);
            double *H = f[hc];
            memcpy(hprev[hc - 3], H, sz[hc] * sizeof(double));
#pragma omp parallel for reduction(+ : w_h) schedule(static)
            for (int k = 0; k < szz; ++k)
                for (int j = 0; j < sy; ++j)
                    for (int i = 0; i < sx; ++i) {
                        size_t o = (size_t)i + (size_t)sx * ((size_t)j + (size_t)sy * k);
                        int r[3] = {i, j, k};
                        double acc = 0.0;
                        for (int t = 0; t < 2; ++t) {
                            const term *tm = &CURL[hc][t];
                            int a = tm->axis, ec = tm->src;
                            int idx[3];
                            double cf[3];
                            int m = dminus_row(n[a], r[a], cfg->faces[2 * a] == F_PEC,
                                               cfg->faces[2 * a + 1] == F_PEC, idx, cf);
                            int es[3] = {dim(ec, 0, n), dim(ec, 1, n), dim(ec, 2, n)};
                            double d = 0.0;
                            for (int q = 0; q < m; ++q) {
                                int rr[3] = {i, j, k};
                                rr[a] = idx[q];
                                d += cf[q] * f[ec][(size_t)rr[0] + (size_t)es[0] * ((size_t)rr[1] + (size_t)es[1] * rr[2])];
                            }
                            acc += tm->sign * d / cfg->h[a];
                        }
                        double hn = H[o] + db[hc - 3][o] * acc;
                        w_h += 0.5 * wh[hc - 3][o] * hn * H[o];
                        H[o] = hn;
                    }
        }
        /* E part of W^n uses E^n, before the E update */
        for (int c = EX; c <= EZ; ++c) {
            double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
            for (long o = 0; o < (long)sz[c]; ++o) acc += 0.5 * we[c][o] * f[c][o] * f[c][o];
            w_e += acc;
        }
        if (energy) energy[s] = w_e + w_h;
        /* ---------------- E^{n+1} = Ca E^n + Cb (sum sign D+(H) + J) */
        double t = ((double)nstep + 0.5) * dt;
        for (int c = EX; c <= EZ; ++c) {
            int sx = dim(c, 0, n), sy = dim(c, 1, n), szz = dim(c, 2, n);
#pragma omp parallel for schedule(static)
            for (int k = 0; k < szz; ++k)
                for (int j = 0; j < sy; ++j)
                    for (int i = 0; i < sx; ++i) {
                        size_t o = (size_t)i + (size_t)sx * ((size_t)j + (size_t)sy * k);
                        int r[3] = {i, j, k};
                        double acc = 0.0;
                        for (int tt = 0; tt < 2; ++tt) {
                            const term *tm = &CURL[c][tt];
                            int a = tm->axis, hc = tm->src;
                            int idx[3];
                            double cf[3];
                            int flo = cfg->faces[2 * a] == F_PMC || cfg->faces[2 * a] == F_ABC;
                            int fhi = cfg->faces[2 * a + 1] == F_PMC || cfg->faces[2 * a + 1] == F_ABC;
                            int m = dplus_row(n[a], r[a], flo, fhi, idx, cf);
                            int hs[3] = {dim(hc, 0, n), dim(hc, 1, n), dim(hc, 2, n)};
                            double d = 0.0;
                            for (int q = 0; q < m; ++q) {
                                int rr[3] = {i, j, k};
                                rr[a] = idx[q];
                                d += cf[q] * f[hc][(size_t)rr[0] + (size_t)hs[0] * ((size_t)rr[1] + (size_t)hs[1] * rr[2])];
                            }
                            acc += tm->sign * d / cfg->h[a];
                        }
                        for (int q = 0; q < cfg->nsrc; ++q) {
                            const int *nd = cfg->src_node + 3 * q;
                            if (cfg->src_comp[q] == c && nd[0] == i && nd[1] == j && nd[2] == k)
                                acc += cfg->src_par[4 * q + 3] * wave(cfg->src_wave[q], t, cfg->src_par + 4 * q);
                        }
                        f[c][o] = ca[c][o] * f[c][o] + cb[c][o] * acc;
                    }
        }
        for (int p = 0; p < cfg->nprobe; ++p) {
            int c = cfg->probe_comp[p];
            const int *nd = cfg->probe_node + 3 * p;
            size_t o = (size_t)nd[0] + (size_t)dim(c, 0, n) * ((size_t)nd[1] + (size_t)dim(c, 1, n) * nd[2]);
            if (probes) probes[(size_t)p * nsteps + s] = f[c][o];
        }
    }
    free(hold);
    for (int c = 0; c < 3; ++c) {
        free(ca[c]); free(cb[c]); free(we[c]); free(db[c]); free(wh[c]);
    }
    return 0;
}

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

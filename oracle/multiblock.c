/*
 * Loop form of the 3D SBP-SAT FDTD leapfrog step over several coupled
 * blocks, fp64.
 *
 * TEST INFRASTRUCTURE ONLY (the oracle): used by the tests.  It shares no
 * code with the HIP library, and none with the single-block loop form
 * (loops.c) either.
 *
 * What it computes, per block (paper references by section / equation):
 *  - the grids of Table T1 ("+" grid n+1 nodes, "-" grid n+2), arrays x
 *    fastest (the Kronecker order of ED_1-ED_3);
 *  - E7-E12 row by row: interior rows are the two-point difference, the
 *    first and last rows the Appendix closures (D+: two rows per end, D-:
 *    three rows per end), all divided by h;
 *  - the face penalties folded into the boundary rows: PEC (E13-E15 with
 *    the values of E18 placed as E17 assigns them) flips the boundary-E
 *    coefficient of the first / last D- row of the H equations; PMC
 *    (E19-E21 with E23) flips the boundary-H coefficient of the first /
 *    last D+ row of the E equations; an absorbing face (not in the paper)
 *    is the PMC row change plus the damping 2/(eta h) of the tangential E
 *    nodes on the face, taken semi-implicitly with the conductivity;
 *  - block interfaces, the pattern of EPBC1-EPBC6 at zero phase with
 *    sigma = chi = +-1/2 (EPBCP): the own boundary value's coefficient in
 *    the boundary row moves onto the neighbour's value at the same face
 *    node, which is the neighbour's face value itself (same mesh) or its
 *    interpolation (1:2, tensor product of one-dimensional maps along the
 *    two tangential axes, supplied by the caller as sparse rows);
 *  - the leapfrog of Section V: H^{n+1/2} = H^{n-1/2} + dt/mu curl_h(E^n),
 *    E^{n+1} = Ca E^n + Cb (curl_e(H^{n+1/2}) + J), Ca = (1-b)/(1+b),
 *    Cb = (dt/eps)/(1+b), b = dt (sigma + sigma_abc)/(2 eps);
 *  - the energy W^n of E16 with the leapfrog pairing of H, summed over the
 *    blocks.
 * Node materials: the mean of the per-cell values over the cells of the
 * node's own block whose closed box contains the node.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { EX, EY, EZ, HX, HY, HZ };
enum { MB_PEC = 0, MB_PMC = 1, MB_ABC = 2, MB_IFACE = 3 };

static const double PI = 3.14159265358979323846;
static const double MU0 = 4e-7 * 3.14159265358979323846;
static const double C0 = 299792458.0;

/* Table T1: 1 = "+" grid along the axis, 0 = "-" grid */
static const int GP[6][3] = {{0, 1, 1}, {1, 0, 1}, {1, 1, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

/* E7-E12: d(target)/dt = D^axis0(source0) - D^axis1(source1) */
static const int TERM_SRC[6][2] = {{HZ, HY}, {HX, HZ}, {HY, HX}, {EY, EZ}, {EZ, EX}, {EX, EY}};
static const int TERM_AX[6][2] = {{1, 2}, {2, 0}, {0, 1}, {2, 1}, {0, 2}, {1, 0}};

typedef struct {
    int n[3];
    double h[3];
    const double *eps_r, *mu_r, *sigma; /* per cell (nz, ny, nx), NULL: 1, 1, 0 */
    int faces[6];                       /* -x +x -y +y -z +z: MB_* */
    double *f[6];                       /* Ex Ey Ez Hx Hy Hz, x fastest, in place */
} mb_block;

/* Sparse rows of a one-dimensional map from the neighbour's face nodes to
 * the own face nodes along one tangential axis: own node r takes
 * sum_{q = ptr[r]}^{ptr[r+1]-1} val[q] * nb[col[q]].  NULL ptr: identity. */
typedef struct {
    const int *ptr, *col;
    const double *val;
} mb_map;

/* A coupled face: `block`'s face `face` takes its neighbour values from
 * `nb`'s face `nb_face`; map[t][g] is the map along the t-th tangential axis
 * (ascending) for components on grid g ("+" 1, "-" 0) along that axis. */
typedef struct {
    int block, face, nb, nb_face;
    mb_map map[2][2];
} mb_link;

typedef struct {
    int nblocks;
    mb_block *blocks;
    int nlinks;
    const mb_link *links;
    double dt;
    int nsrc;
    const int *src; /* block, comp, i, j, k, waveform (0 gauss, 1 modulated) */
    const double *src_par; /* tw, t0, f0, amp */
    int nprobe;
    const int *probe; /* block, comp, i, j, k */
    long step0;
} mb_cfg;

/* one boundary-aware row of D+ or D- along an axis: taps at node offsets
 * d[q] (relative to the row's node), coefficients c[q] (already / h), and
 * cn (already / h) times the neighbour value on an interface face */
typedef struct {
    int d[3];
    double c[3];
    double cn;
    int nbr;
} row_t;

static int dimc(const int n[3], int c, int a) { return GP[c][a] ? n[a] + 1 : n[a] + 2; }

/* Appendix row r of D+ ("-" data -> "+" node r), with the face rules. */
static row_t dplus(int n, int r, int lo, int hi, double h) {
    row_t w = {{0, 0, 0}, {0.0, 0.0, 0.0}, 0.0, 0};
    int idx[3] = {r, r + 1, r + 1};
    double c[3] = {-1.0, 1.0, 0.0};
    if (r == 0) {
        idx[0] = 0; idx[1] = 1; idx[2] = 2;
        c[0] = -1.0; c[1] = 0.5; c[2] = 0.5;
        if (lo == MB_PMC || lo == MB_ABC) c[0] = 1.0;
        if (lo == MB_IFACE) { w.cn = c[0]; w.nbr = 1; c[0] = 0.0; }
    } else if (r == 1) {
        idx[0] = 0; idx[1] = 1; idx[2] = 2;
        c[0] = -0.5; c[1] = -0.25; c[2] = 0.75;
    } else if (r == n - 1) {
        idx[0] = n - 1; idx[1] = n; idx[2] = n + 1;
        c[0] = -0.75; c[1] = 0.25; c[2] = 0.5;
    } else if (r == n) {
        idx[0] = n - 1; idx[1] = n; idx[2] = n + 1;
        c[0] = -0.5; c[1] = -0.5; c[2] = 1.0;
        if (hi == MB_PMC || hi == MB_ABC) c[2] = -1.0;
        if (hi == MB_IFACE) { w.cn = c[2]; w.nbr = 1; c[2] = 0.0; }
    }
    for (int q = 0; q < 3; ++q) {
        w.d[q] = idx[q] - r;
        w.c[q] = c[q] / h;
    }
    w.cn /= h;
    return w;
}

/* Appendix row r of D- ("+" data -> "-" node r), with the face rules. */
static row_t dminus(int n, int r, int lo, int hi, double h) {
    row_t w = {{0, 0, 0}, {0.0, 0.0, 0.0}, 0.0, 0};
    int idx[3] = {r - 1, r, r};
    double c[3] = {-1.0, 1.0, 0.0};
    if (r == 0 || r == 1) {
        idx[0] = 0; idx[1] = 1; idx[2] = 1;
        if (r == 0 && lo == MB_PEC) c[0] = 1.0;
        if (r == 0 && lo == MB_IFACE) { w.cn = c[0]; w.nbr = 1; c[0] = 0.0; }
    } else if (r == 2) {
        idx[0] = 0; idx[1] = 1; idx[2] = 2;
        c[0] = -0.2; c[1] = -0.6; c[2] = 0.8;
    } else if (r == n - 1) {
        idx[0] = n - 2; idx[1] = n - 1; idx[2] = n;
        c[0] = -0.8; c[1] = 0.6; c[2] = 0.2;
    } else if (r == n || r == n + 1) {
        idx[0] = n - 1; idx[1] = n; idx[2] = n;
        if (r == n + 1 && hi == MB_PEC) c[1] = -1.0;
        if (r == n + 1 && hi == MB_IFACE) { w.cn = c[1]; w.nbr = 1; c[1] = 0.0; }
    }
    for (int q = 0; q < 3; ++q) {
        w.d[q] = idx[q] - r;
        w.c[q] = c[q] / h;
    }
    w.cn /= h;
    return w;
}

/* norm weight of node r (Appendix P+, P-, times h) */
static double wnode(int plus, int n, int r, double h) {
    if (plus) return (r == 0 || r == n) ? 0.5 * h : h;
    if (r == 0 || r == n + 1) return 0.5 * h;
    if (r == 1 || r == n) return 0.25 * h;
    if (r == 2 || r == n - 1) return 1.25 * h;
    return h;
}

/* mean of per-cell values over the cells whose closed box holds the node */
static double node_mean(const double *cells, double dflt, const int n[3], int c, int i, int j, int k) {
    if (!cells) return dflt;
    int r[3] = {i, j, k}, lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        if (GP[c][a]) {
            lo[a] = r[a] - 1 < 0 ? 0 : r[a] - 1;
            hi[a] = r[a] > n[a] - 1 ? n[a] - 1 : r[a];
        } else {
            lo[a] = hi[a] = r[a] == 0 ? 0 : (r[a] == n[a] + 1 ? n[a] - 1 : r[a] - 1);
        }
    }
    double s = 0.0;
    int cnt = 0;
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
                s += cells[(size_t)x + (size_t)n[0] * ((size_t)y + (size_t)n[1] * z)];
                ++cnt;
            }
    return s / cnt;
}

static double pulse(int kind, double t, const double *p) {
    const double g = exp(-4.0 * PI * (t - p[1]) * (t - p[1]) / (p[0] * p[0]));
    return kind == 1 ? sin(2.0 * PI * p[2] * t) * g : g;
}

/* per block: coefficients, rows, face buffers */
typedef struct {
    size_t sz[6];
    double *ca[3], *cb[3], *we[3], *db[3], *wh[3];
    row_t *rp[3], *rm[3]; /* D+ rows 0..n, D- rows 0..n+1 per axis */
    /* neighbour values of the tangential components on each interface face:
     * fb[face][c] over the own face nodes of component c (NULL otherwise) */
    double *fb[6][6];
    const mb_link *link[6];
} blk_t;

static void tangential(int axis, int t[2]) {
    t[0] = axis == 0 ? 1 : 0;
    t[1] = axis == 2 ? 1 : 2;
}

/* the two components of field `h_field` (0 E, 1 H) tangential to `axis` */
static void tcomps(int axis, int h_field, int c[2]) {
    int t[2];
    tangential(axis, t);
    c[0] = 3 * h_field + t[0];
    c[1] = 3 * h_field + t[1];
}

/* face node count of component c on a face normal to `axis` */
static size_t face_nodes(const int n[3], int c, int axis) {
    int t[2];
    tangential(axis, t);
    return (size_t)dimc(n, c, t[0]) * dimc(n, c, t[1]);
}

/* neighbour values of component c on link L: own face node (p0, p1) takes
 * sum_q0 sum_q1 M0[p0, q0] M1[p1, q1] nb(q0, q1) */
static void gather(const mb_cfg *cfg, const mb_link *L, int c, double *out, double *tmp) {
    const mb_block *B = &cfg->blocks[L->block], *N = &cfg->blocks[L->nb];
    const int axis = L->face / 2;
    int t[2];
    tangential(axis, t);
    const int nbn = (L->nb_face & 1) ? dimc(N->n, c, axis) - 1 : 0; /* neighbour face index */
    const int m0 = dimc(N->n, c, t[0]), m1 = dimc(N->n, c, t[1]);
    const int p0n = dimc(B->n, c, t[0]), p1n = dimc(B->n, c, t[1]);
    const int s[3] = {1, dimc(N->n, c, 0), dimc(N->n, c, 0) * dimc(N->n, c, 1)};
    const double *src = N->f[c];
    const mb_map *M0 = &L->map[0][GP[c][t[0]]], *M1 = &L->map[1][GP[c][t[1]]];
    /* along the first tangential axis: tmp[q1][p0] */
    for (int q1 = 0; q1 < m1; ++q1)
        for (int p0 = 0; p0 < p0n; ++p0) {
            double v = 0.0;
            const size_t base = (size_t)nbn * s[axis] + (size_t)q1 * s[t[1]];
            if (!M0->ptr) {
                v = src[base + (size_t)p0 * s[t[0]]];
            } else {
                for (int q = M0->ptr[p0]; q < M0->ptr[p0 + 1]; ++q)
                    v += M0->val[q] * src[base + (size_t)M0->col[q] * s[t[0]]];
            }
            tmp[(size_t)q1 * p0n + p0] = v;
        }
    (void)m0;
    /* along the second: out[p1][p0] */
    for (int p1 = 0; p1 < p1n; ++p1)
        for (int p0 = 0; p0 < p0n; ++p0) {
            double v = 0.0;
            if (!M1->ptr) {
                v = tmp[(size_t)p1 * p0n + p0];
            } else {
                for (int q = M1->ptr[p1]; q < M1->ptr[p1 + 1]; ++q)
                    v += M1->val[q] * tmp[(size_t)M1->col[q] * p0n + p0];
            }
            out[(size_t)p1 * p0n + p0] = v;
        }
}

static void gather_all(const mb_cfg *cfg, blk_t *bk, int h_field, double *tmp) {
    for (int l = 0; l < cfg->nlinks; ++l) {
        const mb_link *L = &cfg->links[l];
        int cc[2];
        tcomps(L->face / 2, h_field, cc);
        for (int q = 0; q < 2; ++q) gather(cfg, L, cc[q], bk[L->block].fb[L->face][cc[q]], tmp);
    }
}

/* one curl term of a target component: D^a of the source component, with
 * the rows of the target's grid along a (D+ for E targets, D- for H
 * targets) and the neighbour values of the source on the two faces of a */
typedef struct {
    const double *u;      /* source component */
    size_t sy, sz, sa;    /* its strides along y, z and along a */
    int a, t0, t1;        /* difference axis, tangential axes */
    const row_t *rows;
    const double *nb[2];  /* neighbour values on the low / high face, or NULL */
    size_t nbw;           /* face-row width (nodes along t0) */
} term_t;

static term_t term_of(const mb_block *B, const blk_t *K, int tgt, int t) {
    term_t T;
    const int src = TERM_SRC[tgt][t], a = TERM_AX[tgt][t];
    const int *n = B->n;
    int tt[2];
    tangential(a, tt);
    T.u = B->f[src];
    T.sy = (size_t)dimc(n, src, 0);
    T.sz = T.sy * dimc(n, src, 1);
    T.sa = a == 0 ? 1 : (a == 1 ? T.sy : T.sz);
    T.a = a;
    T.t0 = tt[0];
    T.t1 = tt[1];
    T.rows = tgt >= HX ? K->rm[a] : K->rp[a];
    T.nb[0] = K->fb[2 * a][src];
    T.nb[1] = K->fb[2 * a + 1][src];
    T.nbw = (size_t)dimc(n, src, tt[0]);
    return T;
}

/* the term's difference at target node r (whose indices along the other two
 * axes index the source, both sharing the grid type there) */
static double apply(const term_t *T, const int r[3]) {
    const row_t *R = &T->rows[r[T->a]];
    const size_t o = (size_t)r[0] + T->sy * r[1] + T->sz * r[2];
    const long sa = (long)T->sa;
    double d = R->c[0] * T->u[o + R->d[0] * sa] + R->c[1] * T->u[o + R->d[1] * sa] + R->c[2] * T->u[o + R->d[2] * sa];
    if (R->nbr) {
        const double *f = T->nb[r[T->a] == 0 ? 0 : 1];
        d += R->cn * f[(size_t)r[T->t1] * T->nbw + r[T->t0]];
    }
    return d;
}

/* Runs nsteps steps in place; energy[s] = W^{step0+s}; probes[p*nsteps+s]
 * = the probed node after step step0+s (E^{n+1}, or H^{n+1/2}). */
int mb_run(const mb_cfg *cfg, long nsteps, double *energy, double *probes, int nthreads) {
    const double eps0 = 1.0 / (MU0 * C0 * C0), dt = cfg->dt;
    const int nb = cfg->nblocks;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    for (int b = 0; b < nb; ++b)
        for (int a = 0; a < 3; ++a)
            if (cfg->blocks[b].n[a] < 4) return -1;
    blk_t *bk = calloc((size_t)nb, sizeof(blk_t));
    size_t tmpn = 0;
    for (int l = 0; l < cfg->nlinks; ++l) {
        const mb_link *L = &cfg->links[l];
        if (L->block < 0 || L->block >= nb || L->nb < 0 || L->nb >= nb) return -2;
        bk[L->block].link[L->face] = L;
        const mb_block *B = &cfg->blocks[L->block], *N = &cfg->blocks[L->nb];
        for (int c = 0; c < 6; ++c) {
            int t[2];
            tangential(L->face / 2, t);
            if (c % 3 == L->face / 2) continue;
            bk[L->block].fb[L->face][c] = calloc(face_nodes(B->n, c, L->face / 2), sizeof(double));
            const size_t need = (size_t)dimc(N->n, c, t[1]) * dimc(B->n, c, t[0]);
            if (need > tmpn) tmpn = need;
        }
    }
    double *tmp = malloc((tmpn ? tmpn : 1) * sizeof(double));
    for (int b = 0; b < nb; ++b) {
        const mb_block *B = &cfg->blocks[b];
        blk_t *K = &bk[b];
        const int *n = B->n;
        for (int a = 0; a < 3; ++a) {
            const int lo = B->faces[2 * a], hi = B->faces[2 * a + 1];
            K->rp[a] = malloc((size_t)(n[a] + 1) * sizeof(row_t));
            K->rm[a] = malloc((size_t)(n[a] + 2) * sizeof(row_t));
            for (int r = 0; r <= n[a]; ++r) K->rp[a][r] = dplus(n[a], r, lo, hi, B->h[a]);
            for (int r = 0; r <= n[a] + 1; ++r) K->rm[a][r] = dminus(n[a], r, lo, hi, B->h[a]);
        }
        for (int c = 0; c < 6; ++c) K->sz[c] = (size_t)dimc(n, c, 0) * dimc(n, c, 1) * dimc(n, c, 2);
        for (int c = 0; c < 3; ++c) {
            K->ca[c] = malloc(K->sz[c] * sizeof(double));
            K->cb[c] = malloc(K->sz[c] * sizeof(double));
            K->we[c] = malloc(K->sz[c] * sizeof(double));
            K->db[c] = malloc(K->sz[c + 3] * sizeof(double));
            K->wh[c] = malloc(K->sz[c + 3] * sizeof(double));
            const int sx = dimc(n, c, 0), sy = dimc(n, c, 1), szz = dimc(n, c, 2);
#pragma omp parallel for schedule(static)
            for (int k = 0; k < szz; ++k)
                for (int j = 0; j < sy; ++j)
                    for (int i = 0; i < sx; ++i) {
                        const size_t o = (size_t)i + (size_t)sx * ((size_t)j + (size_t)sy * k);
                        const double eps = eps0 * node_mean(B->eps_r, 1.0, n, c, i, j, k);
                        const double mu = MU0 * node_mean(B->mu_r, 1.0, n, c, i, j, k);
                        double sig = node_mean(B->sigma, 0.0, n, c, i, j, k);
                        const double eta = sqrt(mu / eps);
                        const int r[3] = {i, j, k};
                        for (int a = 0; a < 3; ++a) {
                            if (a == c) continue; /* the normal component takes no damping */
                            if (r[a] == 0 && B->faces[2 * a] == MB_ABC) sig += 2.0 / (eta * B->h[a]);
                            if (r[a] == n[a] && B->faces[2 * a + 1] == MB_ABC) sig += 2.0 / (eta * B->h[a]);
                        }
                        const double beta = dt * sig / (2.0 * eps);
                        K->ca[c][o] = (1.0 - beta) / (1.0 + beta);
                        K->cb[c][o] = (dt / eps) / (1.0 + beta);
                        K->we[c][o] = eps * wnode(GP[c][0], n[0], i, B->h[0]) * wnode(GP[c][1], n[1], j, B->h[1]) *
                                      wnode(GP[c][2], n[2], k, B->h[2]);
                    }
            const int hc = c + 3;
            const int hx = dimc(n, hc, 0), hy = dimc(n, hc, 1), hz = dimc(n, hc, 2);
#pragma omp parallel for schedule(static)
            for (int k = 0; k < hz; ++k)
                for (int j = 0; j < hy; ++j)
                    for (int i = 0; i < hx; ++i) {
                        const size_t o = (size_t)i + (size_t)hx * ((size_t)j + (size_t)hy * k);
                        const double mu = MU0 * node_mean(B->mu_r, 1.0, n, hc, i, j, k);
                        K->db[c][o] = dt / mu;
                        K->wh[c][o] = mu * wnode(GP[hc][0], n[0], i, B->h[0]) * wnode(GP[hc][1], n[1], j, B->h[1]) *
                                      wnode(GP[hc][2], n[2], k, B->h[2]);
                    }
        }
    }

    for (long s = 0; s < nsteps; ++s) {
        const long nstep = cfg->step0 + s;
        double w = 0.0;
        /* ---- H^{n+1/2} from E^n */
        gather_all(cfg, bk, 0, tmp);
        for (int b = 0; b < nb; ++b) {
            const mb_block *B = &cfg->blocks[b];
            blk_t *K = &bk[b];
            const int *n = B->n;
            for (int hc = HX; hc <= HZ; ++hc) {
                const int sx = dimc(n, hc, 0), sy = dimc(n, hc, 1), szz = dimc(n, hc, 2);
                double *H = B->f[hc];
                const double *db = K->db[hc - 3], *wh = K->wh[hc - 3];
                term_t T[2];
                for (int t = 0; t < 2; ++t) T[t] = term_of(B, K, hc, t);
                double acc_w = 0.0;
#pragma omp parallel for reduction(+ : acc_w) schedule(static)
                for (int k = 0; k < szz; ++k)
                    for (int j = 0; j < sy; ++j)
                        for (int i = 0; i < sx; ++i) {
                            const int r[3] = {i, j, k};
                            const double curl = apply(&T[0], r) - apply(&T[1], r);
                            const size_t o = (size_t)i + (size_t)sx * ((size_t)j + (size_t)sy * k);
                            const double hn = H[o] + db[o] * curl;
                            acc_w += 0.5 * wh[o] * hn * H[o];
                            H[o] = hn;
                        }
                w += acc_w;
            }
        }
        /* ---- the E part of W^n, from E^n */
        for (int b = 0; b < nb; ++b)
            for (int c = EX; c <= EZ; ++c) {
                const double *E = cfg->blocks[b].f[c], *we = bk[b].we[c];
                double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
                for (long o = 0; o < (long)bk[b].sz[c]; ++o) acc += 0.5 * we[o] * E[o] * E[o];
                w += acc;
            }
        if (energy) energy[s] = w;
        /* ---- E^{n+1} from H^{n+1/2} */
        gather_all(cfg, bk, 1, tmp);
        const double tn = ((double)nstep + 0.5) * dt;
        for (int b = 0; b < nb; ++b) {
            const mb_block *B = &cfg->blocks[b];
            blk_t *K = &bk[b];
            const int *n = B->n;
            for (int c = EX; c <= EZ; ++c) {
                const int sx = dimc(n, c, 0), sy = dimc(n, c, 1), szz = dimc(n, c, 2);
                double *E = B->f[c];
                const double *ca = K->ca[c], *cb = K->cb[c];
                term_t T[2];
                for (int t = 0; t < 2; ++t) T[t] = term_of(B, K, c, t);
#pragma omp parallel for schedule(static)
                for (int k = 0; k < szz; ++k)
                    for (int j = 0; j < sy; ++j)
                        for (int i = 0; i < sx; ++i) {
                            const int r[3] = {i, j, k};
                            double curl = apply(&T[0], r) - apply(&T[1], r);
                            for (int q = 0; q < cfg->nsrc; ++q) {
                                const int *S = cfg->src + 6 * q;
                                if (S[0] == b && S[1] == c && S[2] == i && S[3] == j && S[4] == k)
                                    curl += cfg->src_par[4 * q + 3] * pulse(S[5], tn, cfg->src_par + 4 * q);
                            }
                            const size_t o = (size_t)i + (size_t)sx * ((size_t)j + (size_t)sy * k);
                            E[o] = ca[o] * E[o] + cb[o] * curl;
                        }
            }
        }
        for (int p = 0; p < cfg->nprobe; ++p) {
            const int *P = cfg->probe + 5 * p;
            const mb_block *B = &cfg->blocks[P[0]];
            const int c = P[1];
            const size_t o = (size_t)P[2] + (size_t)dimc(B->n, c, 0) * ((size_t)P[3] + (size_t)dimc(B->n, c, 1) * P[4]);
            if (probes) probes[(size_t)p * nsteps + s] = B->f[c][o];
        }
    }
    free(tmp);
    for (int b = 0; b < nb; ++b) {
        blk_t *K = &bk[b];
        for (int a = 0; a < 3; ++a) {
            free(K->rp[a]);
            free(K->rm[a]);
            free(K->ca[a]); free(K->cb[a]); free(K->we[a]); free(K->db[a]); free(K->wh[a]);
        }
        for (int f = 0; f < 6; ++f)
            for (int c = 0; c < 6; ++c) free(K->fb[f][c]);
    }
    free(bk);
    return 0;
}

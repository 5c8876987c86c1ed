/*
 * FP64 CPU oracle for the FWI-gradient hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this file's library.  It shares no code with the HIP library: it is the
 * plain, slow definition of what that library must compute, written from
 * the paper's forward model and the adjoint-state gradient of its misfit.
 *
 * What it computes, per medium (all in double precision):
 *
 *  Coefficients (Sec. II-A, eq. 1-2; Sec. IV for the absorbing layer).
 *    kappa = rho c^2, b = 1/rho.
 *    D(ix,iz) = Dx(ix) + Dz(iz); Dx(i) = Dmax ((N-i)/N)^2 for i < N,
 *    Dmax ((i-(nx-1-N))/N)^2 for i > nx-1-N, 0 otherwise;
 *    Dmax = 3 cref ln(1/R) / (2 N h)   (quadratic profile, N = 20, R = 1e-3
 *    reproduces the paper's 1.46e6 at cref = 1500 m/s, h = 10 cm / 188).
 *    a = (2 - D^2 dt^2)/(1 + D dt), beta = (D dt - 1)/(1 + D dt),
 *    gamma = dt^2/(1 + D dt)    (eq. 2 with the Laplacian coefficient read as
 *    C^2 dt^2/(1+D dt); the printed single dt is dimensionally inconsistent).
 *
 *  Operator.  (L_b u)_x = h^-2 sum_{faces f=(x,x')} b_f (u_x' - u_x), with
 *    b_f = (b_x + b_x')/2 and, for a face on the grid border, u_x' = 0 and
 *    b_f = b_x.  This is eq. 1's rho d/dx(1/rho d/dx) in flux form; for
 *    constant rho, kappa L_b = c^2 * (5-point Laplacian), i.e. eq. 2.
 *
 *  Forward, transmit p (eq. 2-3).  u^-1 = u^0 = 0; for n = 0..T-1:
 *    u^{n+1} = a u^n + beta u^{n-1} + gamma kappa L_b u^n;
 *    u^{n+1}[src_p] += w_p[n];  d_p[n][r] = u^{n+1}[rcv_{p,r}].
 *
 *  Misfit (eq. 5-6, data term).  r = d - d_obs, J = sum r^2.
 *
 *  Adjoint (exact gradient of the discrete J, eq. 6).  lam^{T+1} = lam^{T+2} = 0;
 *    for t = T..1: lam^t = a lam^{t+1} + L_b(gamma kappa lam^{t+1}) + beta lam^{t+2}
 *                 + sum_r s_p[t-1][r] e_{rcv_{p,r}},   s = 2 r (or a given source);
 *    g_kappa(x) += gamma_x lam^t_x (L_b u^{t-1})_x;
 *    for each face f of x: G_f = -h^-2 (Delta_f u^{t-1}) (Delta_f w^t), w = gamma kappa lam^t;
 *    g_b(x) += G_f / 2 for an interior face, G_f for a border face.
 *    dJ/dw_p[n] = lam^{n+1}[src_p].
 *  Output: g_c = 2 rho c g_kappa, g_rho = c^2 g_kappa - b^2 g_b, summed over transmits.
 *
 * Fourth-order variant (order = 4).  Along each axis, the face flux between
 *    cells j and j+1 is F = b_f (9/8 (u_{j+1} - u_j) - 1/24 (u_{j+2} - u_{j-1}))
 *    with b_f = (b_j + b_{j+1})/2, and (L_b u)_i = h^-2 sum over both axes of
 *    9/8 (F_{i+1/2} - F_{i-1/2}) - 1/24 (F_{i+3/2} - F_{i-3/2})  (staggered
 *    fourth-order differences, so L_b = -h^-2 D^T B D stays symmetric).  Outside
 *    the grid u = 0 and b repeats the nearest cell of that row or column, which
 *    for order 2 is the border rule above.  The imaging term of a face becomes
 *    G_f = -h^-2 (D u)_f (D w)_f, shared half and half by the cells whose b
 *    make up b_f (ghost cells counting as the cell they repeat).
 *
 * Attenuation (the Sec. VII extension of the forward model): a per-cell
 *    damping rate eta(x) >= 0 (1/s) is added to eq. 1's damping term, so that
 *    D becomes D + eta everywhere in the coefficients above (eq. 2's a and
 *    beta discretise u_tt + 2 D u_t + D^2 u, so in a homogeneous medium the
 *    loss-free response is multiplied by exp(-eta t) in the continuum).  Its
 *    gradient follows from the update's dependence on e = (D + eta) dt:
 *      dJ/deta(x) = dt sum_{t=1..T} lam^t_x ( a'(e) u^{t-1}_x + beta'(e) u^{t-2}_x
 *                                            + gamma'(e) kappa_x (L_b u^{t-1})_x ),
 *      a' = -(e^2 + 2e + 2)/(1+e)^2, beta' = 2/(1+e)^2, gamma' = -dt^2/(1+e)^2,
 *    with lam^t the adjoint of the update that produced u^t (above).
 *
 * Replay of u^{t-1} in reverse order: every u^t is kept (store-all), or
 * (u^{jK}, u^{jK-1}) pairs are kept every K steps and each segment is
 * recomputed with the same step routine (bitwise identical to store-all).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, nz, nt, npml;
    double h, dt, pml_r, pml_cref;
    const double *c, *rho;          /* [nz*nx] */
    int32_t n_tx, n_rcv;
    const int32_t *src;             /* [n_tx] cell indices */
    const int32_t *rcv;             /* [n_tx*n_rcv] cell indices, duplicates allowed */
    const double *wavelet;          /* [n_tx][wavelet_stride], stride 0 = one shared row */
    int64_t wavelet_stride;
    const double *d_obs;            /* [n_tx][nt][n_rcv] or NULL */
    const double *d_adj;            /* adjoint source used instead of 2 (d - d_obs), or NULL */
    double *traces;                 /* out [n_tx][nt][n_rcv] or NULL */
    double *grad_c, *grad_rho;      /* out [nz*nx] or NULL */
    double *grad_kappa, *grad_b;    /* out [nz*nx] or NULL */
    double *grad_wavelet;           /* out [n_tx][nt] or NULL */
    double *misfit;                 /* out scalar or NULL */
    double *fields;                 /* out: forward fields u^1..u^T of transmit 0, [nt][nz*nx], or NULL */
    int32_t order;                  /* spatial order of L_b: 2 (default when 0) or 4 */
    int32_t pad;
    const double *eta;              /* [nz*nx] attenuation rate (1/s), or NULL (= 0) */
    double *grad_eta;               /* out [nz*nx] dJ/deta, or NULL */
} om_medium;

enum { OM_OK = 0, OM_ERR_INVALID = 1, OM_ERR_NOMEM = 4 };

/* ---------------------------------------------------------------- coefficients */

double om_dmax(double cref, double R, int N, double h)
{
    return 3.0 * cref * log(1.0 / R) / (2.0 * N * h);
}

static double om_prof(int i, int n, int N, double dmax)
{
    if (i < N) {
        double r = (double)(N - i) / N;
        return dmax * r * r;
    }
    if (i > n - 1 - N) {
        double r = (double)(i - (n - 1 - N)) / N;
        return dmax * r * r;
    }
    return 0.0;
}

/* D(ix, iz) for a whole grid, exposed for the tests. */
void om_damping(int nx, int nz, int N, double dmax, double *D)
{
    for (int iz = 0; iz < nz; ++iz)
        for (int ix = 0; ix < nx; ++ix)
            D[iz * nx + ix] = om_prof(ix, nx, N, dmax) + om_prof(iz, nz, N, dmax);
}

typedef struct {
    int nx, nz;
    int order;                      /* 2 or 4 */
    int nthr;                       /* OpenMP threads of the row loops */
    double ih2;                     /* h^-2 */
    double *a, *beta, *gam, *kap, *b, *gk;   /* gk = gamma * kappa */
    double *da, *dbeta, *dgam;      /* derivatives of a, beta, gamma with respect to e = D dt */
} om_coef;

static void coef_free(om_coef *k)
{
    free(k->a); free(k->beta); free(k->gam); free(k->kap); free(k->b); free(k->gk);
    free(k->da); free(k->dbeta); free(k->dgam);
}

static int coef_make(const om_medium *m, om_coef *k)
{
    int n = m->nx * m->nz;
    k->nx = m->nx; k->nz = m->nz;
    k->order = m->order == 4 ? 4 : 2;
    k->ih2 = 1.0 / (m->h * m->h);
    k->a = malloc(sizeof(double) * n); k->beta = malloc(sizeof(double) * n);
    k->gam = malloc(sizeof(double) * n); k->kap = malloc(sizeof(double) * n);
    k->b = malloc(sizeof(double) * n); k->gk = malloc(sizeof(double) * n);
    k->da = malloc(sizeof(double) * n); k->dbeta = malloc(sizeof(double) * n); k->dgam = malloc(sizeof(double) * n);
    if (!k->a || !k->beta || !k->gam || !k->kap || !k->b || !k->gk || !k->da || !k->dbeta || !k->dgam) {
        coef_free(k);
        return OM_ERR_NOMEM;
    }
    double dmax = om_dmax(m->pml_cref, m->pml_r, m->npml, m->h);
    double dt = m->dt;
    for (int iz = 0; iz < m->nz; ++iz)
        for (int ix = 0; ix < m->nx; ++ix) {
            int x = iz * m->nx + ix;
            double D = om_prof(ix, m->nx, m->npml, dmax) + om_prof(iz, m->nz, m->npml, dmax);
            if (m->eta) D += m->eta[x];
            double e = D * dt, den = 1.0 + e;
            k->a[x] = (2.0 - e * e) / den;
            k->beta[x] = (e - 1.0) / den;
            k->gam[x] = dt * dt / den;
            k->da[x] = -(e * e + 2.0 * e + 2.0) / (den * den);
            k->dbeta[x] = 2.0 / (den * den);
            k->dgam[x] = -dt * dt / (den * den);
            k->kap[x] = m->rho[x] * m->c[x] * m->c[x];
            k->b[x] = 1.0 / m->rho[x];
            k->gk[x] = k->gam[x] * k->kap[x];
        }
    return OM_OK;
}

/* ---------------------------------------------------------------- operator */

/* The four neighbours of cell (ix, iz): W, E, N(up), S(down); -1 = outside. */
static void neighbours(int nx, int nz, int ix, int iz, int nb[4])
{
    int x = iz * nx + ix;
    nb[0] = ix > 0 ? x - 1 : -1;
    nb[1] = ix < nx - 1 ? x + 1 : -1;
    nb[2] = iz > 0 ? x - nx : -1;
    nb[3] = iz < nz - 1 ? x + nx : -1;
}

static double face_b(const om_coef *k, int x, int xn)
{
    return xn < 0 ? k->b[x] : 0.5 * (k->b[x] + k->b[xn]);
}

/* ---- fourth order: faces along one axis of a row (axis 0) or column (axis 1) */

/* v at position i along the axis through (ix, iz); 0 outside the grid */
static double val_ax(const om_coef *k, const double *v, int ix, int iz, int axis, int i)
{
    int n = axis == 0 ? k->nx : k->nz;
    if (i < 0 || i >= n) return 0.0;
    return axis == 0 ? v[iz * k->nx + i] : v[i * k->nx + ix];
}

/* cell index of position i along the axis, clamped to the grid (b repeats outward) */
static int cell_ax(const om_coef *k, int ix, int iz, int axis, int i)
{
    int n = axis == 0 ? k->nx : k->nz;
    if (i < 0) i = 0;
    if (i > n - 1) i = n - 1;
    return axis == 0 ? iz * k->nx + i : i * k->nx + ix;
}

/* (D v) at the face between positions j and j+1 along the axis */
static double d4_face(const om_coef *k, const double *v, int ix, int iz, int axis, int j)
{
    return 9.0 / 8.0 * (val_ax(k, v, ix, iz, axis, j + 1) - val_ax(k, v, ix, iz, axis, j))
         - 1.0 / 24.0 * (val_ax(k, v, ix, iz, axis, j + 2) - val_ax(k, v, ix, iz, axis, j - 1));
}

static double b4_face(const om_coef *k, int ix, int iz, int axis, int j)
{
    return 0.5 * (k->b[cell_ax(k, ix, iz, axis, j)] + k->b[cell_ax(k, ix, iz, axis, j + 1)]);
}

/* flux b_f (D v)_f at the face between j and j+1 */
static double flux4(const om_coef *k, const double *v, int ix, int iz, int axis, int j)
{
    return b4_face(k, ix, iz, axis, j) * d4_face(k, v, ix, iz, axis, j);
}

static double lb4_at(const om_coef *k, const double *v, int ix, int iz)
{
    double s = 0.0;
    for (int axis = 0; axis < 2; ++axis) {
        int i = axis == 0 ? ix : iz;
        s += 9.0 / 8.0 * (flux4(k, v, ix, iz, axis, i) - flux4(k, v, ix, iz, axis, i - 1))
           - 1.0 / 24.0 * (flux4(k, v, ix, iz, axis, i + 1) - flux4(k, v, ix, iz, axis, i - 2));
    }
    return k->ih2 * s;
}

/* (L_b v)_x */
static double lb_at(const om_coef *k, const double *v, int ix, int iz)
{
    if (k->order == 4) return lb4_at(k, v, ix, iz);

    int nb[4], x = iz * k->nx + ix;
    neighbours(k->nx, k->nz, ix, iz, nb);
    double s = 0.0;
    for (int f = 0; f < 4; ++f) {
        double vn = nb[f] >= 0 ? v[nb[f]] : 0.0;
        s += face_b(k, x, nb[f]) * (vn - v[x]);
    }
    return k->ih2 * s;
}

/* One forward step without the source: next = a cur + beta prev + gamma kappa L_b cur. */
static void fwd_step(const om_coef *k, const double *prev, const double *cur, double *next, int par)
{
    int nx = k->nx, nz = k->nz;
#pragma omp parallel for schedule(static) if (par) num_threads(k->nthr)
    for (int iz = 0; iz < nz; ++iz)
        for (int ix = 0; ix < nx; ++ix) {
            int x = iz * nx + ix;
            next[x] = k->a[x] * cur[x] + k->beta[x] * prev[x] + k->gk[x] * lb_at(k, cur, ix, iz);
        }
}

/* One adjoint step without the receiver source:
 * out = a l1 + L_b(gamma kappa l1) + beta l2, using w = gamma kappa l1 as scratch. */
static void adj_step(const om_coef *k, const double *l2, const double *l1, double *w, double *out, int par)
{
    int nx = k->nx, nz = k->nz, n = nx * nz;
    for (int x = 0; x < n; ++x) w[x] = k->gk[x] * l1[x];
#pragma omp parallel for schedule(static) if (par) num_threads(k->nthr)
    for (int iz = 0; iz < nz; ++iz)
        for (int ix = 0; ix < nx; ++ix) {
            int x = iz * nx + ix;
            out[x] = k->a[x] * l1[x] + lb_at(k, w, ix, iz) + k->beta[x] * l2[x];
        }
}

/* Fourth-order imaging: g_kappa as below; every face of every row and column
 * (those between positions -2 .. n along the axis carry non-zero D u) gives
 * G_f = -h^-2 (D u)_f (D w)_f, half to each cell whose b enters b_f. */
static void imaging4(const om_coef *k, const double *lam, const double *u, const double *w,
                     double *gkap, double *gb)
{
    int nx = k->nx, nz = k->nz;
    for (int iz = 0; iz < nz; ++iz)
        for (int ix = 0; ix < nx; ++ix) {
            int x = iz * nx + ix;
            gkap[x] += k->gam[x] * lam[x] * lb_at(k, u, ix, iz);
        }
    for (int axis = 0; axis < 2; ++axis) {
        int nl = axis == 0 ? nz : nx;          /* lines */
        int n = axis == 0 ? nx : nz;           /* cells per line */
        for (int l = 0; l < nl; ++l) {
            int ix = axis == 0 ? 0 : l, iz = axis == 0 ? l : 0;
            for (int j = -2; j <= n; ++j) {
                double G = -k->ih2 * d4_face(k, u, ix, iz, axis, j) * d4_face(k, w, ix, iz, axis, j);
                gb[cell_ax(k, ix, iz, axis, j)] += 0.5 * G;
                gb[cell_ax(k, ix, iz, axis, j + 1)] += 0.5 * G;
            }
        }
    }
}

/* Zero-lag cross-correlation of lam^t with u^{t-1}: adds to g_kappa, g_b. */
static void imaging(const om_coef *k, const double *lam, const double *u, double *w,
                    double *gkap, double *gb, int par)
{
    int nx = k->nx, nz = k->nz, n = nx * nz;
    for (int x = 0; x < n; ++x) w[x] = k->gk[x] * lam[x];
    if (k->order == 4) { imaging4(k, lam, u, w, gkap, gb); return; }
#pragma omp parallel for schedule(static) if (par) num_threads(k->nthr)
    for (int iz = 0; iz < nz; ++iz)
        for (int ix = 0; ix < nx; ++ix) {
            int nb[4], x = iz * nx + ix;
            gkap[x] += k->gam[x] * lam[x] * lb_at(k, u, ix, iz);
            neighbours(nx, nz, ix, iz, nb);
            for (int f = 0; f < 4; ++f) {
                double du = (nb[f] >= 0 ? u[nb[f]] : 0.0) - u[x];
                double dw = (nb[f] >= 0 ? w[nb[f]] : 0.0) - w[x];
                double G = -k->ih2 * du * dw;
                gb[x] += (nb[f] >= 0 ? 0.5 : 1.0) * G;
            }
        }
}

/* Attenuation term of the gradient at one adjoint time t:
 * ge(x) += lam^t_x (a' u^{t-1} + beta' u^{t-2} + gamma' kappa L_b u^{t-1})_x, derivatives in e. */
static void att_imaging(const om_coef *k, const double *lam, const double *u1, const double *u2, double *ge)
{
    for (int iz = 0; iz < k->nz; ++iz)
        for (int ix = 0; ix < k->nx; ++ix) {
            int x = iz * k->nx + ix;
            ge[x] += lam[x] * (k->da[x] * u1[x] + k->dbeta[x] * u2[x] + k->dgam[x] * k->kap[x] * lb_at(k, u1, ix, iz));
        }
}

/* ---------------------------------------------------------------- one transmit */

typedef struct {
    const om_medium *m;
    const om_coef *k;
    int p;                          /* transmit index */
    int K;                          /* checkpoint interval; K >= nt means store-all */
    int par;                        /* parallelise rows */
    double *traces;                 /* [nt][n_rcv] for this transmit */
    double *gkap, *gb;              /* [n] per-transmit accumulators */
    double *ge;                     /* [n] dJ/de accumulator, or NULL */
    double *gw;                     /* [nt] or NULL */
    double J;
} om_tx;

static double wav(const om_medium *m, int p, int n)
{
    return m->wavelet[(int64_t)p * m->wavelet_stride + n];
}

/* Forward steps n = n0..n1-1 from (prev, cur) = (u^{n0-1}, u^{n0}); plane u^{n+1} goes to
 * store[n + 1 - n0] (store has n1 - n0 planes).  Traces sampled when smp != 0. */
static void fwd_run(om_tx *t, const double *prev, const double *cur, double *store, int n0, int n1, int smp)
{
    const om_medium *m = t->m;
    int n = m->nx * m->nz;
    for (int s = n0; s < n1; ++s) {
        /* u^{s-1} and u^s: the given pair at the segment start, else planes of the store */
        const double *pp, *cc;
        if (s == n0) { pp = prev; cc = cur; }
        else if (s == n0 + 1) { pp = cur; cc = store; }
        else { pp = store + (size_t)(s - n0 - 2) * n; cc = store + (size_t)(s - n0 - 1) * n; }
        double *nx_ = store + (size_t)(s - n0) * n;
        fwd_step(t->k, pp, cc, nx_, t->par);
        nx_[m->src[t->p]] += wav(m, t->p, s);
        if (smp)
            for (int r = 0; r < m->n_rcv; ++r)
                t->traces[(size_t)s * m->n_rcv + r] = nx_[m->rcv[(size_t)t->p * m->n_rcv + r]];
    }
}

static int run_transmit(om_tx *t)
{
    const om_medium *m = t->m;
    const om_coef *k = t->k;
    int n = m->nx * m->nz, T = m->nt, nr = m->n_rcv;
    int K = t->K < 1 ? 1 : t->K;
    if (K > T) K = T;
    int want_adj = (m->d_obs || m->d_adj) &&
                   (m->grad_c || m->grad_rho || m->grad_kappa || m->grad_b || m->grad_wavelet || m->grad_eta);
    if (!want_adj && m->fields) K = T;             /* keep every plane to hand them out */
    int J = (T + K - 1) / K;                       /* segments */

    /* forward only: no replay, so segments of two planes and one checkpoint slot */
    if (!want_adj && T >= 2) { K = 2; J = (T + K - 1) / K; }
    int nck = want_adj ? J : 2;                                    /* checkpoint slots kept */
    double *zero = calloc((size_t)n, sizeof(double));
    double *seg = malloc(sizeof(double) * (size_t)n * K);          /* u^{jK+1..jK+K} */
    double *ck = calloc((size_t)2 * nck * n, sizeof(double));      /* (u^{jK-1}, u^{jK}) */
    if (!zero || !seg || !ck) { free(zero); free(seg); free(ck); return OM_ERR_NOMEM; }

    /* ---- forward, segment by segment, keeping checkpoint pairs */
    for (int j = 0; j < J; ++j) {
        int n0 = j * K, n1 = n0 + K < T ? n0 + K : T;
        double *cp = ck + (size_t)2 * (j % nck) * n;    /* prev, cur */
        if (j > 0) {
            /* the checkpoint pair of segment j is the last two planes of segment j-1 */
            memcpy(cp + n, seg + (size_t)(K - 1) * n, sizeof(double) * n);
            memcpy(cp, K >= 2 ? seg + (size_t)(K - 2) * n : ck + (size_t)(2 * ((j - 1) % nck) + 1) * n,
                   sizeof(double) * n);
        }
        fwd_run(t, cp, cp + n, seg, n0, n1, 1);
        if (m->fields && t->p == 0)
            memcpy(m->fields + (size_t)n0 * n, seg, sizeof(double) * (size_t)(n1 - n0) * n);
    }

    /* ---- misfit */
    double Jm = 0.0;
    if (m->d_obs) {
        const double *dob = m->d_obs + (size_t)t->p * T * nr;
        for (size_t i = 0; i < (size_t)T * nr; ++i) {
            double r = t->traces[i] - dob[i];
            Jm += r * r;
        }
    }
    t->J = Jm;

    if (want_adj) {
        double *l1 = calloc((size_t)n, sizeof(double));   /* lam^{t+1} */
        double *l2 = calloc((size_t)n, sizeof(double));   /* lam^{t+2} */
        double *l0 = calloc((size_t)n, sizeof(double));   /* lam^t */
        double *w = malloc(sizeof(double) * n);
        if (!l1 || !l2 || !l0 || !w) { free(l1); free(l2); free(l0); free(w); free(zero); free(seg); free(ck); return OM_ERR_NOMEM; }
        const double *dob = m->d_obs ? m->d_obs + (size_t)t->p * T * nr : NULL;
        const double *dad = m->d_adj ? m->d_adj + (size_t)t->p * T * nr : NULL;
        const int32_t *rc = m->rcv + (size_t)t->p * nr;
        for (int j = J - 1; j >= 0; --j) {
            int n0 = j * K, n1 = n0 + K < T ? n0 + K : T;
            if (j < J - 1) {   /* recompute segment j from its checkpoint pair */
                double *cp = ck + (size_t)2 * j * n;
                fwd_run(t, cp, cp + n, seg, n0, n1, 0);
            }
            /* adjoint times t = n1 .. n0+1 use u^{t-1}; u^{n0} is the checkpoint plane */
            for (int tt = n1; tt >= n0 + 1; --tt) {
                adj_step(k, l2, l1, w, l0, t->par);
                for (int r = 0; r < nr; ++r) {
                    double s;
                    if (dad) s = dad[(size_t)(tt - 1) * nr + r];
                    else s = 2.0 * (t->traces[(size_t)(tt - 1) * nr + r] - dob[(size_t)(tt - 1) * nr + r]);
                    l0[rc[r]] += s;
                }
                if (t->gw) t->gw[tt - 1] = l0[m->src[t->p]];
                const double *um1 = (tt - 1 == 0) ? zero
                                   : (tt - 1 == n0) ? ck + (size_t)(2 * j + 1) * n
                                   : seg + (size_t)(tt - 2 - n0) * n;
                imaging(k, l0, um1, w, t->gkap, t->gb, t->par);
                if (t->ge) {
                    /* u^{t-2}: checkpoint pair (u^{n0-1}, u^{n0}) at the segment start, zero before u^1 */
                    const double *um2 = (tt - 2 <= 0) ? zero
                                       : (tt - 2 == n0) ? ck + (size_t)(2 * j + 1) * n
                                       : (tt - 2 == n0 - 1) ? ck + (size_t)(2 * j) * n
                                       : seg + (size_t)(tt - 3 - n0) * n;
                    att_imaging(k, l0, um1, um2, t->ge);
                }
                double *tmp = l2; l2 = l1; l1 = l0; l0 = tmp;
            }
        }
        free(l1); free(l2); free(l0); free(w);
    }
    free(zero); free(seg); free(ck);
    return OM_OK;
}

/* ---------------------------------------------------------------- driver */

static int valid(const om_medium *m)
{
    if (!m || m->nx < 1 || m->nz < 1 || m->nt < 1 || m->npml < 0 || m->n_tx < 1 || m->n_rcv < 0) return 0;
    if (!(m->h > 0) || !(m->dt > 0) || !m->c || !m->rho || !m->src || !m->wavelet) return 0;
    if (m->n_rcv > 0 && !m->rcv) return 0;
    if (m->wavelet_stride != 0 && m->wavelet_stride < m->nt) return 0;
    if (m->order != 0 && m->order != 2 && m->order != 4) return 0;
    int n = m->nx * m->nz;
    if (m->eta)
        for (int x = 0; x < n; ++x)
            if (!(m->eta[x] >= 0.0) || !isfinite(m->eta[x])) return 0;
    for (int p = 0; p < m->n_tx; ++p) {
        if (m->src[p] < 0 || m->src[p] >= n) return 0;
        for (int r = 0; r < m->n_rcv; ++r)
            if (m->rcv[(size_t)p * m->n_rcv + r] < 0 || m->rcv[(size_t)p * m->n_rcv + r] >= n) return 0;
    }
    return 1;
}

/* Forward (+ misfit + adjoint gradient when d_obs or d_adj is given).
 * ckpt: checkpoint interval K (0 or >= nt: store-all).  threads: OpenMP threads (<=0: default). */
int om_run(om_medium *m, int ckpt, int threads)
{
    if (!valid(m)) return OM_ERR_INVALID;
    int n = m->nx * m->nz, T = m->nt, nr = m->n_rcv, P = m->n_tx;
    int K = (ckpt <= 0 || ckpt > T) ? T : ckpt;
#ifdef _OPENMP
    int nthr = threads > 0 ? threads : omp_get_num_procs();
    if ((int64_t)n * P < 16384) nthr = 1;          /* tiny grids: threads cost more than they save */
#else
    int nthr = 1;
#endif
    om_coef k;
    if (coef_make(m, &k) != OM_OK) return OM_ERR_NOMEM;
    k.nthr = nthr;

    double *tr = m->traces ? m->traces : malloc(sizeof(double) * (size_t)P * T * (nr > 0 ? nr : 1));
    double *gk = calloc((size_t)P * n, sizeof(double));
    double *gb = calloc((size_t)P * n, sizeof(double));
    double *Jp = calloc((size_t)P, sizeof(double));
    double *ge = m->grad_eta ? calloc((size_t)P * n, sizeof(double)) : NULL;
    if (!tr || !gk || !gb || !Jp || (m->grad_eta && !ge)) {
        coef_free(&k); free(gk); free(gb); free(Jp); free(ge); if (!m->traces) free(tr);
        return OM_ERR_NOMEM;
    }

    int over_tx = P >= nthr && nthr > 1;
    int rc = OM_OK;
#pragma omp parallel for schedule(dynamic, 1) if (over_tx) reduction(max : rc) num_threads(nthr)
    for (int p = 0; p < P; ++p) {
        om_tx t;
        t.J = 0.0;
        t.m = m; t.k = &k; t.p = p; t.K = K; t.par = !over_tx;
        t.traces = tr + (size_t)p * T * nr;
        t.gkap = gk + (size_t)p * n; t.gb = gb + (size_t)p * n;
        t.ge = ge ? ge + (size_t)p * n : NULL;
        t.gw = m->grad_wavelet ? m->grad_wavelet + (size_t)p * T : NULL;
        int r = run_transmit(&t);
        Jp[p] = t.J;
        if (r > rc) rc = r;
    }

    if (rc == OM_OK) {
        /* sum over transmits in transmit order */
        double Jsum = 0.0;
        for (int p = 0; p < P; ++p) Jsum += Jp[p];
        if (m->misfit) *m->misfit = Jsum;
        for (int x = 0; x < n; ++x) {
            double sk = 0.0, sb = 0.0;
            for (int p = 0; p < P; ++p) { sk += gk[(size_t)p * n + x]; sb += gb[(size_t)p * n + x]; }
            double c = m->c[x], rho = m->rho[x], b = 1.0 / rho;
            if (m->grad_kappa) m->grad_kappa[x] = sk;
            if (m->grad_b) m->grad_b[x] = sb;
            if (m->grad_c) m->grad_c[x] = 2.0 * rho * c * sk;
            if (m->grad_rho) m->grad_rho[x] = c * c * sk - b * b * sb;
            if (m->grad_eta) {
                double se = 0.0;
                for (int p = 0; p < P; ++p) se += ge[(size_t)p * n + x];
                m->grad_eta[x] = m->dt * se;
            }
        }
    }
    coef_free(&k);
    free(gk); free(gb); free(Jp); free(ge);
    if (!m->traces) free(tr);
    return rc;
}

/* Tangent-linear (Born) traces for a perturbation (dc, drho), test-only:
 *   du^{n+1} = a du^n + beta du^{n-1} + gamma kappa L_b du^n
 *            + gamma dkappa L_b u^n + gamma kappa L_db u^n,
 *   dkappa = 2 rho c dc + c^2 drho, db = -drho / rho^2, db_f averaged like b_f;
 *   with deta (may be NULL) also + de (a' u^n + beta' u^{n-1} + gamma' kappa L_b u^n),
 *   de = deta dt;
 *   dd_p[n][r] = du^{n+1}[rcv_{p,r}]. */
int om_born(om_medium *m, const double *dc, const double *drho, const double *deta, double *dtraces)
{
    if (!valid(m) || !dc || !drho || !dtraces) return OM_ERR_INVALID;
    int nx = m->nx, nz = m->nz, n = nx * nz, T = m->nt, nr = m->n_rcv;
    om_coef k;
    if (coef_make(m, &k) != OM_OK) return OM_ERR_NOMEM;
    k.nthr = 1;
    om_coef kd = k;                                /* perturbation operator: b -> db */
    double *dkap = malloc(sizeof(double) * n), *db = malloc(sizeof(double) * n);
    double *u[3], *du[3];
    for (int i = 0; i < 3; ++i) { u[i] = calloc(n, sizeof(double)); du[i] = calloc(n, sizeof(double)); }
    for (int x = 0; x < n; ++x) {
        dkap[x] = 2.0 * m->rho[x] * m->c[x] * dc[x] + m->c[x] * m->c[x] * drho[x];
        db[x] = -drho[x] / (m->rho[x] * m->rho[x]);
    }
    kd.b = db;
    for (int p = 0; p < m->n_tx; ++p) {
        for (int i = 0; i < 3; ++i) { memset(u[i], 0, sizeof(double) * n); memset(du[i], 0, sizeof(double) * n); }
        double *up = u[0], *uc = u[1], *un = u[2], *dp = du[0], *dcu = du[1], *dn = du[2];
        for (int s = 0; s < T; ++s) {
            for (int iz = 0; iz < nz; ++iz)
                for (int ix = 0; ix < nx; ++ix) {
                    int x = iz * nx + ix;
                    dn[x] = k.a[x] * dcu[x] + k.beta[x] * dp[x] + k.gk[x] * lb_at(&k, dcu, ix, iz)
                          + k.gam[x] * dkap[x] * lb_at(&k, uc, ix, iz)
                          + k.gk[x] * lb_at(&kd, uc, ix, iz);
                    if (deta) {
                        double de = deta[x] * m->dt;   /* perturbation of e = (D + eta) dt */
                        dn[x] += de * (k.da[x] * uc[x] + k.dbeta[x] * up[x] + k.dgam[x] * k.kap[x] * lb_at(&k, uc, ix, iz));
                    }
                }
            fwd_step(&k, up, uc, un, 0);
            un[m->src[p]] += wav(m, p, s);
            for (int r = 0; r < nr; ++r)
                dtraces[((size_t)p * T + s) * nr + r] = dn[m->rcv[(size_t)p * nr + r]];
            double *t1 = up; up = uc; uc = un; un = t1;
            double *t2 = dp; dp = dcu; dcu = dn; dn = t2;
        }
    }
    for (int i = 0; i < 3; ++i) { free(u[i]); free(du[i]); }
    free(dkap); free(db);
    coef_free(&k);
    return OM_OK;
}

/* out = L_b v on the grid of m (test-only: the operator's order of accuracy). */
int om_apply_lb(const om_medium *m, const double *v, double *out)
{
    if (!m || m->nx < 1 || m->nz < 1 || !m->rho || !m->c || !v || !out) return OM_ERR_INVALID;
    om_coef k;
    if (coef_make(m, &k) != OM_OK) return OM_ERR_NOMEM;
    for (int iz = 0; iz < m->nz; ++iz)
        for (int ix = 0; ix < m->nx; ++ix) out[iz * m->nx + ix] = lb_at(&k, v, ix, iz);
    coef_free(&k);
    return OM_OK;
}

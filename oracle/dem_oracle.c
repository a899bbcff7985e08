/*
 * FP64 ORACLE of the superparameterised floe DEM (Deng, Stechmann & Chen,
 * "Particle-continuum multiscale modeling of sea ice floes").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP implementation.
 *
 * Plain, slow and written to be checked against the paper by eye:
 *   - state in FP64; positions as cell fractions xs, ys in [0, 1) of a doubly
 *     periodic cell (Sec. 3.1: one DEM per coarse cell, periodic in both
 *     directions);
 *   - one fine step follows the DEM system eq:dem (Sec. 2.1): ocean drag and
 *     drag torque, contact forces and torques from the contact law of Sec. 2.1,
 *     then the time update;
 *   - the per-cell statistics feed the moment equations eq:pde (Sec. 2.3),
 *     advanced by Lax-Friedrichs with the Oseen treatment of the momentum
 *     advection (Sec. 3.2);
 *   - the coarse-to-fine re-synchronisation follows the proportional updates of
 *     Sec. 3.3, applied in one go.
 *
 * Readings where the paper is silent or ambiguous (each is listed, with its
 * reason, in the design notes of the repository):
 *   mass m = rho_ice h pi r^2 (thickness h; the paper assumes h = 1);
 *   I = m r^2 as printed; alpha = Cd rho_o pi r^2; beta = Cd rho_o pi r^5
 *   (one more power of r than printed, so that beta (..)|..| is a torque);
 *   n points from floe l to floe j; r^l = +r_l n, r^j = -r_j n, hence
 *   v_t = (v_j - v_l).t - w_j r_j - w_l r_l and the spin torque on l is r_l F_t;
 *   chord c = common chord of the two overlapping disks (2 min(r) when one
 *   contains the other); contact iff d < r_l + r_j, decided by one fixed FP64
 *   expression (see contact_pred); minimum image in [-L/2, L/2);
 *   time update: velocities first, then positions with the new velocities
 *   (semi-implicit Euler; the literal forward Euler is a flag).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OCEAN_OFF 1
#define ORC_FORWARD_EULER 2
#define ORC_BINNED 4
#define ORC_TSPRING 8   /* tangential force as an incremental spring with contact history */
#define ORC_WALLS_X 16  /* fixed walls at x = 0 and x = Lx (the DEM is periodic in y only) */
#define ORC_DIRICHLET_X 32  /* continuum: zero state beyond the x edges (Sec. 4.4) */
#define ORC_HCAP 16     /* contacts remembered per floe */

#define NMOM 11
enum { M_N = 0, M_MASS, M_PX, M_PY, M_L, M_UX, M_UY, M_SVX, M_SVY, M_SW, M_AICE };

typedef struct {
    int32_t nx, ny;
    double Lx, Ly;
    double rho_ice, rho_ocean, cd, E, G, mu;
    int32_t flags;
    double u0, v0;
    int32_t nmodes;
    const double *kx, *ky, *au, *av, *phase;
} orc_model;

static const double PI = 3.14159265358979323846;

/* ---------------------------------------------------------------- ocean --- */
/* Prescribed surface current u_o (Sec. 2.1: "assumed to be known") and its
 * curl zeta = dv_o/dX - du_o/dY, evaluated at a global position. */
void orc_ocean_at(const orc_model* m, double X, double Y, double out[3])
{
    double uo = m->u0, vo = m->v0, z = 0.0;
    for (int k = 0; k < m->nmodes; ++k) {
        double th = m->kx[k] * X + m->ky[k] * Y + m->phase[k];
        double s = sin(th), c = cos(th);
        uo += m->au[k] * s;
        vo += m->av[k] * s;
        z += (m->av[k] * m->kx[k] - m->au[k] * m->ky[k]) * c;
    }
    out[0] = uo;
    out[1] = vo;
    out[2] = z;
}

/* --------------------------------------------------------- contact test --- */
static double min_image(double d)
{
    /* fractional difference mapped to [-1/2, 1/2) */
    if (d >= 0.5) d -= 1.0;
    else if (d < -0.5) d += 1.0;
    return d;
}

/* Contact iff |x_j - x_l| < r_l + r_j, as the FP64 expression
 * (dx*dx + dy*dy) < R*R with dx = min_image(xs_j - xs_l) * Lx and
 * R = r_l + r_j, evaluated left to right without fused multiply-add. */
static int contact_pred(const orc_model* m, double xl, double yl, double rl,
                        double xj, double yj, double rj)
{
    /* between walls the x difference is the plain one (no periodic image) */
    double dx = ((m->flags & ORC_WALLS_X) ? xj - xl : min_image(xj - xl)) * m->Lx;
    double dy = min_image(yj - yl) * m->Ly;
    double R = rl + rj;
    double d2 = dx * dx + dy * dy;
    return d2 < R * R;
}

static int cmp_pair(const void* a, const void* b)
{
    const int32_t* p = (const int32_t*)a;
    const int32_t* q = (const int32_t*)b;
    if (p[0] != q[0]) return (p[0] > q[0]) - (p[0] < q[0]);
    return (p[1] > q[1]) - (p[1] < q[1]);
}

/* All unordered contact pairs (l < j) of one cell by brute force; returns the
 * count and writes at most cap pairs, sorted. */
int64_t orc_pairs_brute(const orc_model* m, int64_t n, const double* xs, const double* ys,
                        const double* r, int64_t cap, int32_t* pl, int32_t* pj)
{
    int64_t cnt = 0;
    for (int64_t l = 0; l < n; ++l)
        for (int64_t j = l + 1; j < n; ++j)
            if (contact_pred(m, xs[l], ys[l], r[l], xs[j], ys[j], r[j])) {
                if (cnt < cap) {
                    pl[cnt] = (int32_t)l;
                    pj[cnt] = (int32_t)j;
                }
                ++cnt;
            }
    return cnt;
}

/* The same set through square sub-bins of side >= 2 r_max with a 3x3 periodic
 * sweep (any contact partner lies in a neighbouring bin). */
int64_t orc_pairs_binned(const orc_model* m, int64_t n, const double* xs, const double* ys,
                         const double* r, int64_t cap, int32_t* pl, int32_t* pj)
{
    if (n < 2) return 0;
    double rmax = 0.0;
    for (int64_t l = 0; l < n; ++l)
        if (r[l] > rmax) rmax = r[l];
    int nbx = (int)floor(m->Lx / (2.0 * rmax));
    int nby = (int)floor(m->Ly / (2.0 * rmax));
    if (nbx < 3) nbx = 1;
    if (nby < 3) nby = 1;
    int nb = nbx * nby;
    int32_t* head = (int32_t*)malloc(sizeof(int32_t) * (size_t)nb);
    int32_t* next = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    int32_t* bin = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    for (int b = 0; b < nb; ++b) head[b] = -1;
    for (int64_t l = n - 1; l >= 0; --l) {
        int bx = (int)floor(xs[l] * nbx), by = (int)floor(ys[l] * nby);
        if (bx >= nbx) bx = nbx - 1;
        if (by >= nby) by = nby - 1;
        bin[l] = by * nbx + bx;
        next[l] = head[bin[l]];
        head[bin[l]] = (int32_t)l;
    }
    int64_t tot = 0;
    int32_t(*buf)[2] = NULL;
    int64_t bcap = 0;
    for (int64_t l = 0; l < n; ++l) {
        int bx = bin[l] % nbx, by = bin[l] / nbx;
        int ox0 = nbx >= 3 ? -1 : 0, ox1 = nbx >= 3 ? 1 : 0;
        int oy0 = nby >= 3 ? -1 : 0, oy1 = nby >= 3 ? 1 : 0;
        for (int oy = oy0; oy <= oy1; ++oy)
            for (int ox = ox0; ox <= ox1; ++ox) {
                int b = ((by + oy + nby) % nby) * nbx + (bx + ox + nbx) % nbx;
                for (int32_t j = head[b]; j >= 0; j = next[j]) {
                    if (j <= l) continue;
                    if (!contact_pred(m, xs[l], ys[l], r[l], xs[j], ys[j], r[j])) continue;
                    if (tot == bcap) {
                        bcap = bcap ? 2 * bcap : 64;
                        buf = realloc(buf, sizeof(*buf) * (size_t)bcap);
                    }
                    buf[tot][0] = (int32_t)l;
                    buf[tot][1] = j;
                    ++tot;
                }
            }
    }
    if (tot) qsort(buf, (size_t)tot, sizeof(*buf), cmp_pair);
    for (int64_t k = 0; k < tot && k < cap; ++k) {
        pl[k] = buf[k][0];
        pj[k] = buf[k][1];
    }
    free(buf);
    free(head);
    free(next);
    free(bin);
    return tot;
}

/* ------------------------------------------------------- contact force --- */
/* Common chord of two overlapping disks at centre distance d. */
double orc_chord(double rl, double rj, double d)
{
    if (d <= fabs(rl - rj)) return 2.0 * (rl < rj ? rl : rj);
    double p = (-d + rl + rj) * (d - rl + rj) * (d + rl - rj) * (d + rl + rj);
    if (p < 0.0) p = 0.0;
    return sqrt(p) / d;
}

/* Force f^{lj} on floe l from floe j and the spin torque on l (contact law of
 * Sec. 2.1): f_n = c E delta n, f_t = c G v_t t with |f_t| <= mu |f_n|.
 * With ORC_TSPRING the tangential force is the incremental spring that the
 * cited Cundall-Strack model uses instead: the pair's tangential displacement
 * xi (zero when the contact begins) grows by v_t dt each step, f_t = c G xi t
 * with G a shear modulus, and where |f_t| would pass mu |f_n| the contact
 * slips: f_t takes the Coulomb limit and xi the displacement that gives it.
 * xi_old is the pair's displacement after the previous step (0 for a new
 * contact); *xi receives the new one.  Returns 0, or -1 if the centres
 * coincide. */
static int contact_force(const orc_model* m, const double* xs, const double* ys, const double* u,
                         const double* v, const double* w, const double* r, int64_t l, int64_t j,
                         double dt, double xi_old, double* xi, double* fx, double* fy, double* tq)
{
    double dx = ((m->flags & ORC_WALLS_X) ? xs[j] - xs[l] : min_image(xs[j] - xs[l])) * m->Lx;
    double dy = min_image(ys[j] - ys[l]) * m->Ly;
    double d = sqrt(dx * dx + dy * dy);
    if (!(d > 0.0)) return -1;
    double nx = dx / d, ny = dy / d;       /* normal, from l towards j */
    double tx = -ny, ty = nx;              /* tangent, n x t = +z     */
    double delta = d - (r[l] + r[j]);      /* < 0 in contact          */
    double c = orc_chord(r[l], r[j], d);
    double Fn = c * m->E * delta;
    /* relative tangential velocity of the contact point of j seen from l */
    double vt = (u[j] - u[l]) * tx + (v[j] - v[l]) * ty - w[j] * r[j] - w[l] * r[l];
    double cap = m->mu * fabs(Fn);
    double Ft;
    if (m->flags & ORC_TSPRING) {
        double k = c * m->G;               /* tangential stiffness of the contact */
        double x = xi_old + vt * dt;
        Ft = k * x;
        if (Ft > cap || Ft < -cap) {       /* slip: the spring stretches no further */
            Ft = Ft > cap ? cap : -cap;
            x = k > 0.0 ? Ft / k : 0.0;
        }
        *xi = x;
    } else {
        Ft = c * m->G * vt;
        if (Ft > cap) Ft = cap;
        if (Ft < -cap) Ft = -cap;
        *xi = 0.0;
    }
    *fx = Fn * nx + Ft * tx;
    *fy = Fn * ny + Ft * ty;
    *tq = r[l] * Ft;
    return 0;
}

/* Contact of floe l with a fixed straight wall at distance d from its centre
 * (the contact law of Sec. 2.1 with the wall as the other body: it does not
 * move or spin).  nsx = +1 for a wall on the floe's +x side, -1 for -x; the
 * normal n = (nsx, 0) points from the floe to the wall, t = (-n_y, n_x) =
 * (0, nsx).  In contact iff d < r: overlap delta = d - r, contact chord
 * c = 2 sqrt(r^2 - d^2) (the chord the wall line cuts from the disk: the
 * common chord of two disks as the other radius grows without bound),
 * f_n = c E delta n, v_t = -(v_l . t) - w_l r_l, f_t = c G v_t t capped at
 * mu |f_n|; the spin torque on the floe is r_l f_t.  Returns 1 in contact. */
static int wall_force(const orc_model* m, double d, double nsx, double u, double v, double w, double r,
                      double* fx, double* fy, double* tq)
{
    if (!(d < r)) return 0;
    double delta = d - r;
    double c = 2.0 * sqrt(r * r - d * d);
    double Fn = c * m->E * delta;
    double tx = 0.0, ty = nsx;
    double vt = -(u * tx + v * ty) - w * r;
    double cap = m->mu * fabs(Fn);
    double Ft = c * m->G * vt;
    if (Ft > cap) Ft = cap;
    if (Ft < -cap) Ft = -cap;
    *fx = Fn * nsx + Ft * tx;
    *fy = Ft * ty;
    *tq = r * Ft;
    return 1;
}

/* ---------------------------------------------------- compensated sums --- */
typedef struct { double s, c; } nsum;
static void nadd(nsum* a, double x)
{
    /* Neumaier's improved Kahan-Babuska summation */
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nval(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------- per-floe terms --- */
typedef struct {
    double m, I, Fdx, Fdy, Td;
} floe_terms;

static floe_terms drag_terms(const orc_model* m, int ix, int iy, double xs, double ys, double u,
                             double v, double w, double r, double h)
{
    floe_terms t;
    t.m = m->rho_ice * h * PI * r * r;
    t.I = t.m * r * r;
    t.Fdx = t.Fdy = t.Td = 0.0;
    if (m->flags & ORC_OCEAN_OFF) return t;
    double oc[3];
    orc_ocean_at(m, ((double)ix + xs) * m->Lx, ((double)iy + ys) * m->Ly, oc);
    double du = oc[0] - u, dv = oc[1] - v;
    double sp = sqrt(du * du + dv * dv);
    double alpha = m->cd * m->rho_ocean * PI * r * r;
    t.Fdx = alpha * du * sp;
    t.Fdy = alpha * dv * sp;
    double dW = 0.5 * oc[2] - w;
    double beta = m->cd * m->rho_ocean * PI * r * r * r * r * r;
    t.Td = beta * dW * fabs(dW);
    return t;
}

/* Cell statistics (Sec. 3.2, with the averages of eq:meang): n, M = sum m,
 * P = sum m v, L = sum I w, U = sum v, S_v = sum of drag forces,
 * S_w = sum of drag torques, A_ice = sum pi r^2. */
static void cell_moments(const orc_model* m, int ix, int iy, int64_t n, const double* xs,
                         const double* ys, const double* u, const double* v, const double* w,
                         const double* r, const double* h, double* out)
{
    nsum acc[NMOM];
    memset(acc, 0, sizeof(acc));
    for (int64_t l = 0; l < n; ++l) {
        floe_terms t = drag_terms(m, ix, iy, xs[l], ys[l], u[l], v[l], w[l], r[l], h[l]);
        nadd(&acc[M_N], 1.0);
        nadd(&acc[M_MASS], t.m);
        nadd(&acc[M_PX], t.m * u[l]);
        nadd(&acc[M_PY], t.m * v[l]);
        nadd(&acc[M_L], t.I * w[l]);
        nadd(&acc[M_UX], u[l]);
        nadd(&acc[M_UY], v[l]);
        nadd(&acc[M_SVX], t.Fdx);
        nadd(&acc[M_SVY], t.Fdy);
        nadd(&acc[M_SW], t.Td);
        nadd(&acc[M_AICE], PI * r[l] * r[l]);
    }
    for (int k = 0; k < NMOM; ++k) out[k] = nval(&acc[k]);
}

void orc_moments(const orc_model* m, const int64_t* start, const double* xs, const double* ys,
                 const double* u, const double* v, const double* w, const double* r,
                 const double* h, double* out)
{
    int32_t nc = m->nx * m->ny;
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t c = 0; c < nc; ++c) {
        int64_t s = start[c];
        cell_moments(m, c % m->nx, c / m->nx, start[c + 1] - s, xs + s, ys + s, u + s, v + s,
                     w + s, r + s, h + s, out + (size_t)c * NMOM);
    }
}

static double wrap01(double x)
{
    double y = x - floor(x);
    return y >= 1.0 ? 0.0 : y;
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t p = *(const int32_t*)a, q = *(const int32_t*)b;
    return (p > q) - (p < q);
}

/* One fine step of one cell.  Returns 0, -1 (coincident centres), -2 (NaN) or
 * -3 (a floe in more than ORC_HCAP contacts with ORC_TSPRING).
 * mom (may be NULL) receives the statistics of the state before the step.
 * stats[0] += contacts, stats[1] += candidate pairs considered.
 * hj, hx (ORC_TSPRING only): each floe's contact history, ORC_HCAP partner
 * indices (-1: none) and their tangential displacements; a floe's entries are
 * replaced by its contacts of this step, so a contact that ends is forgotten. */
static int cell_step(const orc_model* m, int ix, int iy, int64_t n, double* xs, double* ys,
                     double* u, double* v, double* w, double* th, const double* r,
                     const double* h, double dt, double* mom, int64_t* stats, int32_t* hj,
                     double* hx)
{
    const int spring = (m->flags & ORC_TSPRING) != 0;
    int64_t nwall = 0;   /* floe-wall contacts of this step */
    if (spring && (m->flags & ORC_WALLS_X)) return -6;
    if (n == 0) {
        if (mom) memset(mom, 0, sizeof(double) * NMOM);
        return 0;
    }
    if (mom) cell_moments(m, ix, iy, n, xs, ys, u, v, w, r, h, mom);

    /* contact pairs at the current state */
    int64_t cap = 16 * n + 64;
    int32_t* pl = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    int32_t* pj = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
    int64_t np;
    for (;;) {
        np = (m->flags & ORC_BINNED) ? orc_pairs_binned(m, n, xs, ys, r, cap, pl, pj)
                                     : orc_pairs_brute(m, n, xs, ys, r, cap, pl, pj);
        if (np <= cap) break;
        cap = np;
        pl = realloc(pl, sizeof(int32_t) * (size_t)cap);
        pj = realloc(pj, sizeof(int32_t) * (size_t)cap);
    }
    if (stats) {
        stats[0] += np;
        stats[1] += n * (n - 1) / 2;
    }
    /* partner lists of every floe, ascending */
    int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t k = 0; k < np; ++k) {
        deg[pl[k] + 1]++;
        deg[pj[k] + 1]++;
    }
    for (int64_t l = 0; l < n; ++l) deg[l + 1] += deg[l];
    int32_t* adj = (int32_t*)malloc(sizeof(int32_t) * (size_t)(2 * np + 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t l = 0; l < n; ++l) fill[l] = deg[l];
    for (int64_t k = 0; k < np; ++k) {
        adj[fill[pl[k]]++] = pj[k];
        adj[fill[pj[k]]++] = pl[k];
    }
    for (int64_t l = 0; l < n; ++l)
        qsort(adj + deg[l], (size_t)(deg[l + 1] - deg[l]), sizeof(int32_t), cmp_i32);

    /* right-hand sides of eq:dem at the current state */
    double* ax = (double*)malloc(sizeof(double) * (size_t)n);
    double* ay = (double*)malloc(sizeof(double) * (size_t)n);
    double* aw = (double*)malloc(sizeof(double) * (size_t)n);
    int rc = 0;
    for (int64_t l = 0; l < n && !rc; ++l) {
        floe_terms t = drag_terms(m, ix, iy, xs[l], ys[l], u[l], v[l], w[l], r[l], h[l]);
        double Fx = t.Fdx, Fy = t.Fdy, T = t.Td;
        int32_t nj[ORC_HCAP];
        double nxi[ORC_HCAP];
        int nh = 0;
        for (int64_t k = deg[l]; k < deg[l + 1]; ++k) {
            double fx, fy, tq, xi, xi_old = 0.0;
            if (spring)
                for (int q = 0; q < ORC_HCAP; ++q)
                    if (hj[l * ORC_HCAP + q] == adj[k]) xi_old = hx[l * ORC_HCAP + q];
            if (contact_force(m, xs, ys, u, v, w, r, l, adj[k], dt, xi_old, &xi, &fx, &fy, &tq)) {
                rc = -1;
                break;
            }
            if (spring) {
                if (nh == ORC_HCAP) {
                    rc = -3;
                    break;
                }
                nj[nh] = adj[k];
                nxi[nh++] = xi;
            }
            Fx += fx;
            Fy += fy;
            T += tq;
        }
        if ((m->flags & ORC_WALLS_X) && !rc) {
            /* the walls at x = 0 and x = Lx, after the floe contacts */
            double fx, fy, tq;
            double dl = xs[l] * m->Lx, dr = (1.0 - xs[l]) * m->Lx;
            if (wall_force(m, dl, -1.0, u[l], v[l], w[l], r[l], &fx, &fy, &tq)) {
                Fx += fx;
                Fy += fy;
                T += tq;
                if (stats) nwall++;
            }
            if (wall_force(m, dr, 1.0, u[l], v[l], w[l], r[l], &fx, &fy, &tq)) {
                Fx += fx;
                Fy += fy;
                T += tq;
                if (stats) nwall++;
            }
        }
        if (spring && !rc)
            for (int q = 0; q < ORC_HCAP; ++q) {
                hj[l * ORC_HCAP + q] = q < nh ? nj[q] : -1;
                hx[l * ORC_HCAP + q] = q < nh ? nxi[q] : 0.0;
            }
        ax[l] = Fx / t.m;
        ay[l] = Fy / t.m;
        aw[l] = T / t.I;
    }
    /* time update */
    for (int64_t l = 0; l < n && !rc; ++l) {
        double u_old = u[l], v_old = v[l], w_old = w[l];
        u[l] += dt * ax[l];
        v[l] += dt * ay[l];
        w[l] += dt * aw[l];
        int fe = (m->flags & ORC_FORWARD_EULER) != 0;
        double uu = fe ? u_old : u[l], vv = fe ? v_old : v[l], ww = fe ? w_old : w[l];
        if (m->flags & ORC_WALLS_X) {
            xs[l] = xs[l] + dt * uu / m->Lx;     /* no periodic wrap between walls */
            if (!(xs[l] >= 0.0 && xs[l] < 1.0)) rc = -5;
        } else {
            xs[l] = wrap01(xs[l] + dt * uu / m->Lx);
        }
        ys[l] = wrap01(ys[l] + dt * vv / m->Ly);
        th[l] += dt * ww;
        if (!isfinite(u[l]) || !isfinite(v[l]) || !isfinite(w[l])) rc = -2;
    }
    if (stats) stats[0] += nwall;
    free(ax);
    free(ay);
    free(aw);
    free(adj);
    free(fill);
    free(deg);
    free(pl);
    free(pj);
    return rc;
}

/* nsteps fine steps of the listed cells (all cells if cells == NULL).
 * mom (may be NULL): [nsteps][ncl][NMOM], statistics of each pre-step state.
 * hj, hx: contact histories [N][ORC_HCAP] (ORC_TSPRING only, else NULL). */
int orc_dem_steps(const orc_model* m, const int64_t* start, const int32_t* cells, int32_t ncl,
                  double* xs, double* ys, double* u, double* v, double* w, double* th,
                  const double* r, const double* h, double dt, int64_t nsteps, double* mom,
                  int64_t* stats, int32_t* hj, double* hx)
{
    int32_t nc = cells ? ncl : m->nx * m->ny;
    int rc = 0;
    int64_t st0 = 0, st1 = 0;
    if ((m->flags & ORC_TSPRING) && !(hj && hx)) return -4;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : st0, st1)
    for (int32_t k = 0; k < nc; ++k) {
        int32_t c = cells ? cells[k] : k;
        int64_t s = start[c], n = start[c + 1] - s;
        int64_t loc[2] = {0, 0};
        for (int64_t it = 0; it < nsteps; ++it) {
            double* mo = mom ? mom + ((size_t)it * nc + k) * NMOM : NULL;
            int e = cell_step(m, c % m->nx, c / m->nx, n, xs + s, ys + s, u + s, v + s, w + s,
                              th + s, r + s, h + s, dt, mo, loc, hj ? hj + s * ORC_HCAP : NULL,
                              hx ? hx + s * ORC_HCAP : NULL);
            if (e) {
#pragma omp critical
                { if (!rc) rc = e; }
                break;
            }
        }
        st0 += loc[0];
        st1 += loc[1];
    }
    if (stats) {
        stats[0] += st0;
        stats[1] += st1;
    }
    return rc;
}

/* Threads of the parallel loops over cells (timing only; results do not
 * depend on it).  Returns the number now in effect. */
int orc_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

/* ----------------------------------------------------------- continuum --- */
/* Q = (rho, P_x, P_y, P_w) per cell: cell sums over the cell area
 * (initialisation of the coarse model from DEM statistics, Algorithm 1). */
void orc_q_from_moments(const orc_model* m, const double* mom, double* Q)
{
    double A = m->Lx * m->Ly;
    for (int32_t c = 0; c < m->nx * m->ny; ++c) {
        const double* s = mom + (size_t)c * NMOM;
        Q[4 * c + 0] = s[M_MASS] / A;
        Q[4 * c + 1] = s[M_PX] / A;
        Q[4 * c + 2] = s[M_PY] / A;
        Q[4 * c + 3] = s[M_L] / A;
    }
}

/* One Lax-Friedrichs step of eq:pde on the periodic coarse grid (Sec. 3.2).
 * Mass and spin angular momentum in conservative form with flux <v> q;
 * momentum with the Oseen approximation <v>.grad<rho v>.  Coefficients <v>
 * (number average U/n, 0 in an empty cell) and drag sources (S/A) come from
 * the DEM statistics of the same time level.  Returns the CFL number
 * max(|u| dT/dX + |v| dT/dY). */
double orc_lf_step(const orc_model* m, const double* Q, const double* mom, double dT, double* Qn)
{
    const int nx = m->nx, ny = m->ny;
    const double A = m->Lx * m->Ly;
    const double cx = dT / (2.0 * m->Lx), cy = dT / (2.0 * m->Ly);
    double cfl = 0.0;
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) {
            int C = iy * nx + ix;
            int E = iy * nx + (ix + 1) % nx, W = iy * nx + (ix + nx - 1) % nx;
            int N = ((iy + 1) % ny) * nx + ix, S = ((iy + ny - 1) % ny) * nx + ix;
            /* Dirichlet in x (Sec. 4.4): beyond the first and last column lies
             * a ghost cell with zero state and zero coefficients (no ice, no
             * drift); E or W = -1 marks it */
            if (m->flags & ORC_DIRICHLET_X) {
                if (ix == nx - 1) E = -1;
                if (ix == 0) W = -1;
            }
            const double* sC = mom + (size_t)C * NMOM;
#define UBAR(K) ((K) >= 0 && mom[(size_t)(K) * NMOM + M_N] > 0 ? mom[(size_t)(K) * NMOM + M_UX] / mom[(size_t)(K) * NMOM + M_N] : 0.0)
#define VBAR(K) ((K) >= 0 && mom[(size_t)(K) * NMOM + M_N] > 0 ? mom[(size_t)(K) * NMOM + M_UY] / mom[(size_t)(K) * NMOM + M_N] : 0.0)
#define QV(K, F) ((K) >= 0 ? Q[4 * (K) + (F)] : 0.0)
            double uE = UBAR(E), uW = UBAR(W), vN = VBAR(N), vS = VBAR(S);
            double uC = UBAR(C), vC = VBAR(C);
#undef UBAR
#undef VBAR
            double c = fabs(uC) * dT / m->Lx + fabs(vC) * dT / m->Ly;
            if (c > cfl) cfl = c;
            /* mass, conservative */
            {
                int f = 0;
                double qE = QV(E, f), qW = QV(W, f), qN = QV(N, f), qS = QV(S, f);
                Qn[4 * C + f] = 0.25 * (qE + qW + qN + qS) - cx * (uE * qE - uW * qW) -
                                cy * (vN * qN - vS * qS);
            }
            /* momentum, Oseen form, drag source */
            for (int f = 1; f <= 2; ++f) {
                double qE = QV(E, f), qW = QV(W, f), qN = QV(N, f), qS = QV(S, f);
                double src = sC[f == 1 ? M_SVX : M_SVY] / A;
                Qn[4 * C + f] = 0.25 * (qE + qW + qN + qS) -
                                dT * (uC * (qE - qW) / (2.0 * m->Lx) + vC * (qN - qS) / (2.0 * m->Ly)) +
                                dT * src;
            }
            /* spin angular momentum, conservative, drag-torque source */
            {
                int f = 3;
                double qE = QV(E, f), qW = QV(W, f), qN = QV(N, f), qS = QV(S, f);
                Qn[4 * C + f] = 0.25 * (qE + qW + qN + qS) - cx * (uE * qE - uW * qW) -
                                cy * (vN * qN - vS * qS) + dT * sC[M_SW] / A;
            }
#undef QV
        }
    return cfl;
}

/* ------------------------------------------------- coarse-to-fine update --- */
/* Re-synchronise the floes of one cell to target coarse values (rho, P_x, P_y,
 * P_w) (Sec. 3.3, all n_t sub-steps at once): radii scaled by the common factor
 * that makes the cell mass hit rho A (the increment is distributed in
 * proportion to the radii), then a uniform velocity shift A dP / M and a
 * uniform spin shift A dP_w / sum I (increments distributed in proportion to
 * mass and inertia).  Returns -1 for an empty cell with a nonzero target. */
int orc_resync_cell(const orc_model* m, int64_t n, double* u, double* v, double* w, double* r,
                    const double* h, const double target[4])
{
    const double A = m->Lx * m->Ly;
    if (n == 0) return (target[0] != 0.0) ? -1 : 0;
    nsum M = {0, 0};
    for (int64_t l = 0; l < n; ++l) nadd(&M, m->rho_ice * h[l] * PI * r[l] * r[l]);
    double s = sqrt(target[0] * A / nval(&M));
    for (int64_t l = 0; l < n; ++l) r[l] *= s;
    nsum M2 = {0, 0}, Px = {0, 0}, Py = {0, 0}, L = {0, 0}, I = {0, 0};
    for (int64_t l = 0; l < n; ++l) {
        double ml = m->rho_ice * h[l] * PI * r[l] * r[l];
        nadd(&M2, ml);
        nadd(&Px, ml * u[l]);
        nadd(&Py, ml * v[l]);
        nadd(&L, ml * r[l] * r[l] * w[l]);
        nadd(&I, ml * r[l] * r[l]);
    }
    double dvx = (target[1] * A - nval(&Px)) / nval(&M2);
    double dvy = (target[2] * A - nval(&Py)) / nval(&M2);
    double dw = (target[3] * A - nval(&L)) / nval(&I);
    for (int64_t l = 0; l < n; ++l) {
        u[l] += dvx;
        v[l] += dvy;
        w[l] += dw;
    }
    return 0;
}

/*
 * nis_oracle.c -- plain FP64 CPU oracle of the neural in-scattering hot path
 * (Fang, Feng, Cui, "A real-time rendering method for high albedo anisotropic
 * materials with multiple scattering", arXiv 2401.14051).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the HIP library is
 * checked against.  It is called only from the test-suite, the smoke check and
 * the benchmark's CPU-baseline leg; the library never links, loads or calls it,
 * and it shares no code, header, table or helper with the library.
 *
 * Everything is computed in double precision with plain loops in the order the
 * method defines it: no blocking, no fusion, no reordering beyond the
 * definitions below.  Inputs (density grid, points, directions, weights) are
 * the float32 values the library receives, promoted to double.
 *
 * Conventions (readings of the paper, where it is silent):
 *  - the medium fills the unit cube [0,1]^3; voxel (ix,iy,iz) of a level with
 *    edge n has its centre at ((i+1/2)/n); arrays are [z][y][x], x fastest;
 *  - extinction is mu_t(x) = sigma_t * rho(x) (Sec. III.C.1, eq. 15);
 *  - l is the unit vector towards the distant light (eq. 16), omega the unit
 *    camera-ray direction; the single-scatter cosine is omega . l;
 *  - interpolation is index-clamped multilinear: i0 = floor(c), w = c - i0,
 *    value = (1-w) A[clamp(i0)] + w A[clamp(i0+1)] along each axis.
 *
 * Parity pins: every function is checked in the CPU test-suite against closed
 * forms, invariants, library routines or brute force (see the tests).  The
 * end-to-end value of a random network has no printed value in the paper and
 * is pinned through those parts plus zero- and selector-weight probes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OM_LAYERS 12          /* 8 diffuse + 4 highlight template layers */
#define OM_DIFFUSE 8
#define OM_SITES 225          /* 9 (along the light) x 5 x 5 lattice sites */
#define OM_FEAT 80            /* 16 channels x 5 positions after the CNN */
#define OM_STATS 8            /* squeeze vector of eq. (24) */
#define OM_DESC (OM_LAYERS * (OM_FEAT + OM_STATS) + 1)
#define OM_GROUP (216 + 8 + 3456 + 16 + 64 + 4 + 64 + 16)

static const double OM_PI = 3.14159265358979323846;

typedef struct {
    int n, levels;
    int64_t *off;           /* offset of level m in rho */
    double *rho;            /* density pyramid, all levels */
    int has_light;
    double l[3];            /* unit vector towards the light */
    int a, b, c, sigma;     /* dominant axis, lateral axes, sign of l_a */
    double sb, sc;          /* lateral shear l_b/|l_a|, l_c/|l_a| */
    int *ulo, *uhi, *vlo, *vhi;
    double **D;             /* path density per level, [J][V][U] */
} om_medium;

/* ------------------------------------------------------------------ */
/* Henyey-Greenstein phase function, Sec. III.B.3 eq. (5).  The printed
 * denominator "1+g^2.2g cos" is read as 1 + g^2 - 2 g cos(theta).          */
double om_hg(double g, double mu)
{
    double den = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (4.0 * OM_PI * den * sqrt(den));
}

/* Complete elliptic integral of the second kind,
 * E(m) = int_0^(pi/2) sqrt(1 - m sin^2 t) dt, 0 <= m < 1, by the
 * arithmetic-geometric mean: a0 = 1, b0 = sqrt(1-m), c0 = sqrt(m),
 * K = pi / (2 a_N), E = K (1 - sum_n 2^(n-1) c_n^2). */
static double om_ellip_e(double m)
{
    double a = 1.0, b = sqrt(1.0 - m), c = sqrt(m), sum = 0.5 * c * c, pw = 0.5;
    for (int it = 0; it < 40 && fabs(c) > 1e-17; it++) {
        double an = 0.5 * (a + b);
        c = 0.5 * (a - b);
        b = sqrt(a * b);
        a = an;
        pw *= 2.0;
        sum += pw * c * c;
    }
    return (OM_PI / (2.0 * a)) * (1.0 - sum);
}

/* 64-point Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_64). */
static double om_gl_x[64], om_gl_w[64];
static int om_gl_ready = 0;
static void om_gl_init(void)
{
    if (om_gl_ready) return;
    const int n = 64;
    for (int i = 0; i < n; i++) {
        double x = cos(OM_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; k++) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        om_gl_x[i] = x;
        om_gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    om_gl_ready = 1;
}

/* Volume phase of one HG lobe (Sec. III.A, eq. 9): the mean of HG(g, w.phi)
 * over the directions phi of a cone of half-angle beta around a unit
 * direction d, given mu0 = w.d.  With phi at polar angle theta from d and
 * azimuth psi, w.phi = mu0 cos theta + sqrt(1 - mu0^2) sin theta cos psi, so
 * 1 + g^2 - 2 g w.phi = A - B cos psi; the azimuthal integral of
 * (A - B cos psi)^(-3/2) over [0, 2 pi) is 4 E(2B/(A+B)) / ((A-B) sqrt(A+B))
 * (B taken >= 0, cos psi being symmetric), and cos theta in [cos beta, 1] is
 * integrated by 64-point Gauss-Legendre.  The cone's solid angle is
 * 2 pi (1 - cos beta).  om_gl_init() must have run. */
double om_hg_cone(double g, double mu0, double beta)
{
    double cb = cos(beta), s0 = sqrt(fmax(0.0, 1.0 - mu0 * mu0));
    double half = 0.5 * (1.0 - cb), mid = 0.5 * (1.0 + cb), acc = 0.0;
    for (int i = 0; i < 64; i++) {
        double t = mid + half * om_gl_x[i];
        double A = 1.0 + g * g - 2.0 * g * mu0 * t;
        double B = fabs(2.0 * g * s0 * sqrt(fmax(0.0, 1.0 - t * t)));
        double az = 4.0 * om_ellip_e(2.0 * B / (A + B)) / ((A - B) * sqrt(A + B));
        acc += om_gl_w[i] * half * az;
    }
    return (1.0 - g * g) / (4.0 * OM_PI) * acc / (2.0 * OM_PI * (1.0 - cb));
}

/* Multi-lobe HG phase (Sec. III.A, eq. 6): a linear combination of HG lobes
 * with weights lw[i] (summing to one) and asymmetries lg[i].  One lobe of
 * weight 1 is the HG phase of eq. 5. */
void om_volume_init(void) { om_gl_init(); }

double om_mhg(int nl, const double *lw, const double *lg, double mu)
{
    double v = 0.0;
    for (int i = 0; i < nl; i++) v += lw[i] * om_hg(lg[i], mu);
    return v;
}

static int clampi(int i, int lo, int hi) { return i < lo ? lo : (i > hi ? hi : i); }

/* Threads of the OpenMP loops (for timing the oracle on a given core count). */
void om_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int om_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Density pyramid, Sec. III.B.1: the grid is down-sampled level by level to
 * 1^3 with the 2x2x2 box mean (the filter the paper leaves unstated).      */
om_medium *om_create(const float *rho0, int n)
{
    if (n < 1 || (n & (n - 1)) != 0) return NULL;
    om_medium *M = (om_medium *)calloc(1, sizeof(om_medium));
    int L = 1;
    while ((1 << (L - 1)) < n) L++;
    M->n = n;
    M->levels = L;
    M->off = (int64_t *)calloc((size_t)L + 1, sizeof(int64_t));
    for (int m = 0; m < L; m++) {
        int64_t nm = n >> m;
        M->off[m + 1] = M->off[m] + nm * nm * nm;
    }
    M->rho = (double *)malloc((size_t)M->off[L] * sizeof(double));
    for (int64_t i = 0; i < (int64_t)n * n * n; i++) M->rho[i] = (double)rho0[i];
    for (int m = 0; m + 1 < L; m++) {
        int nf = n >> m, nc = n >> (m + 1);
        const double *f = M->rho + M->off[m];
        double *cc = M->rho + M->off[m + 1];
        for (int z = 0; z < nc; z++)
            for (int y = 0; y < nc; y++)
                for (int x = 0; x < nc; x++) {
                    double s = 0.0;
                    for (int dz = 0; dz < 2; dz++)
                        for (int dy = 0; dy < 2; dy++)
                            for (int dx = 0; dx < 2; dx++)
                                s += f[((int64_t)(2 * z + dz) * nf + (2 * y + dy)) * nf + (2 * x + dx)];
                    cc[((int64_t)z * nc + y) * nc + x] = s / 8.0;
                }
    }
    M->ulo = (int *)calloc((size_t)L, sizeof(int));
    M->uhi = (int *)calloc((size_t)L, sizeof(int));
    M->vlo = (int *)calloc((size_t)L, sizeof(int));
    M->vhi = (int *)calloc((size_t)L, sizeof(int));
    M->D = (double **)calloc((size_t)L, sizeof(double *));
    return M;
}

void om_free(om_medium *M)
{
    if (!M) return;
    for (int m = 0; m < M->levels; m++) free(M->D[m]);
    free(M->D); free(M->ulo); free(M->uhi); free(M->vlo); free(M->vhi);
    free(M->rho); free(M->off); free(M);
}

int om_levels(const om_medium *M) { return M->levels; }
int64_t om_level_offset(const om_medium *M, int m) { return M->off[m]; }
const double *om_pyramid(const om_medium *M) { return M->rho; }

/* value of level m at integer voxel (x,y,z) with index clamping */
static double vox(const om_medium *M, int m, int x, int y, int z)
{
    int nm = M->n >> m;
    x = clampi(x, 0, nm - 1); y = clampi(y, 0, nm - 1); z = clampi(z, 0, nm - 1);
    return M->rho[M->off[m] + ((int64_t)z * nm + y) * nm + x];
}

/* ------------------------------------------------------------------ */
/* Light frame: the sweep runs along the dominant axis a of l (lowest index on
 * ties), with sigma = sign(l_a), lateral axes (b,c) ascending and shears
 * s = l_lateral / |l_a|.  Slice J = 0 is the slice nearest the light.      */
static int slice_index(const om_medium *M, int nm, int J) { return M->sigma > 0 ? nm - 1 - J : J; }

static void ray_range(double s, int nm, int *lo, int *hi)
{
    double a = (nm - 1) * s;
    *lo = (int)floor(a < 0.0 ? a : 0.0) - 1;
    *hi = (int)ceil((double)(nm - 1) + (a > 0.0 ? a : 0.0)) + 1;
}

/* bilinear density on slice ia of level m at lateral index coordinates (u,v)
 * along axes (b,c); zero when (u,v) lies outside [-1/2, nm-1/2]^2.          */
static double slice_sample(const om_medium *M, int m, int ia, double u, double v)
{
    int nm = M->n >> m;
    if (u < -0.5 || u > nm - 0.5 || v < -0.5 || v > nm - 0.5) return 0.0;
    int iu = (int)floor(u), iv = (int)floor(v);
    double wu = u - iu, wv = v - iv;
    double acc = 0.0;
    for (int dv = 0; dv < 2; dv++)
        for (int du = 0; du < 2; du++) {
            int idx[3];
            idx[M->a] = ia;
            idx[M->b] = iu + du;
            idx[M->c] = iv + dv;
            double w = (du ? wu : 1.0 - wu) * (dv ? wv : 1.0 - wv);
            acc += w * vox(M, m, idx[0], idx[1], idx[2]);
        }
    return acc;
}

/* Graded transmittance fields, Sec. III.B.1 eq. (1): the path integral of
 * density from each point towards the light is stored, unscaled by the
 * coefficient, as a path density D_m(U,V,J) on light-sheared rays: ray (U,V)
 * crosses slice J at lateral coordinates (U - J sb, V - J sc), and
 *   D_m(U,V,J) = ds_m * ( sum_{J'<J} r(U,V,J') + r(U,V,J)/2 ),
 * ds_m = h_m / |l_a|, a trapezoid rule from the light-facing face plane.    */
int om_set_light(om_medium *M, const float dir[3])
{
    double l[3] = {dir[0], dir[1], dir[2]};
    double nrm = sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
    if (!(nrm > 0.0) || !isfinite(nrm)) return -1;
    for (int i = 0; i < 3; i++) M->l[i] = l[i] / nrm;
    int a = 0;
    for (int i = 1; i < 3; i++)
        if (fabs(M->l[i]) > fabs(M->l[a])) a = i;
    M->a = a;
    M->b = a == 0 ? 1 : 0;
    M->c = a == 2 ? 1 : 2;
    M->sigma = M->l[a] > 0.0 ? 1 : -1;
    M->sb = M->l[M->b] / fabs(M->l[a]);
    M->sc = M->l[M->c] / fabs(M->l[a]);
    for (int m = 0; m < M->levels; m++) {
        int nm = M->n >> m;
        ray_range(M->sb, nm, &M->ulo[m], &M->uhi[m]);
        ray_range(M->sc, nm, &M->vlo[m], &M->vhi[m]);
        int nu = M->uhi[m] - M->ulo[m] + 1, nv = M->vhi[m] - M->vlo[m] + 1;
        free(M->D[m]);
        M->D[m] = (double *)malloc((size_t)nu * nv * nm * sizeof(double));
        double ds = (1.0 / nm) / fabs(M->l[a]);
        /* rays are independent: one thread per row of rays */
#pragma omp parallel for schedule(dynamic, 1)
        for (int V = M->vlo[m]; V <= M->vhi[m]; V++)
            for (int U = M->ulo[m]; U <= M->uhi[m]; U++) {
                double sum = 0.0;
                for (int J = 0; J < nm; J++) {
                    double r = slice_sample(M, m, slice_index(M, nm, J), U - J * M->sb, V - J * M->sc);
                    M->D[m][((int64_t)J * nv + (V - M->vlo[m])) * nu + (U - M->ulo[m])] = ds * (sum + 0.5 * r);
                    sum += r;
                }
            }
    }
    M->has_light = 1;
    return 0;
}

/* frame[0..3] = a, b, c, sigma; shear[0..1] = sb, sc; l[0..2] */
void om_light_frame(const om_medium *M, int *frame, double *shear, double *l)
{
    frame[0] = M->a; frame[1] = M->b; frame[2] = M->c; frame[3] = M->sigma;
    shear[0] = M->sb; shear[1] = M->sc;
    for (int i = 0; i < 3; i++) l[i] = M->l[i];
}

/* dims[0..4] = U_lo, U_hi, V_lo, V_hi, n_J */
const double *om_path_density(const om_medium *M, int m, int *dims)
{
    dims[0] = M->ulo[m]; dims[1] = M->uhi[m]; dims[2] = M->vlo[m]; dims[3] = M->vhi[m];
    dims[4] = M->n >> m;
    return M->D[m];
}

/* ------------------------------------------------------------------ */
/* Density at a point x of the unit cube at level m: zero outside the closed
 * cube, otherwise index-clamped trilinear at grid coordinates x*n_m - 1/2.  */
double om_sample_rho(const om_medium *M, int m, const double x[3])
{
    int nm = M->n >> m;
    for (int i = 0; i < 3; i++)
        if (x[i] < 0.0 || x[i] > 1.0) return 0.0;
    double gx = x[0] * nm - 0.5, gy = x[1] * nm - 0.5, gz = x[2] * nm - 0.5;
    int ix = (int)floor(gx), iy = (int)floor(gy), iz = (int)floor(gz);
    double wx = gx - ix, wy = gy - iy, wz = gz - iz;
    double acc = 0.0;
    for (int dz = 0; dz < 2; dz++)
        for (int dy = 0; dy < 2; dy++)
            for (int dx = 0; dx < 2; dx++) {
                double w = (dx ? wx : 1.0 - wx) * (dy ? wy : 1.0 - wy) * (dz ? wz : 1.0 - wz);
                acc += w * vox(M, m, ix + dx, iy + dy, iz + dz);
            }
    return acc;
}

/* Path density towards the light at x, level m: x is mapped to sheared ray
 * coordinates (U_f, V_f, J_f) and D_m is interpolated trilinearly with index
 * clamping over its ray and slice ranges.                                   */
double om_sample_D(const om_medium *M, int m, const double x[3])
{
    int nm = M->n >> m;
    double g[3];
    for (int i = 0; i < 3; i++) g[i] = x[i] * nm - 0.5;
    double Jf = M->sigma > 0 ? (nm - 1) - g[M->a] : g[M->a];
    double Uf = g[M->b] + Jf * M->sb;
    double Vf = g[M->c] + Jf * M->sc;
    int nu = M->uhi[m] - M->ulo[m] + 1, nv = M->vhi[m] - M->vlo[m] + 1;
    int iu = (int)floor(Uf), iv = (int)floor(Vf), ij = (int)floor(Jf);
    double wu = Uf - iu, wv = Vf - iv, wj = Jf - ij;
    double acc = 0.0;
    for (int dj = 0; dj < 2; dj++)
        for (int dv = 0; dv < 2; dv++)
            for (int du = 0; du < 2; du++) {
                int U = clampi(iu + du, M->ulo[m], M->uhi[m]) - M->ulo[m];
                int V = clampi(iv + dv, M->vlo[m], M->vhi[m]) - M->vlo[m];
                int J = clampi(ij + dj, 0, nm - 1);
                double w = (du ? wu : 1.0 - wu) * (dv ? wv : 1.0 - wv) * (dj ? wj : 1.0 - wj);
                acc += w * M->D[m][((int64_t)J * nv + V) * nu + U];
            }
    return acc;
}

/* ------------------------------------------------------------------ */
/* Template lattice (Sec. III.B.2, in the light-aligned 12 x (5x5x9) form):
 * site t = ((q+4)*5 + (j+2))*5 + (i+2) has offset o = i e_b + j e_c + q l/|l_a|
 * and, in layer k, position p + 2^k h_0 o.  Layers 0-7 form the diffuse
 * group, 8-11 the highlight group; layer k samples level min(k, L-1).      */
static void site_offset(const om_medium *M, int t, double o[3])
{
    int q = t / 25 - 4, j = (t / 5) % 5 - 2, i = t % 5 - 2;
    double la = fabs(M->l[M->a]);
    for (int d = 0; d < 3; d++) o[d] = q * M->l[d] / la;
    o[M->b] += i;
    o[M->c] += j;
}

/* Per-point features of every layer (Sec. III.B.2-4, eq. 1, 8, 15, 24) for
 * a phase of nl HG lobes (eq. 6; f below; one lobe is plain HG):
 *   tbar[p][k][t] graded transmittance exp(-lam^(m+1) sigma_t D_m(site)),
 *   rho [p][k][t] density at the site,
 *   phi [p][t]    log1p of the phase feature f(w.d_t) f(d_t.l), d_t = o/|o|
 *                 (f(w.l) at the centre site),
 *   stats[p][k][8] = mean rho, mean phi, mean tbar, max rho, max phi,
 *                 max tbar, g, alpha = acos(w.l), where g is the phase's
 *                 mean cosine, sum_i lw[i] lg[i],
 *   tp[p] = exp(-sigma_t D_0(p)) (eq. 15), f0[p] = f(w.l) tp[p] (eq. 19).
 * With volume != 0 both factors of the phase feature are volume phases
 * (eq. 9): means of f over the cone under which the site, a ball of half the
 * lattice spacing, is seen from p (om_hg_cone); the centre site keeps f(w.l).
 * Any output pointer may be NULL.                                           */
void om_features(const om_medium *M, double sigma_t, int nl, const double *lw, const double *lg,
                 int volume, double lam, const float *pts, const float *dirs, int64_t np,
                 double *tbar, double *rho, double *phi, double *stats,
                 double *tp, double *f0)
{
    double g = 0.0;
    for (int i = 0; i < nl; i++) g += lw[i] * lg[i];
    om_gl_init();
    int L = M->levels;
    double h0 = 1.0 / M->n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < np; p++) {
        double x[3], w[3];
        for (int d = 0; d < 3; d++) { x[d] = pts[3 * p + d]; w[d] = dirs[3 * p + d]; }
        double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        for (int d = 0; d < 3; d++) w[d] /= wn;
        double wl = w[0] * M->l[0] + w[1] * M->l[1] + w[2] * M->l[2];
        double alpha = acos(wl < -1.0 ? -1.0 : (wl > 1.0 ? 1.0 : wl));
        double ph[OM_SITES];
        double phmean = 0.0, phmax = -INFINITY;
        for (int t = 0; t < OM_SITES; t++) {
            double o[3];
            site_offset(M, t, o);
            double on = sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
            double P;
            if (on == 0.0) {
                P = om_mhg(nl, lw, lg, wl);
            } else {
                double wd = (w[0] * o[0] + w[1] * o[1] + w[2] * o[2]) / on;
                double dl = (o[0] * M->l[0] + o[1] * M->l[1] + o[2] * M->l[2]) / on;
                if (volume) {
                    /* eq. 9: the site seen from p as a ball of half the lattice
                     * spacing, i.e. a cone of half-angle asin(1 / (2 |o|)) */
                    double beta = asin(0.5 / on), fw = 0.0, fl = 0.0;
                    for (int i = 0; i < nl; i++) {
                        fw += lw[i] * om_hg_cone(lg[i], wd, beta);
                        fl += lw[i] * om_hg_cone(lg[i], dl, beta);
                    }
                    P = fw * fl;
                } else {
                    P = om_mhg(nl, lw, lg, wd) * om_mhg(nl, lw, lg, dl);
                }
            }
            ph[t] = log1p(P);
            phmean += ph[t];
            if (ph[t] > phmax) phmax = ph[t];
            if (phi) phi[p * OM_SITES + t] = ph[t];
        }
        phmean /= OM_SITES;
        for (int k = 0; k < OM_LAYERS; k++) {
            int m = k < L - 1 ? k : L - 1;
            double scale = ldexp(h0, k);
            double coef = pow(lam, m + 1) * sigma_t;
            double rs = 0.0, rm = -INFINITY, ts = 0.0, tm = -INFINITY;
            for (int t = 0; t < OM_SITES; t++) {
                double o[3], s[3];
                site_offset(M, t, o);
                for (int d = 0; d < 3; d++) s[d] = x[d] + scale * o[d];
                double r = om_sample_rho(M, m, s);
                double T = exp(-coef * om_sample_D(M, m, s));
                if (rho) rho[(p * OM_LAYERS + k) * OM_SITES + t] = r;
                if (tbar) tbar[(p * OM_LAYERS + k) * OM_SITES + t] = T;
                rs += r; ts += T;
                if (r > rm) rm = r;
                if (T > tm) tm = T;
            }
            if (stats) {
                double *v = stats + (p * OM_LAYERS + k) * OM_STATS;
                v[0] = rs / OM_SITES; v[1] = phmean; v[2] = ts / OM_SITES;
                v[3] = rm; v[4] = phmax; v[5] = tm; v[6] = g; v[7] = alpha;
            }
        }
        double T0 = exp(-sigma_t * om_sample_D(M, 0, x));
        if (tp) tp[p] = T0;
        if (f0) f0[p] = om_mhg(nl, lw, lg, wl) * T0;
    }
}

/* ------------------------------------------------------------------ */
/* Network.  Parameter block layout (this file's own): for each of the two
 * groups (diffuse, highlight): w1[8][1][3][3][3], b1[8], w2[16][8][3][3][3],
 * b2[16], s1[4][16], c1[4], s2[16][4], c2[16]; then for each backbone layer
 * A_i[out][in] followed by beta_i[out].                                      */

/* 3D-CNN over one layer's transmittance lattice (Sec. III.B.1, Fig. 3): the
 * 9x5x5 lattice (depth q, height j, width i) goes through conv 3^3 valid
 * 1->8, ReLU, conv 3^3 valid 8->16, ReLU, giving H[16][5].  Convolution is
 * cross-correlation with bias.  Then squeeze-excitation channel attention
 * (Sec. III.C.4, eq. 24-26, with the standard two-FC excitation, ratio 4):
 * z = mean over the 5 positions, e = sigmoid(s2 relu(s1 z + c1) + c2),
 * out[c*5+pos] = e[c] * H[c][pos].                                           */
void om_cnn_se(const double *grp, const double *lattice, double *out80)
{
    const double *w1 = grp, *b1 = w1 + 216, *w2 = b1 + 8, *b2 = w2 + 3456;
    const double *s1 = b2 + 16, *c1 = s1 + 64, *s2 = c1 + 4, *c2 = s2 + 64;
    double y1[8][7][3][3];
    for (int o = 0; o < 8; o++)
        for (int z = 0; z < 7; z++)
            for (int y = 0; y < 3; y++)
                for (int x = 0; x < 3; x++) {
                    double acc = b1[o];
                    for (int dz = 0; dz < 3; dz++)
                        for (int dy = 0; dy < 3; dy++)
                            for (int dx = 0; dx < 3; dx++)
                                acc += w1[(o * 3 + dz) * 9 + dy * 3 + dx] *
                                       lattice[((z + dz) * 5 + (y + dy)) * 5 + (x + dx)];
                    y1[o][z][y][x] = acc > 0.0 ? acc : 0.0;
                }
    double H[16][5];
    for (int o = 0; o < 16; o++)
        for (int z = 0; z < 5; z++) {
            double acc = b2[o];
            for (int c = 0; c < 8; c++)
                for (int dz = 0; dz < 3; dz++)
                    for (int dy = 0; dy < 3; dy++)
                        for (int dx = 0; dx < 3; dx++)
                            acc += w2[(((o * 8 + c) * 3 + dz) * 3 + dy) * 3 + dx] * y1[c][z + dz][dy][dx];
            H[o][z] = acc > 0.0 ? acc : 0.0;
        }
    double zc[16], hid[4], e[16];
    for (int c = 0; c < 16; c++) {
        double s = 0.0;
        for (int z = 0; z < 5; z++) s += H[c][z];
        zc[c] = s / 5.0;
    }
    for (int r = 0; r < 4; r++) {
        double acc = c1[r];
        for (int c = 0; c < 16; c++) acc += s1[r * 16 + c] * zc[c];
        hid[r] = acc > 0.0 ? acc : 0.0;
    }
    for (int c = 0; c < 16; c++) {
        double acc = c2[c];
        for (int r = 0; r < 4; r++) acc += s2[c * 4 + r] * hid[r];
        e[c] = 1.0 / (1.0 + exp(-acc));
    }
    for (int c = 0; c < 16; c++)
        for (int z = 0; z < 5; z++) out80[c * 5 + z] = e[c] * H[c][z];
}

/* Descriptor of one point: for k = 0..11 the 80 attention-weighted CNN
 * features of layer k (weights of its group) followed by its squeeze vector,
 * then the albedo: 12*88 + 1 = 1057 entries.                                */
void om_descriptor(const double *params, const double *tbar, const double *stats,
                   double albedo, double *desc)
{
    for (int k = 0; k < OM_LAYERS; k++) {
        const double *grp = params + (k < OM_DIFFUSE ? 0 : OM_GROUP);
        om_cnn_se(grp, tbar + k * OM_SITES, desc + k * (OM_FEAT + OM_STATS));
        for (int s = 0; s < OM_STATS; s++)
            desc[k * (OM_FEAT + OM_STATS) + OM_FEAT + s] = stats[k * OM_STATS + s];
    }
    desc[OM_DESC - 1] = albedo;
}

/* Backbone (Sec. III.C.2, Fig. 6, in MLP form): n_linear Linear layers of
 * width `width`, ReLU after all but the last; returns the scalar output y.  */
double om_mlp(const double *params, int width, int n_linear, const double *desc)
{
    const double *A = params + 2 * OM_GROUP;
    double *h = (double *)malloc(sizeof(double) * (width > OM_DESC ? width : OM_DESC));
    double *nx = (double *)malloc(sizeof(double) * width);
    memcpy(h, desc, sizeof(double) * OM_DESC);
    int din = OM_DESC;
    double y = 0.0;
    for (int li = 0; li < n_linear; li++) {
        int dout = li == n_linear - 1 ? 1 : width;
        const double *beta = A + (int64_t)dout * din;
        for (int o = 0; o < dout; o++) {
            double acc = beta[o];
            for (int i = 0; i < din; i++) acc += A[(int64_t)o * din + i] * h[i];
            nx[o] = (li == n_linear - 1) ? acc : (acc > 0.0 ? acc : 0.0);
        }
        A = beta + dout;
        if (li == n_linear - 1) y = nx[0];
        else memcpy(h, nx, sizeof(double) * dout);
        din = dout;
    }
    free(h);
    free(nx);
    return y;
}

/* Whole query: radiance L = I (f(w.l) T(p) + F) for a phase f of nl HG
 * lobes, with the network output decoded from the log space of the loss
 * (Sec. III.C.3, eq. 21, gamma = 4): F = albedo^gamma * expm1(y).
 * F0 = f(w.l) T(p) I is the single-scatter term of the scattering-order
 * series (eq. 19).  y_out/fhat_out may be NULL. */
void om_query(const om_medium *M, double sigma_t, double albedo, int nl, const double *lw,
              const double *lg, int volume, double lam,
              double gamma, double radiance, const double *params, int width, int n_linear,
              const float *pts, const float *dirs, int64_t np,
              double *L_out, double *y_out, double *fhat_out, double *desc_out)
{
    om_gl_init();
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < np; p++) {
        double *tb = (double *)malloc(sizeof(double) * OM_LAYERS * OM_SITES);
        double st[OM_LAYERS * OM_STATS];
        double f0;
        double *desc = desc_out ? desc_out + p * OM_DESC : (double *)malloc(sizeof(double) * OM_DESC);
        om_features(M, sigma_t, nl, lw, lg, volume, lam, pts + 3 * p, dirs + 3 * p, 1, tb, NULL, NULL, st, NULL, &f0);
        om_descriptor(params, tb, st, albedo, desc);
        double y = om_mlp(params, width, n_linear, desc);
        double F = pow(albedo, gamma) * expm1(y);
        L_out[p] = radiance * (f0 + F);
        if (y_out) y_out[p] = y;
        if (fhat_out) fhat_out[p] = F;
        if (!desc_out) free(desc);
        free(tb);
    }
}

/* ------------------------------------------------------------------ */
/* The paper's own templates (Sec. III.B.2, eq. 2-4), in place of the
 * lattices.  Readings (the paper gives counts, a uniformity measure and a
 * radius rule, but no construction):
 *  - diffuse sphere, 8 layers of 6, 8, 12, 16, 24, 32, 48, 48 points (the
 *    per-layer counts as printed; they sum to 194, not the 182 the text
 *    states); highlight cone, 4 layers of 32, 16, 16, 8 points;
 *  - unit templates: layer 0 is the centre plus 5 points on the unit
 *    sphere (of all arrangements in the closed unit ball, those farthest
 *    from the centre and each other, the most even by eq. 3), layer i >= 1
 *    fills the shell 1/2 <= |u| <= 1 (the sphere of the
 *    previous layer, about half as large, is the inner surface); "evenly
 *    distributed" is a spherical-Fibonacci direction (golden-angle
 *    azimuth, stratified z) per point with an equal-volume radial stratum
 *    taken from the additive sequence frac(1/2 + k c), c = 0.5698402909980532
 *    (the plastic-number step, decorrelated from the golden angle);
 *  - D(S_i) (eq. 3) is the mean over the layer's points of the distance to
 *    the nearest other point of the unit template, and the layer's radius is
 *    r_i = 2^(i-1) xi_i / (2^8 D(S_i)) with xi_i = 1 - 0.08 min(i, 5)
 *    (eq. 4), in unit-cube lengths; so neighbouring points of layer i are
 *    2^(i-1) xi_i voxels of a 256^3 grid apart;
 *  - the highlight cone has its apex at the point, its axis along l, unit
 *    length and unit base radius (the text's unit-size cone); it is scaled by
 *    d_l, the distance from the point towards the light to where that ray
 *    leaves the unit cube (the light's entry into the medium; 0 when the ray
 *    misses it), and its 4 layers split the axis into equal quarters;
 *    point k of layer h sits at the axial t that divides the layer's
 *    frustum volume at the fraction (k+1/2)/n, at radius sqrt(w_k) t (w_k
 *    as above) and golden-angle azimuth in the orthonormal
 *    frame of l of Duff et al. (2017), "Building an orthonormal basis,
 *    revisited";
 *  - each layer samples the level whose voxel matches its point spacing:
 *    m = the number of k >= 0 with spacing * N >= sqrt(2) 2^k (capped at
 *    L-1), spacing = r_i D(S_i) for a diffuse layer and D(C_h) d_l for a
 *    highlight layer;
 *  - features per template point as for the lattice sites (density, graded
 *    transmittance, point phase with d the unit direction from p to the
 *    point, f(w.l) where the point is p itself), the squeeze vector of
 *    eq. (24) per layer over its points;
 *  - descriptor: per layer, its graded transmittances, densities, phase
 *    features (template order) and squeeze vector; zeros up to the albedo
 *    entry, which keeps index 1056 (the lattice descriptor's).            */
#define OM_TPL_SITES 266
static const int om_tpl_count[OM_LAYERS] = {6, 8, 12, 16, 24, 32, 48, 48, 32, 16, 16, 8};
static const double OM_GOLDEN_ANGLE = 2.39996322972865332;   /* pi (3 - sqrt 5) */
static const double OM_R2STEP = 0.5698402909980532;

int om_tpl_count_of(int layer) { return om_tpl_count[layer]; }

static int om_tpl_first(int layer)
{
    int f = 0;
    for (int i = 0; i < layer; i++) f += om_tpl_count[i];
    return f;
}

static double om_frac(double x) { return x - floor(x); }

/* Unit template point k of a layer: diffuse layers in world axes, highlight
 * layers as (t along l, x1, x2) in the frame of l.                          */
void om_tpl_unit(int layer, int k, double u[3])
{
    int n = om_tpl_count[layer];
    if (layer < OM_DIFFUSE) {
        int kk = k, nn = n;
        double rad;
        if (layer == 0) {
            if (k == 0) { u[0] = u[1] = u[2] = 0.0; return; }
            kk = k - 1;
            nn = n - 1;
            rad = 1.0;
        } else {
            double w = om_frac(0.5 + kk * OM_R2STEP);
            rad = cbrt(0.125 + w * 0.875);
        }
        double z = 1.0 - (2.0 * kk + 1.0) / nn;
        double rxy = sqrt(1.0 - z * z);
        double az = kk * OM_GOLDEN_ANGLE;
        u[0] = rad * (rxy * cos(az));
        u[1] = rad * (rxy * sin(az));
        u[2] = rad * z;
    } else {
        int h = layer - OM_DIFFUSE;
        double lo = h / 4.0, hi = (h + 1) / 4.0;
        double t = cbrt(lo * lo * lo + ((k + 0.5) / n) * (hi * hi * hi - lo * lo * lo));
        double w = om_frac(0.5 + k * OM_R2STEP);
        double rad = sqrt(w) * t;
        double az = k * OM_GOLDEN_ANGLE;
        u[0] = t;
        u[1] = rad * cos(az);
        u[2] = rad * sin(az);
    }
}

/* eq. (3): mean over the layer's unit points of the nearest-neighbour distance */
double om_tpl_D(int layer)
{
    int n = om_tpl_count[layer];
    double sum = 0.0;
    for (int j = 0; j < n; j++) {
        double a[3], best = INFINITY;
        om_tpl_unit(layer, j, a);
        for (int k = 0; k < n; k++) {
            if (k == j) continue;
            double b[3];
            om_tpl_unit(layer, k, b);
            double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
            double d = sqrt(dx * dx + dy * dy + dz * dz);
            if (d < best) best = d;
        }
        sum += best;
    }
    return sum / n;
}

/* eq. (4): radius of diffuse layer i in unit-cube lengths */
double om_tpl_radius(int layer)
{
    double xi = 1.0 - 0.08 * (layer < 5 ? layer : 5);
    return ldexp(1.0, layer - 1) * xi / (256.0 * om_tpl_D(layer));
}

/* level whose voxel matches a spacing (unit-cube length) on an n^3 grid */
static int om_tpl_level(double spacing, int n, int L)
{
    double x = spacing * n;
    int m = 0;
    while (m < L - 1 && x >= 1.4142135623730951 * ldexp(1.0, m)) m++;
    return m;
}

/* distance from x towards the light to where that ray leaves the unit cube
 * (0 when it misses the cube or leaves it behind x)                         */
double om_tpl_light_extent(const double l[3], const double x[3])
{
    double t0 = -INFINITY, t1 = INFINITY;
    for (int d = 0; d < 3; d++) {
        if (l[d] == 0.0) {
            if (x[d] < 0.0 || x[d] > 1.0) return 0.0;
            continue;
        }
        double a = (0.0 - x[d]) / l[d], b = (1.0 - x[d]) / l[d];
        double lo = a < b ? a : b, hi = a < b ? b : a;
        if (lo > t0) t0 = lo;
        if (hi < t1) t1 = hi;
    }
    if (t1 < t0 || t1 <= 0.0) return 0.0;
    return t1;
}

/* orthonormal frame (e1, e2) of unit l, Duff et al. 2017 */
static void om_onb(const double l[3], double e1[3], double e2[3])
{
    double s = l[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (s + l[2]);
    double b = l[0] * l[1] * a;
    e1[0] = 1.0 + s * l[0] * l[0] * a;
    e1[1] = s * b;
    e1[2] = -s * l[0];
    e2[0] = b;
    e2[1] = s + l[1] * l[1] * a;
    e2[2] = -l[1];
}

/* Features at the template points of every layer for np points:
 *   tbar/rho/phi [p][266] in template order (layer by layer), stats
 *   [p][12][8] as eq. (24), f0[p] = f(w.l) T(p); any output may be NULL.    */
void om_tpl_features(const om_medium *M, double sigma_t, int nl, const double *lw, const double *lg,
                     double lam, const float *pts, const float *dirs, int64_t np,
                     double *tbar, double *rho, double *phi, double *stats, double *f0)
{
    double g = 0.0;
    for (int i = 0; i < nl; i++) g += lw[i] * lg[i];
    int L = M->levels;
    double rad[OM_DIFFUSE], Dl[OM_LAYERS];
    int mdiff[OM_DIFFUSE];
    for (int i = 0; i < OM_LAYERS; i++) Dl[i] = om_tpl_D(i);
    for (int i = 0; i < OM_DIFFUSE; i++) {
        rad[i] = om_tpl_radius(i);
        mdiff[i] = om_tpl_level(rad[i] * Dl[i], M->n, L);
    }
    double e1[3], e2[3];
    om_onb(M->l, e1, e2);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < np; p++) {
        double x[3], w[3];
        for (int d = 0; d < 3; d++) { x[d] = pts[3 * p + d]; w[d] = dirs[3 * p + d]; }
        double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        for (int d = 0; d < 3; d++) w[d] /= wn;
        double wl = w[0] * M->l[0] + w[1] * M->l[1] + w[2] * M->l[2];
        double alpha = acos(wl < -1.0 ? -1.0 : (wl > 1.0 ? 1.0 : wl));
        double dlen = om_tpl_light_extent(M->l, x);
        for (int k = 0; k < OM_LAYERS; k++) {
            int n = om_tpl_count[k], f = om_tpl_first(k);
            int m = k < OM_DIFFUSE ? mdiff[k] : om_tpl_level(Dl[k] * dlen, M->n, L);
            double coef = pow(lam, m + 1) * sigma_t;
            double rs = 0.0, rm = -INFINITY, ts = 0.0, tm = -INFINITY, ps = 0.0, pm = -INFINITY;
            for (int j = 0; j < n; j++) {
                double u[3], s[3];
                om_tpl_unit(k, j, u);
                if (k < OM_DIFFUSE) {
                    for (int d = 0; d < 3; d++) s[d] = x[d] + rad[k] * u[d];
                } else {
                    for (int d = 0; d < 3; d++) {
                        double o = u[0] * M->l[d] + u[1] * e1[d] + u[2] * e2[d];
                        s[d] = x[d] + dlen * o;
                    }
                }
                double r = om_sample_rho(M, m, s);
                double T = exp(-coef * om_sample_D(M, m, s));
                double v[3] = {s[0] - x[0], s[1] - x[1], s[2] - x[2]};
                double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                double P;
                if (vn == 0.0) {
                    P = om_mhg(nl, lw, lg, wl);
                } else {
                    double wd = (w[0] * v[0] + w[1] * v[1] + w[2] * v[2]) / vn;
                    double dl = (v[0] * M->l[0] + v[1] * M->l[1] + v[2] * M->l[2]) / vn;
                    P = om_mhg(nl, lw, lg, wd) * om_mhg(nl, lw, lg, dl);
                }
                double ph = log1p(P);
                if (rho) rho[p * OM_TPL_SITES + f + j] = r;
                if (tbar) tbar[p * OM_TPL_SITES + f + j] = T;
                if (phi) phi[p * OM_TPL_SITES + f + j] = ph;
                rs += r; ts += T; ps += ph;
                if (r > rm) rm = r;
                if (T > tm) tm = T;
                if (ph > pm) pm = ph;
            }
            if (stats) {
                double *v = stats + (p * OM_LAYERS + k) * OM_STATS;
                v[0] = rs / n; v[1] = ps / n; v[2] = ts / n;
                v[3] = rm; v[4] = pm; v[5] = tm; v[6] = g; v[7] = alpha;
            }
        }
        if (f0) f0[p] = om_mhg(nl, lw, lg, wl) * exp(-sigma_t * om_sample_D(M, 0, x));
    }
}

/* Template descriptor: per layer its graded transmittances, densities and
 * phase features in template order, then its squeeze vector (3 n_k + 8
 * entries); zeros up to the albedo entry at index OM_DESC - 1.              */
void om_tpl_descriptor(const double *tbar, const double *rho, const double *phi, const double *stats,
                       double albedo, double *desc)
{
    for (int i = 0; i < OM_DESC; i++) desc[i] = 0.0;
    int pos = 0;
    for (int k = 0; k < OM_LAYERS; k++) {
        int n = om_tpl_count[k], f = om_tpl_first(k);
        for (int j = 0; j < n; j++) desc[pos++] = tbar[f + j];
        for (int j = 0; j < n; j++) desc[pos++] = rho[f + j];
        for (int j = 0; j < n; j++) desc[pos++] = phi[f + j];
        for (int s = 0; s < OM_STATS; s++) desc[pos++] = stats[k * OM_STATS + s];
    }
    desc[OM_DESC - 1] = albedo;
}

/* Whole query with the paper's templates: as om_query (point phase) with the
 * template descriptor in place of the lattice CNN's.                        */
void om_tpl_query(const om_medium *M, double sigma_t, double albedo, int nl, const double *lw,
                  const double *lg, double lam, double gamma, double radiance, const double *params, int width,
                  int n_linear, const float *pts, const float *dirs, int64_t np,
                  double *L_out, double *y_out, double *fhat_out, double *desc_out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < np; p++) {
        double tb[OM_TPL_SITES], rh[OM_TPL_SITES], ph[OM_TPL_SITES], st[OM_LAYERS * OM_STATS], f0;
        double *desc = desc_out ? desc_out + p * OM_DESC : (double *)malloc(sizeof(double) * OM_DESC);
        om_tpl_features(M, sigma_t, nl, lw, lg, lam, pts + 3 * p, dirs + 3 * p, 1, tb, rh, ph, st, &f0);
        om_tpl_descriptor(tb, rh, ph, st, albedo, desc);
        double y = om_mlp(params, width, n_linear, desc);
        double F = pow(albedo, gamma) * expm1(y);
        L_out[p] = radiance * (f0 + F);
        if (y_out) y_out[p] = y;
        if (fhat_out) fhat_out[p] = F;
        if (!desc_out) free(desc);
    }
}

/* ------------------------------------------------------------------ */
/* The paper's backbone (Sec. III.C.2, Fig. 6) over the template features:
 * six identical modules, one per feature type tau (0 graded transmittance,
 * 1 density, 2 phase) and template group G (diffuse layers 0-7, highlight
 * layers 8-11).  Readings (the paper names the blocks, not their shapes):
 *  - a module carries h, the features of its current layer (h = x_k0, the
 *    n_k0 values of type tau at the group's first layer); step k (k0 <= k <
 *    k1) fuses h with the configuration parameters c = (g, alpha) into
 *    u = [h; c] (n_k + 2 entries) and applies the attention of eq. (24)-(26)
 *    with the standard two-FC excitation: the squeeze is the layer's
 *    8-entry vector v_k of eq. (24), e = sigmoid(S2 ReLU(S1 v_k + e1) + e2)
 *    (S1 2x8, S2 (n_k+2)x2), a = e * u;
 *  - FC-1 brings a to the next layer's size and it is fused (added) with the
 *    next layer's features: y = x_{k+1} + F1 a + f1 (F1 n_{k+1} x (n_k+2));
 *  - FC-2, then fused with that layer's features again:
 *    h = ReLU(F2 y + f2) + x_{k+1} (F2 n_{k+1} x n_{k+1});
 *  - after its last step a module holds n_k1 values (48 diffuse, 8
 *    highlight); per type the two groups merge through a full connection:
 *    m_tau = ReLU(M_tau [h_diffuse; h_highlight] + mb_tau) (64 x 56);
 *  - the multi-layer perceptron is the backbone MLP of the lattice path, its
 *    input [m_T; m_rho; m_phi; g; alpha] (194 entries), zeros up to the
 *    albedo entry at index 1056 (so the albedo enters once, as before).
 * Parameter block (this file's own order): for tau = 0..2, for G = 0..1, for
 * each step: S1[2][8], e1[2], S2[a][2], e2[a], F1[b][a], f1[b], F2[b][b],
 * f2[b] (a = n_k + 2, b = n_{k+1}); then for tau = 0..2: M[64][56], mb[64]. */
#define OM_MOD_HIDDEN 64

static double om_sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* number of doubles of the module block */
int64_t om_modules_size(void)
{
    int64_t sz = 0;
    for (int tau = 0; tau < 3; tau++)
        for (int G = 0; G < 2; G++) {
            int k0 = G ? OM_DIFFUSE : 0, k1 = G ? OM_LAYERS - 1 : OM_DIFFUSE - 1;
            for (int k = k0; k < k1; k++) {
                int a = om_tpl_count[k] + 2, b = om_tpl_count[k + 1];
                sz += 16 + 2 + 2 * a + a + (int64_t)b * a + b + (int64_t)b * b + b;
            }
        }
    return sz + 3 * (OM_MOD_HIDDEN * (om_tpl_count[OM_DIFFUSE - 1] + om_tpl_count[OM_LAYERS - 1]) + OM_MOD_HIDDEN);
}

/* One module (type tau, group G) over the template features; writes the
 * n_k1 values it ends with and returns the parameter pointer past its steps. */
static const double *om_module(const double *w, int tau, int G, const double *feat, const int *base,
                               double g, double alpha, double *hout)
{
    int k0 = G ? OM_DIFFUSE : 0, k1 = G ? OM_LAYERS - 1 : OM_DIFFUSE - 1;
    double h[64], u[64], av[64], y[64];
    int n0 = om_tpl_count[k0];
    for (int j = 0; j < n0; j++) h[j] = feat[base[k0] + tau * n0 + j];
    for (int k = k0; k < k1; k++) {
        int n = om_tpl_count[k], a = n + 2, b = om_tpl_count[k + 1];
        const double *v = feat + base[k] + 3 * n;              /* squeeze vector of layer k (eq. 24) */
        const double *xn = feat + base[k + 1] + tau * b;       /* next layer's features of type tau */
        const double *S1 = w, *e1 = S1 + 16, *S2 = e1 + 2, *e2 = S2 + 2 * a;
        const double *F1 = e2 + a, *f1 = F1 + (int64_t)b * a, *F2 = f1 + b, *f2 = F2 + (int64_t)b * b;
        w = f2 + b;
        /* fusion with the configuration parameters */
        for (int j = 0; j < n; j++) u[j] = h[j];
        u[n] = g;
        u[n + 1] = alpha;
        /* attention: excitation of the squeeze vector, gate on u */
        double z[2];
        for (int r = 0; r < 2; r++) {
            double acc = e1[r];
            for (int i = 0; i < 8; i++) acc += S1[r * 8 + i] * v[i];
            z[r] = acc > 0.0 ? acc : 0.0;
        }
        for (int i = 0; i < a; i++) av[i] = om_sigmoid(e2[i] + S2[i * 2] * z[0] + S2[i * 2 + 1] * z[1]) * u[i];
        /* FC-1 to the next layer's size, fused with that layer's features */
        for (int o = 0; o < b; o++) {
            double acc = f1[o];
            for (int i = 0; i < a; i++) acc += F1[(int64_t)o * a + i] * av[i];
            y[o] = xn[o] + acc;
        }
        /* FC-2, fused with that layer's features again */
        for (int o = 0; o < b; o++) {
            double acc = f2[o];
            for (int i = 0; i < b; i++) acc += F2[(int64_t)o * b + i] * y[i];
            h[o] = (acc > 0.0 ? acc : 0.0) + xn[o];
        }
    }
    for (int j = 0; j < om_tpl_count[k1]; j++) hout[j] = h[j];
    return w;
}

/* Template features (per layer: tbar, rho, phi in template order, then the
 * squeeze vector, as om_tpl_descriptor lays them out) -> the modules'
 * descriptor: [m_T; m_rho; m_phi; g; alpha], zeros, albedo at OM_DESC - 1. */
void om_modules(const double *mp, const double *feat, double albedo, double *desc)
{
    int base[OM_LAYERS + 1];
    base[0] = 0;
    for (int k = 0; k < OM_LAYERS; k++) base[k + 1] = base[k] + 3 * om_tpl_count[k] + OM_STATS;
    const double g = feat[3 * om_tpl_count[0] + 6], alpha = feat[3 * om_tpl_count[0] + 7];
    const int nd = om_tpl_count[OM_DIFFUSE - 1], nh = om_tpl_count[OM_LAYERS - 1];
    double cat[3][64];
    const double *w = mp;
    for (int tau = 0; tau < 3; tau++) {
        w = om_module(w, tau, 0, feat, base, g, alpha, cat[tau]);
        w = om_module(w, tau, 1, feat, base, g, alpha, cat[tau] + nd);
    }
    for (int i = 0; i < OM_DESC; i++) desc[i] = 0.0;
    for (int tau = 0; tau < 3; tau++) {
        const double *M = w, *mb = M + OM_MOD_HIDDEN * (nd + nh);
        w = mb + OM_MOD_HIDDEN;
        for (int o = 0; o < OM_MOD_HIDDEN; o++) {
            double acc = mb[o];
            for (int i = 0; i < nd + nh; i++) acc += M[o * (nd + nh) + i] * cat[tau][i];
            desc[tau * OM_MOD_HIDDEN + o] = acc > 0.0 ? acc : 0.0;
        }
    }
    desc[3 * OM_MOD_HIDDEN] = g;
    desc[3 * OM_MOD_HIDDEN + 1] = alpha;
    desc[OM_DESC - 1] = albedo;
}

/* Whole query with the paper's templates and backbone: the template
 * features, the six modules and merges, then the backbone MLP and decode. */
void om_tpl_modules_query(const om_medium *M, double sigma_t, double albedo, int nl, const double *lw,
                          const double *lg, double lam, double gamma, double radiance, const double *params,
                          int width, int n_linear, const double *mp, const float *pts, const float *dirs,
                          int64_t np, double *L_out, double *y_out, double *desc_out)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < np; p++) {
        double tb[OM_TPL_SITES], rh[OM_TPL_SITES], ph[OM_TPL_SITES], st[OM_LAYERS * OM_STATS], f0;
        double feat[OM_DESC], desc[OM_DESC];
        om_tpl_features(M, sigma_t, nl, lw, lg, lam, pts + 3 * p, dirs + 3 * p, 1, tb, rh, ph, st, &f0);
        om_tpl_descriptor(tb, rh, ph, st, albedo, feat);
        om_modules(mp, feat, albedo, desc);
        double y = om_mlp(params, width, n_linear, desc);
        L_out[p] = radiance * (f0 + pow(albedo, gamma) * expm1(y));
        if (y_out) y_out[p] = y;
        if (desc_out) memcpy(desc_out + p * OM_DESC, desc, sizeof(desc));
    }
}

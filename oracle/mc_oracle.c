/*
 * mc_oracle.c -- CPU FP64 oracle of the MuCITE ion-pack time step.
 *
 * TEST INFRASTRUCTURE ONLY (see mc_oracle.h).  Plain C11, FP64, glibc libm,
 * built with -O2 -ffp-contract=off; OpenMP over packs inside a step (packs
 * are independent while the space-charge field is frozen, paper "Simulation
 * scope": operator splitting).  Nothing here is blocked, fused or reordered
 * beyond what each cited passage states, so that it can be read against the
 * paper:
 *   - source accumulator and pack emission ............ Eq. 5, "Continuous current Gaussian source"
 *   - field bake E = -grad(phi), Cartesian projection . "Coordinate system..." and Eqs. 3-4
 *   - gas coupling and electrode mask ................. "Gas field and electrode mask coupling"
 *   - CIC deposit, control volumes, cylindrical Poisson  "Axisymmetric PIC space charge update"
 *   - RK4 push, collision rate, IICT adapter, T_eff ... "Particle transport, collisions..." and Eq. 6
 *   - dissociation survival yield ..................... Eq. 7
 *   - terminal classes and exit current ............... "Terminal events..." and Eq. 8
 * Readings taken where the paper is silent are listed with each function.
 */
#include "mc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Exact SI constants and CODATA 2022 values. */
#define KB 1.380649e-23
#define QE 1.602176634e-19
#define HPLANCK 6.62607015e-34
#define NAVO 6.02214076e23
#define EPS0 8.8541878188e-12
#define DALTON 1.66053906892e-27
#define PI 3.14159265358979323846

#define MAX_ION 64
#define MAX_SRC 64

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw,  */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Each round maps   */
/* (c0,c1,c2,c3) with key (k0,k1) to                                         */
/*   (hi(B*c2) ^ c1 ^ k0, lo(B*c2), hi(A*c0) ^ c3 ^ k1, lo(A*c0))            */
/* with A = 0xD2511F53, B = 0xCD9E8D57, and the key is bumped by the Weyl    */
/* constants (0x9E3779B9, 0xBB67AE85) between rounds.                        */
/* Pinned bit-for-bit against an independent library implementation.        */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t pa = (uint64_t)0xD2511F53u * c0;
        uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)pb;
        uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)pa;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One 32-bit word -> uniform in the open interval (0,1). */
static double u01(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

/* Stream layout: counter = (pack id low, step, purpose<<24 | block, pack id high). */
enum { PURPOSE_INJECT = 0, PURPOSE_COLLIDE = 1, PURPOSE_LANGEVIN = 2 };
static void draw(const uint32_t key[2], int64_t id, int64_t step, uint32_t purpose, uint32_t block, uint32_t w[4]) {
    uint32_t ctr[4] = {(uint32_t)((uint64_t)id & 0xffffffffu), (uint32_t)step, (purpose << 24) | block,
                       (uint32_t)((uint64_t)id >> 32)};
    orc_philox4x32_10(ctr, key, w);
}

/* ------------------------------------------------------------------------ */
/* Field bake: E = -grad(phi) on the nodes (the field comes from the baked  */
/* potentials; "Coordinate system, static fields, and RF convention").  Reading: second- */
/* order central differences, one-sided at the outer edges, E_r = 0 on the   */
/* axis (symmetry).  Exact for a potential linear in r or z.                 */
/* Pinned: linear potentials give uniform fields; a quadratic in r gives the  */
/* exact derivative at interior nodes.                                      */
/* ------------------------------------------------------------------------ */
void orc_bake(const double *phi, int32_t nr, int32_t nz, double dr, double dz, double *er, double *ez) {
    for (int32_t j = 0; j < nz; ++j) {
        for (int32_t i = 0; i < nr; ++i) {
            const double *p = phi + (int64_t)j * nr;
            double vr;
            if (i == 0) vr = 0.0;
            else if (i == nr - 1) vr = -(p[i] - p[i - 1]) / dr;
            else vr = -(p[i + 1] - p[i - 1]) / (2.0 * dr);
            double vz;
            if (j == 0) vz = -(phi[(int64_t)1 * nr + i] - phi[i]) / dz;
            else if (j == nz - 1) vz = -(phi[(int64_t)j * nr + i] - phi[(int64_t)(j - 1) * nr + i]) / dz;
            else vz = -(phi[(int64_t)(j + 1) * nr + i] - phi[(int64_t)(j - 1) * nr + i]) / (2.0 * dz);
            er[(int64_t)j * nr + i] = vr;
            ez[(int64_t)j * nr + i] = vz;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Bilinear interpolation of a node table at (r, z) (interpolation of the    */
/* baked tables at the particle position, field and gas sections).  Reading */
/* outside the grid: the cell index and the weights are clamped (constant    */
/* extension).  Pinned: reproduces node values, exact for bilinear fields.   */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t i, j; double f, g; } cell_t;

static cell_t locate(int32_t nr, int32_t nz, double inv_dr, double inv_dz, double r, double z) {
    cell_t c;
    double ur = r * inv_dr, uz = z * inv_dz;
    double fi = floor(ur), fj = floor(uz);
    if (fi < 0.0) fi = 0.0;
    if (fi > (double)(nr - 2)) fi = (double)(nr - 2);
    if (fj < 0.0) fj = 0.0;
    if (fj > (double)(nz - 2)) fj = (double)(nz - 2);
    c.f = ur - fi;
    c.g = uz - fj;
    if (c.f < 0.0) c.f = 0.0;
    if (c.f > 1.0) c.f = 1.0;
    if (c.g < 0.0) c.g = 0.0;
    if (c.g > 1.0) c.g = 1.0;
    c.i = (int64_t)fi;
    c.j = (int64_t)fj;
    return c;
}

static double interp(const double *t, int32_t nr, cell_t c) {
    const double *row0 = t + c.j * nr, *row1 = t + (c.j + 1) * nr;
    return (1.0 - c.f) * (1.0 - c.g) * row0[c.i] + c.f * (1.0 - c.g) * row0[c.i + 1] +
           (1.0 - c.f) * c.g * row1[c.i] + c.f * c.g * row1[c.i + 1];
}

double orc_gather(const double *tab, int32_t nr, int32_t nz, double dr, double dz, double r, double z) {
    return interp(tab, nr, locate(nr, nz, 1.0 / dr, 1.0 / dz, r, z));
}

/* ------------------------------------------------------------------------ */
/* Heat-capacity profile: the paper converts internal energy to an effective */
/* temperature through a heat-capacity profile (IICT paragraph).  Reading:   */
/* Einstein model with s = 3N - 6 oscillators of temperature theta,          */
/*   U(T) = s kB theta / (exp(theta/T) - 1),  T(U) = theta / ln(1 + s kB theta / U). */
/* Pinned: T(U(T)) = T and the classical limit U -> s kB (T - theta/2).      */
/* ------------------------------------------------------------------------ */
double orc_einstein_u(double t, int32_t n_atoms, double theta) {
    double s = 3.0 * n_atoms - 6.0;
    if (t <= 0.0) return 0.0;
    return s * KB * theta / expm1(theta / t);
}

double orc_einstein_t(double e, int32_t n_atoms, double theta) {
    double s = 3.0 * n_atoms - 6.0;
    if (e <= 0.0) return 0.0;
    return theta / log1p(s * KB * theta / e);
}

/* ------------------------------------------------------------------------ */
/* Dissociation rate k(T_eff) of Eq. 7.  Eyring transition-state rate        */
/*   k = (kB T / h) exp(dS/R) exp(-dH/(R T))                                 */
/* (the paper's rate from T_eff, dH and dS), or Arrhenius A exp(-Ea/(kB T)). */
/* Pinned against the closed forms at tabulated temperatures.               */
/* ------------------------------------------------------------------------ */
double orc_rate(int32_t kind, double p1, double p2, double t) {
    if (t <= 0.0 || kind == 0) return 0.0;
    const double R = NAVO * KB;
    if (kind == 1) return (KB * t / HPLANCK) * exp(p2 / R) * exp(-p1 / (R * t));
    return p1 * exp(-(p2 * QE) / (KB * t));
}

/* ------------------------------------------------------------------------ */
/* Discrete sine transform DST-I by its definition,                          */
/*   out[k-1] = sum_{j=1..m} in[j-1] sin(pi k j / (m+1)),  k = 1..m.         */
/* The sine is taken from a table of sin(pi q/(m+1)), q in [0, 2(m+1)), at   */
/* q = (k j) mod 2(m+1) (exact periodicity).  Pinned: DST-I applied twice    */
/* is (m+1)/2 times the identity; single modes map to unit vectors.          */
/* ------------------------------------------------------------------------ */
static double *sine_table(int32_t m) {
    int64_t n2 = 2 * (int64_t)(m + 1);
    double *s = (double *)malloc(sizeof(double) * n2);
    for (int64_t q = 0; q < n2; ++q) s[q] = sin(PI * (double)q / (double)(m + 1));
    return s;
}

static void dst1_with(const double *tab, const double *in, int32_t m, double *out) {
    int64_t n2 = 2 * (int64_t)(m + 1);
    for (int32_t k = 1; k <= m; ++k) {
        double acc = 0.0;
        for (int32_t j = 1; j <= m; ++j) acc += in[j - 1] * tab[((int64_t)k * j) % n2];
        out[k - 1] = acc;
    }
}

void orc_dst1(const double *in, int32_t m, double *out) {
    double *tab = sine_table(m);
    dst1_with(tab, in, m, out);
    free(tab);
}

/* ------------------------------------------------------------------------ */
/* Charge density from the int64 deposit grid (in "Axisymmetric PIC space    */
/* charge update" a node's deposited charge is normalised by the volume of  */
/* its ring-shaped control cell).  The grid holds charge in units of e 2^-32.  Reading:   */
/* the control volume is the finite-volume cell of the radial operator      */
/* below -- the disk of radius dr/2 on the axis, the annulus of width dr    */
/* about r_i elsewhere:                                                     */
/*   V_0 = pi (dr/2)^2 dz,   V_i = 2 pi r_i dr dz (i >= 1),                 */
/* so the solve carries exactly the deposited charge (sum rho_i V_i = sum Q)  */
/* and the discrete Gauss flux through every face equals the deposited     */
/* charge inside it.  (At i >= 1 this volume is also the volume the CIC      */
/* weight of the node covers; on the axis the CIC weight covers             */
/* pi dr^2 dz / 3, so a uniform density reads 4/3 of itself on that node.)  */
/* Pinned: packs deposited on a long grid, solved, give a Gauss flux through */
/* each of the first faces equal to the deposited charge within; uniform    */
/* density reads back at the off-axis nodes.                               */
/* ------------------------------------------------------------------------ */
void orc_rho_from_charge(int32_t nr, int32_t nz, double dr, double dz, const int64_t *q, double *rho) {
    for (int32_t j = 0; j < nz; ++j)
        for (int32_t i = 0; i < nr; ++i) {
            double v = (i == 0) ? PI * (0.5 * dr) * (0.5 * dr) * dz : 2.0 * PI * (i * dr) * dr * dz;
            rho[(int64_t)j * nr + i] = (double)q[(int64_t)j * nr + i] * QE * 0x1p-32 / v;
        }
}

/* ------------------------------------------------------------------------ */
/* Cylindrical finite-volume Poisson equation ("Axisymmetric PIC space      */
/* charge update": the radial operator is a finite-volume balance over ring */
/* cells; dPhi/dr = 0 at r = 0, Phi = 0 at the axial and outer radial       */
/* boundaries).  Unknowns Phi[i][j], 0 <= i <= nr-2, 1 <= j <= nz-2:         */
/*   (A_r Phi)_i + (Phi_{i,j+1} - 2 Phi_{i,j} + Phi_{i,j-1}) / dz^2 = -rho/eps0 */
/*   (A_r Phi)_0 = 4 (Phi_1 - Phi_0) / dr^2              (disk of radius dr/2) */
/*   (A_r Phi)_i = [r_{i+1/2}(Phi_{i+1}-Phi_i) - r_{i-1/2}(Phi_i-Phi_{i-1})] / (r_i dr^2) */
/* This separable direct solver leaves the metal-mask nodes free; the      */
/* masked problem is orc_poisson_masked below.                              */
/* Solve: DST-I along z by definition, one tridiagonal system per sine mode  */
/* with z-eigenvalue -(4/dz^2) sin^2(pi k / (2(nz-1))) (Thomas algorithm),   */
/* inverse DST-I.  Pinned: the 2-D residual, the discrete Gauss law of a     */
/* uniformly charged cylinder, and its analytic field.                       */
/* ------------------------------------------------------------------------ */
void orc_poisson(int32_t nr, int32_t nz, double dr, double dz, const double *rho, double *phi) {
    const int32_t m = nz - 2, nu = nr - 1;
    const double n1 = (double)(nz - 1);
    double *tab = sine_table(m);
    double *bh = (double *)calloc((size_t)nu * m, sizeof(double));
    double *ph = (double *)calloc((size_t)nu * m, sizeof(double));
    /* forward transform of the right-hand side -rho/eps0, row by row */
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < nu; ++i) {
        double *in = (double *)malloc(sizeof(double) * m);
        for (int32_t j = 1; j <= m; ++j) in[j - 1] = -rho[(int64_t)j * nr + i] / EPS0;
        dst1_with(tab, in, m, bh + (int64_t)i * m);
        for (int32_t k = 0; k < m; ++k) bh[(int64_t)i * m + k] *= 2.0 / n1;
        free(in);
    }
    /* one radial tridiagonal system per mode */
#pragma omp parallel for schedule(static)
    for (int32_t k = 1; k <= m; ++k) {
        double sk = sin(PI * k / (2.0 * n1));
        double lam = -(4.0 / (dz * dz)) * sk * sk;
        double *cp = (double *)malloc(sizeof(double) * nu);
        double *dp = (double *)malloc(sizeof(double) * nu);
        for (int32_t i = 0; i < nu; ++i) {
            double lo, di, up;
            if (i == 0) {
                lo = 0.0; di = -4.0 / (dr * dr) + lam; up = 4.0 / (dr * dr);
            } else {
                double ri = i * dr;
                lo = (ri - 0.5 * dr) / (ri * dr * dr);
                up = (ri + 0.5 * dr) / (ri * dr * dr);
                di = -(lo + up) + lam;
            }
            double rhs = bh[(int64_t)i * m + (k - 1)];
            double den = (i == 0) ? di : di - lo * cp[i - 1];
            cp[i] = up / den; /* the last row's upper term multiplies Phi_{nr-1} = 0 */
            dp[i] = (i == 0) ? rhs / den : (rhs - lo * dp[i - 1]) / den;
        }
        double x = 0.0;
        for (int32_t i = nu - 1; i >= 0; --i) {
            x = (i == nu - 1) ? dp[i] : dp[i] - cp[i] * x;
            ph[(int64_t)i * m + (k - 1)] = x;
        }
        free(cp);
        free(dp);
    }
    /* inverse transform; boundary nodes stay at zero */
    memset(phi, 0, sizeof(double) * (size_t)nr * nz);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < nu; ++i) {
        double *out = (double *)malloc(sizeof(double) * m);
        dst1_with(tab, ph + (int64_t)i * m, m, out);
        for (int32_t j = 1; j <= m; ++j) phi[(int64_t)j * nr + i] = out[j - 1];
        free(out);
    }
    free(tab);
    free(bh);
    free(ph);
}

/* ------------------------------------------------------------------------ */
/* The same equation with the metal-mask Dirichlet condition (the space-    */
/* charge section holds the perturbation potential at zero on the mask       */
/* nodes too): Phi = 0 on every mask node among the unknowns, the equation  */
/* above at all others.                                                     */
/* Multiplying row (i, j) by w_i (w_0 = dr/8, w_i = r_i) makes the operator */
/* symmetric; -W L restricted to the non-mask unknowns is symmetric positive */
/* definite and is solved by conjugate gradients.  The preconditioner is the */
/* mask-free direct solver (orc_poisson) applied to the residual with the   */
/* mask entries zeroed -- a compression of an SPD inverse, so SPD on the    */
/* same subspace; it changes only the iteration count, never the solution, */
/* which the matrix-free operator below defines.  Stops when the residual  */
/* of -W L Phi = W rho/eps0 falls below tol times its right-hand side's    */
/* norm.  Returns the iterations used, or -1 without convergence.          */
/* Pinned: an empty mask reproduces orc_poisson; Phi = 0 on the mask and   */
/* the residual vanishes elsewhere; a mask filling a whole z-plane splits   */
/* the problem into two independent boxes solved by orc_poisson; for a    */
/* non-negative charge, 0 <= Phi(masked) <= Phi(no mask) (discrete maximum   */
/* principle).                                                             */
/* ------------------------------------------------------------------------ */
static double fv_weight(int32_t i, double dr) { return i == 0 ? dr / 8.0 : i * dr; }

/* y = -W L x on the unknowns, x = 0 on mask nodes and on the boundary.     */
static void fv_apply(int32_t nr, int32_t nz, double dr, double dz, const uint8_t *mask, const double *x,
                     double *y) {
#pragma omp parallel for schedule(static)
    for (int32_t j = 1; j <= nz - 2; ++j)
        for (int32_t i = 0; i <= nr - 2; ++i) {
            int64_t o = (int64_t)j * nr + i;
            if (mask[o]) {
                y[o] = 0.0;
                continue;
            }
            const double *p = x + (int64_t)j * nr;
            double ar;
            if (i == 0) ar = 4.0 * (p[1] - p[0]) / (dr * dr);
            else {
                double ri = i * dr;
                ar = ((ri + 0.5 * dr) * (p[i + 1] - p[i]) - (ri - 0.5 * dr) * (p[i] - p[i - 1])) / (ri * dr * dr);
            }
            double az = (x[o + nr] - 2.0 * p[i] + x[o - nr]) / (dz * dz);
            y[o] = -fv_weight(i, dr) * (ar + az);
        }
}

static double fv_dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t k = 0; k < n; ++k) s += a[k] * b[k];
    return s;
}

/* z = P r: the mask-free solve of -W L z = r, restricted to non-mask unknowns */
static void fv_precondition(int32_t nr, int32_t nz, double dr, double dz, const uint8_t *mask, const double *r,
                            double *rho, double *z) {
    int64_t nn = (int64_t)nr * nz;
    for (int64_t o = 0; o < nn; ++o) {
        int32_t i = (int32_t)(o % nr), j = (int32_t)(o / nr);
        int unknown = i <= nr - 2 && j >= 1 && j <= nz - 2 && !mask[o];
        /* -W L z = r  <=>  L z = -r / w  <=>  rho / eps0 = r / w */
        rho[o] = unknown ? EPS0 * r[o] / fv_weight(i, dr) : 0.0;
    }
    orc_poisson(nr, nz, dr, dz, rho, z);
    for (int64_t o = 0; o < nn; ++o)
        if (mask[o]) z[o] = 0.0;
}

int32_t orc_poisson_masked(int32_t nr, int32_t nz, double dr, double dz, const double *rho, const uint8_t *mask,
                           double tol, int32_t max_iter, double *phi) {
    int64_t nn = (int64_t)nr * nz;
    double *b = (double *)calloc(nn, sizeof(double)), *r = (double *)calloc(nn, sizeof(double));
    double *z = (double *)calloc(nn, sizeof(double)), *d = (double *)calloc(nn, sizeof(double));
    double *q = (double *)calloc(nn, sizeof(double)), *tmp = (double *)calloc(nn, sizeof(double));
    for (int32_t j = 1; j <= nz - 2; ++j)
        for (int32_t i = 0; i <= nr - 2; ++i) {
            int64_t o = (int64_t)j * nr + i;
            b[o] = mask[o] ? 0.0 : fv_weight(i, dr) * rho[o] / EPS0;
        }
    memset(phi, 0, sizeof(double) * nn);
    memcpy(r, b, sizeof(double) * nn);
    double bn = sqrt(fv_dot(nn, b, b));
    int32_t it = 0, ok = bn == 0.0;
    if (!ok) {
        fv_precondition(nr, nz, dr, dz, mask, r, tmp, z);
        memcpy(d, z, sizeof(double) * nn);
        double rz = fv_dot(nn, r, z);
        for (it = 1; it <= max_iter; ++it) {
            fv_apply(nr, nz, dr, dz, mask, d, q);
            double alpha = rz / fv_dot(nn, d, q);
            for (int64_t o = 0; o < nn; ++o) {
                phi[o] += alpha * d[o];
                r[o] -= alpha * q[o];
            }
            if (sqrt(fv_dot(nn, r, r)) <= tol * bn) {
                ok = 1;
                break;
            }
            fv_precondition(nr, nz, dr, dz, mask, r, tmp, z);
            double rz1 = fv_dot(nn, r, z);
            for (int64_t o = 0; o < nn; ++o) d[o] = z[o] + (rz1 / rz) * d[o];
            rz = rz1;
        }
    }
    free(b); free(r); free(z); free(d); free(q); free(tmp);
    return ok ? it : -1;
}

/* max |L Phi + rho/eps0| / max |rho/eps0| over the unknowns (L as above). */
double orc_poisson_residual(int32_t nr, int32_t nz, double dr, double dz, const double *rho, const double *phi) {
    double num = 0.0, den = 0.0;
    for (int32_t j = 1; j <= nz - 2; ++j)
        for (int32_t i = 0; i <= nr - 2; ++i) {
            const double *p = phi + (int64_t)j * nr;
            double ar;
            if (i == 0) ar = 4.0 * (p[1] - p[0]) / (dr * dr);
            else {
                double ri = i * dr;
                ar = ((ri + 0.5 * dr) * (p[i + 1] - p[i]) - (ri - 0.5 * dr) * (p[i] - p[i - 1])) / (ri * dr * dr);
            }
            double az = (phi[(int64_t)(j + 1) * nr + i] - 2.0 * p[i] + phi[(int64_t)(j - 1) * nr + i]) / (dz * dz);
            double b = -rho[(int64_t)j * nr + i] / EPS0;
            double e = fabs(ar + az - b);
            if (e > num) num = e;
            if (fabs(b) > den) den = fabs(b);
        }
    return den > 0.0 ? num / den : num;
}

/* ------------------------------------------------------------------------ */
/* Impulsive hard-sphere collision with internal-energy exchange (the IICT   */
/* adapter of the collision paragraph).  The paper names improved impulsive  */
/* collision theory but does not print its equations; reading:               */
/*  - centre-of-mass frame of ion (m, v) and gas molecule (mg, vgas):         */
/*    Vcm = (m v + mg vgas)/(m+mg), mu = m mg/(m+mg), Et = mu |g|^2 / 2;      */
/*  - with probability alpha the relative energy is redrawn from the ion's    */
/*    internal bath, Et' ~ Gamma(2, kB T_eff) = -kB T_eff ln(u u'), and the   */
/*    internal energy takes the difference (energy-conserving clamp at 0);    */
/*    otherwise Et' = Et (elastic);                                           */
/*  - isotropic scattering of the relative velocity, |g'| = sqrt(2 Et'/mu).   */
/* Uniforms: u[0] cos(chi), u[1] azimuth, u[2] exchange select, u[3], u[4]   */
/* the Gamma(2) draw.  *exchanged is set when the relative energy was       */
/* redrawn from the bath.                                                   */
/* Pinned: momentum and total (kinetic + internal) energy conservation; the */
/* exchange fraction per accepted collision equals alpha (binomial bound);   */
/* the default alpha equals the head-on elastic transfer fraction derived   */
/* from momentum and energy conservation; the initial relaxation rate of    */
/* E_int in a gas at T, alpha nu 2 kB (T - T_eff), with nu = n sigma <g>;    */
/* the stationary spread sd(T_eff) = sqrt(kB T^2 / C) of a canonical bath.  */
/* The partition against the paper's own adapter (its equations are cited,  */
/* not printed) is parity unpinned.                                         */
/* ------------------------------------------------------------------------ */
void orc_iict_update(double m, double mg, const double v[3], const double vgas[3], double e_int, double t_eff,
                     double alpha, const double u[5], double v_out[3], double vgas_out[3], double *e_int_out,
                     int32_t *clamped, int32_t *exchanged) {
    double M = m + mg, mu = m * mg / M;
    double vcm[3], g[3];
    for (int a = 0; a < 3; ++a) {
        vcm[a] = (m * v[a] + mg * vgas[a]) / M;
        g[a] = v[a] - vgas[a];
    }
    double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    double et = 0.5 * mu * g2, etp = et;
    *clamped = 0;
    *exchanged = 0;
    if (u[2] < alpha) {
        *exchanged = 1;
        etp = -KB * t_eff * log(u[3] * u[4]);
        double e_new = e_int + et - etp;
        if (e_new < 0.0) {
            etp = e_int + et;
            e_new = 0.0;
            *clamped = 1;
        }
        e_int = e_new;
    }
    double cchi = 2.0 * u[0] - 1.0;
    double schi = sqrt(fmax(0.0, 1.0 - cchi * cchi));
    double psi = 2.0 * PI * u[1];
    double gp = sqrt(2.0 * etp / mu);
    double dir[3] = {schi * cos(psi), schi * sin(psi), cchi};
    for (int a = 0; a < 3; ++a) {
        v_out[a] = vcm[a] + (mg / M) * gp * dir[a];
        vgas_out[a] = vcm[a] - (m / M) * gp * dir[a];
    }
    *e_int_out = e_int;
}

/* ------------------------------------------------------------------------ */
/* Stochastic collisions of one pack over one step (Eq. 6 and the explicit   */
/* collision paragraph).  Rate lambda = n_g sigma |v_ion - v_gas| where      */
/* v_gas is the velocity of a gas molecule (flow u plus Maxwellian thermal   */
/* velocity at the local static temperature).  Reading for steps that hold   */
/* many collisions: an exact Poisson process by sequential exponential waits */
/* with thinning.  Candidates come at lambda_c = n sigma (s + abar), s = |v-u|,*/
/* abar = a_g sqrt(8/pi), a_g = sqrt(kB T/mg); the partner's thermal velocity */
/* w is drawn from the mixture (s f(w) + |w| f(w))/(s + abar) of the         */
/* Maxwellian f and its flux-weighted form; the candidate is accepted with   */
/* probability |g|/(s + |w|), g = v - u - w.  Accepted events then occur at  */
/* rate n sigma <|g|> with partners distributed as |g| f(w): the hard-sphere */
/* collision process.  Reduces to the paper's single-collision probability   */
/* when lambda dt << 1.  Pinned: accepted rate against the closed form       */
/* n sigma [a_g sqrt(2/pi) exp(-s^2/2a_g^2) + (s + a_g^2/s) erf(s/(sqrt2 a_g))],*/
/* the partner law, thermalisation and mobility.                            */
/* Partner draw: speed from E = |w|^2 / (2 a_g^2) and an isotropic          */
/* direction; E ~ Gamma(3/2) = -ln u_a - ln u_b cos^2(2 pi u_c) (exponential */
/* plus half a squared normal) for the Maxwellian, E ~ Gamma(2) =            */
/* -ln u_a - ln u_b for the flux-weighted form.                             */
/* Words per candidate c: block 3c = (wait, branch, u_a, u_b), block 3c+1 =  */
/* (u_c, cos theta, azimuth, accept), block 3c+2 = (cos chi, psi, Gamma,     */
/* Gamma), drawn on acceptance; the exchange select is the acceptance        */
/* residual u_acc (s + |w|) / |g|, uniform given acceptance.               */
/* ------------------------------------------------------------------------ */
typedef struct {
    double m, mg, sigma, alpha, theta;
    int32_t n_atoms;
    double n_gas, a_g, abar, u[3];
} coll_env_t;

typedef struct {
    int64_t n_cand, n_acc, n_cap, n_clamp, n_lang, n_exch;
    double sum_g, sum_g2;
} coll_count_t;

static void collide(const coll_env_t *E, const uint32_t key[2], int64_t id, int64_t step, double dt, double v[3],
                    double *e_int, int frozen, coll_count_t *cnt) {
    if (!(E->n_gas > 0.0) || !isfinite(E->n_gas)) return;
    double rel0[3] = {v[0] - E->u[0], v[1] - E->u[1], v[2] - E->u[2]};
    double s0 = sqrt(rel0[0] * rel0[0] + rel0[1] * rel0[1] + rel0[2] * rel0[2]);
    double lam0 = E->n_gas * E->sigma * (s0 + E->abar);
    double nexp = lam0 * dt; /* candidate cap; a non-finite rate ends the loop at once */
    int64_t cap = (nexp < 1e6) ? 64 + 8 * (int64_t)ceil(nexp) : (nexp >= 1e6 ? 8000064 : 0);
    double t_left = dt;
    for (int64_t c = 0;; ++c) {
        if (c == cap) {
            cnt->n_cap++;
            break;
        }
        double rel[3] = {v[0] - E->u[0], v[1] - E->u[1], v[2] - E->u[2]};
        double s = sqrt(rel[0] * rel[0] + rel[1] * rel[1] + rel[2] * rel[2]);
        double lam = E->n_gas * E->sigma * (s + E->abar);
        uint32_t wa[4], wb[4], wc[4];
        draw(key, id, step, PURPOSE_COLLIDE, (uint32_t)(3 * c), wa);
        double tau = -log(u01(wa[0])) / lam;
        if (!(tau < t_left)) break;
        t_left -= tau;
        cnt->n_cand++;
        draw(key, id, step, PURPOSE_COLLIDE, (uint32_t)(3 * c + 1), wb);
        int maxw = u01(wa[1]) < s / (s + E->abar);
        double cc = cos(2.0 * PI * u01(wb[0]));
        double en = -log(u01(wa[2])) - log(u01(wa[3])) * (maxw ? cc * cc : 1.0);
        double wn = E->a_g * sqrt(2.0 * en);
        double ct = 2.0 * u01(wb[1]) - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct));
        double ph = 2.0 * PI * u01(wb[2]);
        double w[3] = {wn * st * cos(ph), wn * st * sin(ph), wn * ct};
        double g[3] = {rel[0] - w[0], rel[1] - w[1], rel[2] - w[2]};
        double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        double uacc = u01(wb[3]);
        if (!(uacc * (s + wn) < gn)) continue;
        cnt->n_acc++;
        cnt->sum_g += gn;
        cnt->sum_g2 += gn * gn;
        if (frozen) continue;
        draw(key, id, step, PURPOSE_COLLIDE, (uint32_t)(3 * c + 2), wc);
        double vgas[3] = {E->u[0] + w[0], E->u[1] + w[1], E->u[2] + w[2]};
        double t_eff = orc_einstein_t(*e_int, E->n_atoms, E->theta);
        double ui[5] = {u01(wc[0]), u01(wc[1]), uacc * (s + wn) / gn, u01(wc[2]), u01(wc[3])};
        double vo[3], vgo[3], eo;
        int32_t clamped, exchanged;
        orc_iict_update(E->m, E->mg, v, vgas, *e_int, t_eff, E->alpha, ui, vo, vgo, &eo, &clamped, &exchanged);
        v[0] = vo[0]; v[1] = vo[1]; v[2] = vo[2];
        *e_int = eo;
        cnt->n_clamp += clamped;
        cnt->n_exch += exchanged;
    }
}

int32_t orc_collision_probe(double m_da, double ccs, double mg_da, double p, double t_gas, const double u[3],
                            const double v[3], double dt, int64_t n_steps, uint64_t seed, orc_probe *out) {
    coll_env_t E;
    memset(&E, 0, sizeof(E));
    E.m = m_da * DALTON;
    E.mg = mg_da * DALTON;
    E.sigma = ccs;
    E.n_gas = p / (KB * t_gas);
    E.a_g = sqrt(KB * t_gas / E.mg);
    E.abar = E.a_g * sqrt(8.0 / PI);
    E.u[0] = u[0]; E.u[1] = u[1]; E.u[2] = u[2];
    E.n_atoms = 3;
    E.theta = 1.0;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    coll_count_t tot;
    memset(&tot, 0, sizeof(tot));
#pragma omp parallel
    {
        coll_count_t loc;
        memset(&loc, 0, sizeof(loc));
#pragma omp for schedule(static)
        for (int64_t n = 0; n < n_steps; ++n) {
            double vv[3] = {v[0], v[1], v[2]}, e = 0.0;
            collide(&E, key, 0, n, dt, vv, &e, 1, &loc);
        }
#pragma omp critical
        {
            tot.n_cand += loc.n_cand; tot.n_acc += loc.n_acc;
            tot.sum_g += loc.sum_g; tot.sum_g2 += loc.sum_g2;
        }
    }
    out->n_cand = tot.n_cand;
    out->n_acc = tot.n_acc;
    out->sum_g = tot.sum_g;
    out->sum_g2 = tot.sum_g2;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Simulation state.                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    orc_ion in;
    double m, qm, alpha, e_int0;
} ion_t;

typedef struct {
    orc_source in;
    double w;
    int64_t w_fx, q_fx, n_real_fx, acc_fx, emitted;
} src_t;

struct orc_sim {
    uint32_t key[2];
    int32_t nr, nz;
    double dr, dz, inv_dr, inv_dz, R;
    int has_fields, has_op;
    double *er_dc, *ez_dc, *er_off, *ez_off, *er_rf, *ez_rf;
    double *gur, *guz, *gp, *gt;
    uint8_t *mask, *hit;
    double *phi_sc, *er_sc, *ez_sc;
    int64_t *qgrid;
    int n_ion, n_src;
    ion_t ion[MAX_ION];
    src_t src[MAX_SRC];
    orc_operating op;
    int64_t step;
    /* packs, kept in emission order for the whole run */
    int64_t n, cap;
    double *x, *y, *z, *vx, *vy, *vz, *eint, *h, *w;
    int64_t *id, *q;
    int32_t *tag, *status;
    /* per-pack exit information */
    int64_t *ex_step;
    int32_t *ex_i, *ex_j;
    double *ex_t, *ex_r;
    /* per-step counters */
    int64_t n_cand, n_coll, n_cap, n_clamp, n_lang, n_exch;
    int64_t emitted_n, emitted_w;
    /* adaptive step (Eq. 1): time, next space-charge time, last step */
    double t, t_next_pic, last_dt;
    /* snapshot records (time-resolved ion distributions) */
    orc_sample *samples;
    int64_t n_samples, cap_samples;
};

static void *xrealloc(void *p, size_t n) { return realloc(p, n ? n : 1); }

static void grow(orc_sim *s, int64_t need) {
    if (need <= s->cap) return;
    int64_t c = s->cap ? s->cap : 1024;
    while (c < need) c *= 2;
#define G(f, T) s->f = (T *)xrealloc(s->f, sizeof(T) * (size_t)c)
    G(x, double); G(y, double); G(z, double); G(vx, double); G(vy, double); G(vz, double);
    G(eint, double); G(h, double); G(w, double); G(id, int64_t); G(q, int64_t);
    G(tag, int32_t); G(status, int32_t); G(ex_step, int64_t); G(ex_i, int32_t); G(ex_j, int32_t);
    G(ex_t, double); G(ex_r, double);
#undef G
    s->cap = c;
}

orc_sim *orc_create(uint64_t seed) {
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->key[0] = (uint32_t)seed;
    s->key[1] = (uint32_t)(seed >> 32);
    return s;
}

void orc_destroy(orc_sim *s) {
    if (!s) return;
    void *fs[] = {s->er_dc, s->ez_dc, s->er_off, s->ez_off, s->er_rf, s->ez_rf, s->gur, s->guz, s->gp, s->gt,
                  s->mask, s->hit, s->phi_sc, s->er_sc, s->ez_sc, s->qgrid, s->x, s->y, s->z, s->vx, s->vy,
                  s->vz, s->eint, s->h, s->w, s->id, s->q, s->tag, s->status, s->ex_step, s->ex_i, s->ex_j,
                  s->ex_t, s->ex_r, s->samples};
    for (size_t k = 0; k < sizeof(fs) / sizeof(fs[0]); ++k) free(fs[k]);
    free(s);
}

static double *dup_or_zero(const double *src, size_t n) {
    double *d = (double *)calloc(n, sizeof(double));
    if (src) memcpy(d, src, n * sizeof(double));
    return d;
}

/* Electrode hit table ("Gas field and electrode mask coupling": a pack is  */
/* lost on an electrode once it is inside a metal cell or nearer the metal   */
/* surface than the hit distance).  Reading: the surface lies half a cell from a metal node,  */
/* so a node is a hit node if it is metal or a metal node lies within         */
/* d_hit + min(dr,dz)/2 of it.                                               */
static void build_hit(orc_sim *s) {
    size_t nn = (size_t)s->nr * s->nz;
    free(s->hit);
    s->hit = (uint8_t *)calloc(nn, 1);
    double reach = s->op.d_hit + 0.5 * fmin(s->dr, s->dz);
    int32_t wi = (int32_t)ceil(reach / s->dr), wj = (int32_t)ceil(reach / s->dz);
    for (int32_t j = 0; j < s->nz; ++j)
        for (int32_t i = 0; i < s->nr; ++i) {
            uint8_t hit = s->mask[(int64_t)j * s->nr + i];
            for (int32_t b = -wj; b <= wj && !hit; ++b)
                for (int32_t a = -wi; a <= wi && !hit; ++a) {
                    int32_t ii = i + a, jj = j + b;
                    if (ii < 0 || jj < 0 || ii >= s->nr || jj >= s->nz) continue;
                    if (!s->mask[(int64_t)jj * s->nr + ii]) continue;
                    double dx = a * s->dr, dy = b * s->dz;
                    if (dx * dx + dy * dy <= reach * reach) hit = 1;
                }
            s->hit[(int64_t)j * s->nr + i] = hit;
        }
}

int32_t orc_load_fields(orc_sim *s, int32_t nr, int32_t nz, double dr, double dz, const double *phi_dc,
                        const double *phi_off, const double *phi_rf, const double *gas_ur, const double *gas_uz,
                        const double *gas_p, const double *gas_t, const uint8_t *mask) {
    if (nr < 3 || nz < 3 || !(dr > 0) || !(dz > 0) || !phi_dc || !gas_p || !gas_t) return -1;
    size_t nn = (size_t)nr * nz;
    s->nr = nr; s->nz = nz; s->dr = dr; s->dz = dz;
    s->inv_dr = 1.0 / dr; s->inv_dz = 1.0 / dz;
    s->R = (nr - 1) * dr;
#define A(f) free(s->f); s->f = (double *)calloc(nn, sizeof(double))
    A(er_dc); A(ez_dc); A(er_off); A(ez_off); A(er_rf); A(ez_rf); A(phi_sc); A(er_sc); A(ez_sc);
#undef A
    orc_bake(phi_dc, nr, nz, dr, dz, s->er_dc, s->ez_dc);
    if (phi_off) orc_bake(phi_off, nr, nz, dr, dz, s->er_off, s->ez_off);
    if (phi_rf) orc_bake(phi_rf, nr, nz, dr, dz, s->er_rf, s->ez_rf);
    free(s->gur); free(s->guz); free(s->gp); free(s->gt); free(s->mask); free(s->qgrid);
    s->gur = dup_or_zero(gas_ur, nn);
    s->guz = dup_or_zero(gas_uz, nn);
    s->gp = dup_or_zero(gas_p, nn);
    s->gt = dup_or_zero(gas_t, nn);
    s->mask = (uint8_t *)calloc(nn, 1);
    if (mask) memcpy(s->mask, mask, nn);
    s->qgrid = (int64_t *)calloc(nn, sizeof(int64_t));
    s->has_fields = 1;
    if (s->has_op) build_hit(s);
    return 0;
}

/* Default exchange probability (reading): the head-on impulsive energy      */
/* transfer fraction to one surface atom, 4 mg ma / (mg + ma)^2, ma = m/N.   */
static void set_alpha(const orc_sim *s, ion_t *I) {
    double mg = s->op.gas_mass_da * DALTON, ma = I->m / I->in.n_atoms;
    I->alpha = I->in.alpha >= 0.0 ? I->in.alpha : 4.0 * mg * ma / ((mg + ma) * (mg + ma));
}

int32_t orc_define_ion(orc_sim *s, const orc_ion *in) {
    if (s->n_ion >= MAX_ION || in->n_atoms < 3 || !(in->mass_da > 0) || in->charge_z == 0) return -1;
    ion_t *I = &s->ion[s->n_ion];
    I->in = *in;
    I->m = in->mass_da * DALTON;
    I->qm = in->charge_z * QE / I->m;
    I->e_int0 = orc_einstein_u(in->t_eff0, in->n_atoms, in->theta_e);
    I->alpha = in->alpha;
    if (s->has_op) set_alpha(s, I);
    return s->n_ion++;
}

/* Fixed-point weights and charges (units of 2^-32 real ions / elementary charges). */
static int64_t fx32(double v) { return llrint(ldexp(v, 32)); }

/* Eq. 5: each step the accumulator receives N_real = I dt / (z e) real ions;
 * a fixed-rate source splits them over its packs_per_step packs.  With the
 * adaptive step this is redone for every step's dt. */
static void source_dt(const orc_sim *s, src_t *S, double dt) {
    double z = (double)s->ion[S->in.ion].in.charge_z;
    double n_real = S->in.current_a * dt / (z * QE);
    if (S->in.kind == 1) S->w = n_real / (double)S->in.packs_per_step;
    else S->w = S->in.weight;
    S->w_fx = fx32(S->w);
    S->q_fx = fx32(z * S->w);
    S->n_real_fx = fx32(n_real);
}

int32_t orc_define_source(orc_sim *s, const orc_source *in) {
    if (s->n_src >= MAX_SRC || in->ion < 0 || in->ion >= s->n_ion || !s->has_op) return -1;
    src_t *S = &s->src[s->n_src];
    memset(S, 0, sizeof(*S));
    S->in = *in;
    source_dt(s, S, s->op.dt);
    return s->n_src++;
}

int32_t orc_set_operating(orc_sim *s, const orc_operating *op) {
    if (!(op->dt > 0) || op->sc_every < 1 || op->n_exit_bins < 1) return -1;
    if (op->langevin_on && !(op->lv_switch >= 0.0)) return -1;
    if (op->sample_every < 0 || op->sample_stride < 0 || !(op->lv_dt_max >= 0.0)) return -1;
    s->op = *op;
    s->has_op = 1;
    for (int k = 0; k < s->n_ion; ++k) set_alpha(s, &s->ion[k]);
    if (s->has_fields) build_hit(s);
    return 0;
}

/* Gas state at a point: flow u projected by Eq. 3 (radial component along  */
/* the pack azimuth, zero on the axis), number density n = p/(kB T).       */
static void gas_at(const orc_sim *s, double x, double y, double z, double u[3], double *p, double *t) {
    double r = sqrt(x * x + y * y);
    cell_t c = locate(s->nr, s->nz, s->inv_dr, s->inv_dz, r, z);
    double ur = interp(s->gur, s->nr, c), uz = interp(s->guz, s->nr, c);
    *p = interp(s->gp, s->nr, c);
    *t = interp(s->gt, s->nr, c);
    if (r > 0.0) {
        u[0] = ur * x / r;
        u[1] = ur * y / r;
    } else {
        u[0] = 0.0;
        u[1] = 0.0;
    }
    u[2] = uz;
}

/* Emission of one pack ("Continuous current Gaussian source": the          */
/* transverse position is drawn from a 2-D Gaussian cut off at a radius).  Reading for the    */
/* synthetic workloads: truncation radius r_trunc, injection at z_inj, and  */
/* velocity = local gas flow + Maxwellian thermal velocity of the ion at the */
/* local gas temperature (stands in for the capillary CFD sampling).         */
/* Words: block 0 = (radius, azimuth, normal pair 1), block 1 = (normal pair 2, -, -). */
static void emit_one(orc_sim *s, const src_t *S, int64_t id, int64_t step, int64_t k) {
    const ion_t *I = &s->ion[S->in.ion];
    uint32_t wa[4], wb[4];
    draw(s->key, id, step, PURPOSE_INJECT, 0, wa);
    draw(s->key, id, step, PURPOSE_INJECT, 1, wb);
    double sg = S->in.sigma_r, rt = S->in.r_trunc;
    double r = sg * sqrt(-2.0 * log(1.0 - u01(wa[0]) * (1.0 - exp(-rt * rt / (2.0 * sg * sg)))));
    double ph = 2.0 * PI * u01(wa[1]);
    double cp = cos(ph), sp = sin(ph);
    double x = r * cp, y = r * sp, z = S->in.z_inj;
    cell_t c = locate(s->nr, s->nz, s->inv_dr, s->inv_dz, r, z);
    double ur = interp(s->gur, s->nr, c), uz = interp(s->guz, s->nr, c), tg = interp(s->gt, s->nr, c);
    double vth = sqrt(KB * tg / I->m);
    double r1 = sqrt(-2.0 * log(u01(wa[2]))), p1 = 2.0 * PI * u01(wa[3]);
    double r2 = sqrt(-2.0 * log(u01(wb[0]))), p2 = 2.0 * PI * u01(wb[1]);
    s->x[k] = x; s->y[k] = y; s->z[k] = z;
    s->vx[k] = ur * cp + vth * r1 * cos(p1);
    s->vy[k] = ur * sp + vth * r1 * sin(p1);
    s->vz[k] = uz + vth * r2 * cos(p2);
    s->eint[k] = I->e_int0;
    s->h[k] = 0.0;
    s->w[k] = S->w;
    s->id[k] = id;
    s->q[k] = S->q_fx;
    s->tag[k] = S->in.ion;
    s->status[k] = ORC_ACTIVE;
    s->ex_step[k] = -1;
}

static void emit(orc_sim *s, int si, int64_t count, int64_t step) {
    src_t *S = &s->src[si];
    if (count <= 0) return;
    grow(s, s->n + count);
    for (int64_t k = 0; k < count; ++k) {
        int64_t id = ((int64_t)si << 32) | (S->emitted + k);
        emit_one(s, S, id, step, s->n + k);
    }
    s->n += count;
    S->emitted += count;
    s->emitted_n += count;
    s->emitted_w += count * S->w_fx;
}

int32_t orc_inject(orc_sim *s, int32_t si, int64_t n) {
    if (si < 0 || si >= s->n_src || !s->has_fields || n < 0) return -1;
    emit(s, si, n, s->step);
    return 0;
}

/* Eq. 5 source accumulator, in integer units of 2^-32 real ions. */
static int64_t due(src_t *S, int64_t step) {
    if (step < S->in.step_start || S->in.kind == 0) return 0;
    int64_t left = S->in.n_total - S->emitted;
    if (left <= 0) return 0;
    int64_t k;
    if (S->in.kind == 1) k = S->in.packs_per_step;
    else {
        S->acc_fx += S->n_real_fx;
        k = S->w_fx > 0 ? S->acc_fx / S->w_fx : 0;
        S->acc_fx -= k * S->w_fx;
    }
    return k < left ? k : left;
}

/* ------------------------------------------------------------------------ */
/* Space-charge update, done at the start of every sc_every-th step from the */
/* current positions (operator splitting: deposit, solve, couple, then the  */
/* field is held while the micro steps run).                                */
/* CIC deposit (bilinear weights to the four surrounding nodes) in int64:    */
/*   a = rint(Q (1-f)), b = Q - a; a0 = rint(a (1-g)), a1 = a - a0;          */
/*   b0 = rint(b (1-g)), b1 = b - b0   ->  (i,j), (i,j+1), (i+1,j), (i+1,j+1) */
/* so every pack deposits exactly its charge.  Pinned: total charge equals   */
/* the charge of the active packs exactly; a pack on a node deposits there.  */
/* ------------------------------------------------------------------------ */
static void deposit(orc_sim *s) {
    memset(s->qgrid, 0, sizeof(int64_t) * (size_t)s->nr * s->nz);
    for (int64_t k = 0; k < s->n; ++k) {
        if (s->status[k] != ORC_ACTIVE) continue;
        if (!isfinite(s->x[k]) || !isfinite(s->y[k]) || !isfinite(s->z[k])) continue;
        double r = sqrt(s->x[k] * s->x[k] + s->y[k] * s->y[k]);
        double ur = r * s->inv_dr, uz = s->z[k] * s->inv_dz;
        double fi = floor(ur), fj = floor(uz);
        if (fi > (double)(s->nr - 2)) fi = (double)(s->nr - 2);
        if (fj > (double)(s->nz - 2)) fj = (double)(s->nz - 2);
        if (fj < 0.0) fj = 0.0;
        double f = ur - fi, g = uz - fj;
        if (f > 1.0) f = 1.0;
        if (g > 1.0) g = 1.0;
        if (g < 0.0) g = 0.0;
        int64_t Q = s->q[k];
        int64_t a = llrint((double)Q * (1.0 - f)), b = Q - a;
        int64_t a0 = llrint((double)a * (1.0 - g)), a1 = a - a0;
        int64_t b0 = llrint((double)b * (1.0 - g)), b1 = b - b0;
        int64_t i = (int64_t)fi, j = (int64_t)fj, nr = s->nr;
        s->qgrid[j * nr + i] += a0;
        s->qgrid[(j + 1) * nr + i] += a1;
        s->qgrid[j * nr + i + 1] += b0;
        s->qgrid[(j + 1) * nr + i + 1] += b1;
    }
}

/* The deposit alone (charge grid only; the potential is left as it was).   */
int32_t orc_deposit(orc_sim *s) {
    deposit(s);
    return 0;
}

int32_t orc_pic_update(orc_sim *s) {
    size_t nn = (size_t)s->nr * s->nz;
    deposit(s);
    double *rho = (double *)malloc(sizeof(double) * nn);
    orc_rho_from_charge(s->nr, s->nz, s->dr, s->dz, s->qgrid, rho);
    if (s->op.sc_mask) {
        if (orc_poisson_masked(s->nr, s->nz, s->dr, s->dz, rho, s->mask, 1e-13, 2000, s->phi_sc) < 0) {
            free(rho);
            return -3;
        }
    } else {
        orc_poisson(s->nr, s->nz, s->dr, s->dz, rho, s->phi_sc);
    }
    orc_bake(s->phi_sc, s->nr, s->nz, s->dr, s->dz, s->er_sc, s->ez_sc);
    free(rho);
    return 0;
}

/* Total field of Eq. 4 at (x, y, z) with RF coefficient c = V_RF cos(...),   */
/* radial part projected by Eq. 3 (no transverse field on the axis).        */
static void efield(const orc_sim *s, double x, double y, double z, double c, double e[3]) {
    double r = sqrt(x * x + y * y);
    cell_t cl = locate(s->nr, s->nz, s->inv_dr, s->inv_dz, r, z);
    double er = interp(s->er_dc, s->nr, cl) + s->op.v_off * interp(s->er_off, s->nr, cl) +
                c * interp(s->er_rf, s->nr, cl) + interp(s->er_sc, s->nr, cl);
    double ez = interp(s->ez_dc, s->nr, cl) + s->op.v_off * interp(s->ez_off, s->nr, cl) +
                c * interp(s->ez_rf, s->nr, cl) + interp(s->ez_sc, s->nr, cl);
    if (r > 0.0) {
        e[0] = er * x / r;
        e[1] = er * y / r;
    } else {
        e[0] = 0.0;
        e[1] = 0.0;
    }
    e[2] = ez;
}

/* ------------------------------------------------------------------------ */
/* Hybrid Langevin branch (collision section; Ermak and Buckholz, ref. 31). */
/* In the dense region the explicit events of a step are replaced by the    */
/* relaxation of the velocity toward the local gas velocity with a          */
/* temperature-dependent random part; T_eff and the hazard are not updated  */
/* in such a step.  Readings:                                               */
/*  - the step is the collision sub-step of the splitting (the RK4 push has */
/*    already applied the field), so the velocity solves                    */
/*    dv = -gamma (v - u) dt + sqrt(2 gamma kB T / m) dW over dt exactly:    */
/*    v' = u + (v - u) e^{-gamma dt} + sqrt(kB T/m (1 - e^{-2 gamma dt})) xi; */
/*  - gamma is the momentum-transfer rate of the same hard-sphere gas at low */
/*    field (first Chapman-Enskog approximation, for which the hard-sphere   */
/*    momentum-transfer cross section equals the CCS):                       */
/*    gamma = (16/3) (n sigma / m) sqrt(mu kB T / (2 pi)),                  */
/*    written with mu/m and kB T/m so single precision cannot underflow;     */
/*  - a pack takes the branch for a step when the branch is on, its z after  */
/*    the push lies in [z_lo, z_hi) (any z when z_hi <= z_lo) and           */
/*    lambda dt >= lv_switch, lambda = n sigma (s + abar) the candidate rate */
/*    of the explicit branch at the post-push velocity;                      */
/*  - xi: Box-Muller normals from one Philox block (purpose 2, block 0):     */
/*    (w0, w1) -> xi_x, xi_y; (w2, w3) -> xi_z.                             */
/* Pinned: gamma against the heavy-ion (Epstein specular) limit            */
/* (4/3) n sigma mg abar / m; the relaxation's mean and variance against   */
/* the Ornstein-Uhlenbeck closed form; equipartition; drift in a uniform   */
/* field equal to (a/gamma)(x/2)coth(x/2), x = gamma dt, the same splitting */
/* factor as the explicit branch; explicit and Langevin low-field drift     */
/* agree.                                                                   */
/* ------------------------------------------------------------------------ */
double orc_langevin_gamma(double m, double mg, double n_sigma, double t_gas) {
    double mu_over_m = mg / (m + mg);
    return (16.0 / 3.0) * n_sigma * sqrt(mu_over_m * (KB * t_gas / m) / (2.0 * PI));
}

void orc_langevin_relax(double m, double gamma, double t_gas, const double u[3], double dt, const double xi[3],
                        double v[3]) {
    double f = exp(-gamma * dt);
    double sd = sqrt((KB * t_gas / m) * (1.0 - f * f));
    for (int a = 0; a < 3; ++a) v[a] = u[a] + (v[a] - u[a]) * f + sd * xi[a];
}

static void langevin_normals(const uint32_t key[2], int64_t id, int64_t step, double xi[3]) {
    uint32_t w[4];
    draw(key, id, step, PURPOSE_LANGEVIN, 0, w);
    double r0 = sqrt(-2.0 * log(u01(w[0]))), r1 = sqrt(-2.0 * log(u01(w[2])));
    xi[0] = r0 * cos(2.0 * PI * u01(w[1]));
    xi[1] = r0 * sin(2.0 * PI * u01(w[1]));
    xi[2] = r1 * cos(2.0 * PI * u01(w[3]));
}

/* One pack, one step: RK4 push, classification, collisions, dissociation.  */
static void advance(orc_sim *s, int64_t k, int64_t step, double t0, double dt, const double cst[3],
                    coll_count_t *cnt) {
    const ion_t *I = &s->ion[s->tag[k]];
    const double qm = I->qm;
    double x0[3] = {s->x[k], s->y[k], s->z[k]}, v0[3] = {s->vx[k], s->vy[k], s->vz[k]};
    /* classical RK4 on (x, v), stages at t, t+dt/2, t+dt/2, t+dt */
    double kx[4][3], kv[4][3], xs[3], e[3];
    for (int st = 0; st < 4; ++st) {
        double hstep = (st == 0) ? 0.0 : (st == 3 ? dt : 0.5 * dt);
        for (int a = 0; a < 3; ++a) {
            xs[a] = (st == 0) ? x0[a] : x0[a] + hstep * kx[st - 1][a];
            kx[st][a] = (st == 0) ? v0[a] : v0[a] + hstep * kv[st - 1][a];
        }
        double c = (st == 0) ? cst[0] : (st == 3 ? cst[2] : cst[1]);
        efield(s, xs[0], xs[1], xs[2], c, e);
        for (int a = 0; a < 3; ++a) kv[st][a] = qm * e[a];
    }
    double x1[3], v1[3];
    for (int a = 0; a < 3; ++a) {
        x1[a] = x0[a] + (dt / 6.0) * (kx[0][a] + 2.0 * kx[1][a] + 2.0 * kx[2][a] + kx[3][a]);
        v1[a] = v0[a] + (dt / 6.0) * (kv[0][a] + 2.0 * kv[1][a] + 2.0 * kv[2][a] + kv[3][a]);
    }
    s->x[k] = x1[0]; s->y[k] = x1[1]; s->z[k] = x1[2];
    s->vx[k] = v1[0]; s->vy[k] = v1[1]; s->vz[k] = v1[2];

    /* terminal classification at the new position (terminal-events section) */
    int cls = ORC_ACTIVE;
    double r1 = sqrt(x1[0] * x1[0] + x1[1] * x1[1]);
    double tcross = 0.0, rcross = 0.0;
    int32_t in = -1, jn = -1;
    int finite = 1;
    for (int a = 0; a < 3; ++a) finite &= isfinite(x1[a]) && isfinite(v1[a]);
    if (!finite) cls = ORC_NUMERIC;
    else if (x1[2] >= s->op.z_det || x1[2] < 0.0) {
        double zp = x1[2] >= s->op.z_det ? s->op.z_det : 0.0;
        double fr = (x1[2] != x0[2]) ? (zp - x0[2]) / (x1[2] - x0[2]) : 1.0;
        double xc = x0[0] + fr * (x1[0] - x0[0]), yc = x0[1] + fr * (x1[1] - x0[1]);
        rcross = sqrt(xc * xc + yc * yc);
        tcross = t0 + fr * dt;
        cls = (x1[2] >= s->op.z_det && rcross <= s->op.r_det) ? ORC_TRANSMITTED : ORC_AXIAL;
    } else if (r1 > s->R) cls = ORC_RADIAL;
    else {
        int32_t ii = (int32_t)floor(r1 * s->inv_dr + 0.5), jj = (int32_t)floor(x1[2] * s->inv_dz + 0.5);
        if (ii < s->nr && jj < s->nz && s->hit[(int64_t)jj * s->nr + ii]) {
            cls = ORC_ELECTRODE;
            in = ii;
            jn = jj;
        }
    }
    if (cls != ORC_ACTIVE) {
        s->status[k] = cls;
        s->ex_step[k] = step;
        s->ex_i[k] = in;
        s->ex_j[k] = jn;
        s->ex_t[k] = tcross;
        s->ex_r[k] = rcross;
        return;
    }

    /* collisions with the gas at the new position */
    if (s->op.collisions_on) {
        coll_env_t E;
        double p, tg;
        gas_at(s, x1[0], x1[1], x1[2], E.u, &p, &tg);
        E.m = I->m;
        E.mg = s->op.gas_mass_da * DALTON;
        E.sigma = I->in.ccs_m2;
        E.alpha = I->alpha;
        E.theta = I->in.theta_e;
        E.n_atoms = I->in.n_atoms;
        E.n_gas = (tg > 0.0) ? p / (KB * tg) : 0.0;
        E.a_g = sqrt(KB * tg / E.mg);
        E.abar = E.a_g * sqrt(8.0 / PI);
        double v[3] = {v1[0], v1[1], v1[2]}, ei = s->eint[k];
        int lv = 0;
        if (s->op.langevin_on && E.n_gas > 0.0 && isfinite(E.n_gas) &&
            (!(s->op.lv_z_hi > s->op.lv_z_lo) || (x1[2] >= s->op.lv_z_lo && x1[2] < s->op.lv_z_hi))) {
            double rel[3] = {v[0] - E.u[0], v[1] - E.u[1], v[2] - E.u[2]};
            double sv = sqrt(rel[0] * rel[0] + rel[1] * rel[1] + rel[2] * rel[2]);
            double lam = E.n_gas * E.sigma * (sv + E.abar);
            lv = lam * s->op.dt >= s->op.lv_switch; /* switch on the reference (largest) step */
        }
        if (lv) {
            double xi[3];
            langevin_normals(s->key, s->id[k], step, xi);
            orc_langevin_relax(E.m, orc_langevin_gamma(E.m, E.mg, E.n_gas * E.sigma, tg), tg, E.u, dt, xi, v);
            cnt->n_lang++;
        } else {
            collide(&E, s->key, s->id[k], step, dt, v, &ei, 0, cnt);
        }
        s->vx[k] = v[0]; s->vy[k] = v[1]; s->vz[k] = v[2];
        s->eint[k] = ei;
        if (lv) return; /* no T_eff or hazard update in an aggregated step */
    }
    /* Eq. 7: hazard H accumulates k(T_eff) dt with the post-collision T_eff */
    double te = orc_einstein_t(s->eint[k], I->in.n_atoms, I->in.theta_e);
    s->h[k] += orc_rate(I->in.act_kind, I->in.act_p1, I->in.act_p2, te) * dt;
}

/* Snapshot of the active packs with id % stride == 0 at the start of `step`. */
static void take_samples(orc_sim *s, int64_t step) {
    for (int64_t k = 0; k < s->n; ++k) {
        if (s->status[k] != ORC_ACTIVE || s->id[k] % s->op.sample_stride != 0) continue;
        if (s->n_samples == s->cap_samples) {
            s->cap_samples = s->cap_samples ? 2 * s->cap_samples : 1024;
            s->samples = (orc_sample *)xrealloc(s->samples, sizeof(orc_sample) * (size_t)s->cap_samples);
        }
        const ion_t *I = &s->ion[s->tag[k]];
        orc_sample *r = &s->samples[s->n_samples++];
        double v2 = s->vx[k] * s->vx[k] + s->vy[k] * s->vy[k] + s->vz[k] * s->vz[k];
        r->id = s->id[k]; r->step = step; r->tag = s->tag[k]; r->pad = 0;
        r->x = s->x[k]; r->y = s->y[k]; r->z = s->z[k];
        r->vx = s->vx[k]; r->vy = s->vy[k]; r->vz = s->vz[k];
        r->ke_ev = 0.5 * I->m * v2 / QE;
        r->t_eff = orc_einstein_t(s->eint[k], I->in.n_atoms, I->in.theta_e);
        r->h = s->h[k]; r->w = s->w[k];
    }
}

static int cmp_sample(const void *a, const void *b) {
    const orc_sample *x = (const orc_sample *)a, *y = (const orc_sample *)b;
    if (x->step != y->step) return x->step < y->step ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

int64_t orc_read_samples(const orc_sim *s, orc_sample *buf, int64_t cap) {
    if (buf && cap > 0) {
        int64_t m = cap < s->n_samples ? cap : s->n_samples;
        memcpy(buf, s->samples, sizeof(orc_sample) * (size_t)m);
        qsort(buf, (size_t)m, sizeof(orc_sample), cmp_sample);
    }
    return s->n_samples;
}

/* ------------------------------------------------------------------------ */
/* Adaptive global step, Eq. 1:                                             */
/*   dt = min(0.05 t_RF, 0.1 tau_collision, dt_acc, dt_CFL, dt_L, dt_rem).   */
/* Readings, per active pack at the start of the step (time t0):            */
/*  - tau_collision = 1/lambda, lambda = n sigma (|v - u| + abar) the       */
/*    candidate rate of the explicit branch, for packs on that branch;     */
/*  - dt_acc = 0.1 (|v - u| + sqrt(kB T/m)) / |a|, a = (q/m) E(x, t0): the  */
/*    velocity change of a step stays within a tenth of the pack's speed   */
/*    relative to the gas plus its thermal speed; a pack with no such speed */
/*    (at rest, no gas) takes sqrt(min(dr, dz)/|a|) instead, the time to    */
/*    move half a spacing from rest;                                       */
/*  - dt_CFL = (1/2) min(dr, dz) / |v| (half the smallest spacing);        */
/*  - dt_L = lv_dt_max while any active pack takes the Langevin branch,     */
/*    whose switch compares lambda with the reference step dt_max;         */
/*  - dt_rem: time left to the next space-charge update, which runs every   */
/*    sc_every * dt_max of simulated time (dt_max = the operating dt, also  */
/*    the largest step);                                                   */
/*  - t_RF = 1/f_RF when an RF amplitude is set.                           */
/* Pinned: each term alone against its closed form, the space-charge       */
/* updates landing on their times, and the time sum.  A space-charge       */
/* update is due once t0 is within 1e-6 dt_max of its time.                */
/* ------------------------------------------------------------------------ */
static double pack_dt_limit(const orc_sim *s, int64_t k, double c0, int *langevin) {
    const ion_t *I = &s->ion[s->tag[k]];
    double x[3] = {s->x[k], s->y[k], s->z[k]}, v[3] = {s->vx[k], s->vy[k], s->vz[k]}, e[3], u[3], p, tg;
    double lim = INFINITY;
    double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (vn > 0.0) lim = fmin(lim, 0.5 * fmin(s->dr, s->dz) / vn);
    efield(s, x[0], x[1], x[2], c0, e);
    double an = fabs(I->qm) * sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    gas_at(s, x[0], x[1], x[2], u, &p, &tg);
    double rel[3] = {v[0] - u[0], v[1] - u[1], v[2] - u[2]};
    double sv = sqrt(rel[0] * rel[0] + rel[1] * rel[1] + rel[2] * rel[2]);
    double vth = tg > 0.0 ? sqrt(KB * tg / I->m) : 0.0;
    if (an > 0.0) lim = fmin(lim, (sv + vth) > 0.0 ? 0.1 * (sv + vth) / an : sqrt(fmin(s->dr, s->dz) / an));
    double n_gas = tg > 0.0 ? p / (KB * tg) : 0.0;
    if (s->op.collisions_on && n_gas > 0.0 && isfinite(n_gas)) {
        double abar = sqrt(KB * tg / (s->op.gas_mass_da * DALTON)) * sqrt(8.0 / PI);
        double lam = n_gas * I->in.ccs_m2 * (sv + abar);
        int in_window = !(s->op.lv_z_hi > s->op.lv_z_lo) || (x[2] >= s->op.lv_z_lo && x[2] < s->op.lv_z_hi);
        if (s->op.langevin_on && in_window && lam * s->op.dt >= s->op.lv_switch) *langevin = 1;
        else if (lam > 0.0) lim = fmin(lim, 0.1 / lam);
    }
    return lim;
}

static double global_dt(orc_sim *s, double t0) {
    double c0 = s->op.v_rf * cos(2.0 * PI * s->op.f_rf * t0 + s->op.phase_rf);
    double dt = s->op.dt, lim = INFINITY;
    int lang = 0;
#pragma omp parallel for reduction(min : lim) reduction(| : lang) schedule(static)
    for (int64_t k = 0; k < s->n; ++k) {
        if (s->status[k] != ORC_ACTIVE) continue;
        int l = 0;
        double v = pack_dt_limit(s, k, c0, &l);
        lim = fmin(lim, v);
        lang |= l;
    }
    dt = fmin(dt, lim);
    if (s->op.v_rf != 0.0 && s->op.f_rf > 0.0) dt = fmin(dt, 0.05 / s->op.f_rf);
    if (lang && s->op.lv_dt_max > 0.0) dt = fmin(dt, s->op.lv_dt_max);
    if (s->op.sc_on) dt = fmin(dt, s->t_next_pic - t0);
    return dt;
}

double orc_current_time(const orc_sim *s) { return s->t; }
double orc_last_dt(const orc_sim *s) { return s->last_dt; }

int32_t orc_step(orc_sim *s, int64_t n_steps) {
    if (!s->has_fields || !s->has_op) return -2;
    for (int64_t it = 0; it < n_steps; ++it) {
        int64_t step = s->step;
        if (s->op.sample_every > 0 && s->op.sample_stride > 0 && step % s->op.sample_every == 0) take_samples(s, step);
        double dt = s->op.dt, t0 = (double)step * s->op.dt;
        if (s->op.adaptive) {
            t0 = s->t;
            const double tol = 1e-6 * s->op.dt;
            if (s->op.sc_on && t0 >= s->t_next_pic - tol) {
                if (orc_pic_update(s) < 0) return -3;
                const double period = s->op.sc_every * s->op.dt;
                while (s->t_next_pic <= t0 + tol) s->t_next_pic += period;
            }
            dt = global_dt(s, t0);
            if (!(dt > 1e-9 * s->op.dt)) return -4; /* step collapsed */
            for (int si = 0; si < s->n_src; ++si) source_dt(s, &s->src[si], dt);
        } else if (s->op.sc_on && step % s->op.sc_every == 0 && orc_pic_update(s) < 0) {
            return -3;
        }
        for (int si = 0; si < s->n_src; ++si) emit(s, si, due(&s->src[si], step), step);
        const double w2 = 2.0 * PI * s->op.f_rf;
        double cst[3] = {s->op.v_rf * cos(w2 * t0 + s->op.phase_rf),
                         s->op.v_rf * cos(w2 * (t0 + 0.5 * dt) + s->op.phase_rf),
                         s->op.v_rf * cos(w2 * (t0 + dt) + s->op.phase_rf)};
        int64_t nc = 0, na = 0, ncap = 0, ncl = 0, nlv = 0, nex = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : nc, na, ncap, ncl, nlv, nex)
        for (int64_t k = 0; k < s->n; ++k) {
            if (s->status[k] != ORC_ACTIVE) continue;
            coll_count_t cnt;
            memset(&cnt, 0, sizeof(cnt));
            advance(s, k, step, t0, dt, cst, &cnt);
            nc += cnt.n_cand;
            na += cnt.n_acc;
            ncap += cnt.n_cap;
            ncl += cnt.n_clamp;
            nlv += cnt.n_lang;
            nex += cnt.n_exch;
        }
        s->n_cand += nc;
        s->n_coll += na;
        s->n_cap += ncap;
        s->n_clamp += ncl;
        s->n_lang += nlv;
        s->n_exch += nex;
        s->last_dt = dt;
        s->t = s->op.adaptive ? t0 + dt : (double)(step + 1) * s->op.dt;
        s->step++;
    }
    return 0;
}

int64_t orc_num_packs(const orc_sim *s) { return s->n; }

int32_t orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
int64_t orc_current_step(const orc_sim *s) { return s->step; }

int32_t orc_read_packs(const orc_sim *s, orc_packs *o) {
    if (o->n < s->n) return -1;
#define C(f, g) if (o->f) memcpy(o->f, s->g, sizeof(*s->g) * (size_t)s->n)
    C(x, x); C(y, y); C(z, z); C(vx, vx); C(vy, vy); C(vz, vz); C(e_int, eint); C(h, h); C(w, w);
    C(id, id); C(q, q); C(tag, tag); C(status, status);
#undef C
    o->n = s->n;
    return 0;
}

/* Replace the population by a snapshot of active packs (parity tests). */
int32_t orc_write_packs(orc_sim *s, const orc_packs *in) {
    s->n = 0;
    grow(s, in->n);
    for (int64_t k = 0; k < in->n; ++k) {
        int32_t t = in->tag[k];
        if (t < 0 || t >= s->n_ion) return -1;
        if (!isfinite(in->x[k]) || !isfinite(in->y[k]) || !isfinite(in->z[k]) || !isfinite(in->vx[k]) ||
            !isfinite(in->vy[k]) || !isfinite(in->vz[k]) || !isfinite(in->e_int[k]) || !isfinite(in->w[k]))
            return -1;
        s->x[k] = in->x[k]; s->y[k] = in->y[k]; s->z[k] = in->z[k];
        s->vx[k] = in->vx[k]; s->vy[k] = in->vy[k]; s->vz[k] = in->vz[k];
        s->eint[k] = in->e_int[k]; s->h[k] = in->h[k]; s->w[k] = in->w[k];
        s->id[k] = in->id[k]; s->tag[k] = t;
        s->q[k] = fx32((double)s->ion[t].in.charge_z * in->w[k]);
        s->status[k] = ORC_ACTIVE;
        s->ex_step[k] = -1;
    }
    s->n = in->n;
    return 0;
}

/* Histogram bins (stated with every result): KE 200 log bins over          */
/* [1e-3, 1e3] eV, T_eff 200 bins over [0, 5000] K, exit radius 100 bins    */
/* over [0, r_det]; index 0 = underflow, last = overflow.                   */
static int bin_ke(double ke_ev) {
    if (!(ke_ev > 0.0)) return 0;
    double u = (log10(ke_ev) + 3.0) * (200.0 / 6.0);
    if (!(u >= 0.0)) return 0;
    if (u >= 200.0) return 201;
    return 1 + (int)floor(u);
}
static int bin_teff(double t) {
    double u = t * (200.0 / 5000.0);
    if (!(u >= 0.0)) return 0;
    if (u >= 200.0) return 201;
    return 1 + (int)floor(u);
}
static int bin_r(double r, double rdet) {
    double u = r / rdet * 100.0;
    if (!(u >= 0.0)) return 0;
    if (u >= 100.0) return 101;
    return 1 + (int)floor(u);
}

int32_t orc_read_tallies(const orc_sim *s, orc_tallies *t) {
    int64_t nn = (int64_t)s->nr * s->nz;
    memset(t->class_n, 0, sizeof(t->class_n));
    memset(t->class_w, 0, sizeof(t->class_w));
    if (t->exit_bins) memset(t->exit_bins, 0, sizeof(int64_t) * (size_t)s->op.n_exit_bins);
    if (t->loss_map) memset(t->loss_map, 0, sizeof(int64_t) * (size_t)nn);
    int64_t *hs[5] = {t->hist_ke, t->hist_teff, t->hist_r, t->act_hist_ke, t->act_hist_teff};
    int hn[5] = {ORC_HIST_KE, ORC_HIST_TEFF, ORC_HIST_R, ORC_HIST_KE, ORC_HIST_TEFF};
    for (int a = 0; a < 5; ++a)
        if (hs[a]) memset(hs[a], 0, sizeof(int64_t) * hn[a]);
    t->exit_overflow = 0;
    t->sum_w_ke_active = t->sum_w_eint_active = t->sum_w_dissoc_terminal = 0.0;
    for (int64_t k = 0; k < s->n; ++k) {
        const ion_t *I = &s->ion[s->tag[k]];
        int64_t wfx = fx32(s->w[k]);
        int cls = s->status[k];
        t->class_n[cls]++;
        t->class_w[cls] += wfx;
        double v2 = s->vx[k] * s->vx[k] + s->vy[k] * s->vy[k] + s->vz[k] * s->vz[k];
        double ke = 0.5 * I->m * v2;
        double te = orc_einstein_t(s->eint[k], I->in.n_atoms, I->in.theta_e);
        if (cls == ORC_ACTIVE) {
            t->sum_w_ke_active += s->w[k] * ke;
            t->sum_w_eint_active += s->w[k] * s->eint[k];
            if (t->act_hist_ke) t->act_hist_ke[bin_ke(ke / QE)] += wfx;
            if (t->act_hist_teff) t->act_hist_teff[bin_teff(te)] += wfx;
            continue;
        }
        t->sum_w_dissoc_terminal += s->w[k] * (-expm1(-s->h[k]));
        if (cls == ORC_ELECTRODE && t->loss_map) t->loss_map[(int64_t)s->ex_j[k] * s->nr + s->ex_i[k]] += wfx;
        if (cls == ORC_TRANSMITTED) {
            /* Eq. 8: exit current bins collect the weights crossing in each bin */
            double u = s->ex_t[k] / s->op.exit_bin_dt;
            if (u >= 0.0 && u < (double)s->op.n_exit_bins) {
                if (t->exit_bins) t->exit_bins[(int64_t)floor(u)] += wfx;
            } else t->exit_overflow += wfx;
            if (t->hist_ke) t->hist_ke[bin_ke(ke / QE)] += wfx;
            if (t->hist_teff) t->hist_teff[bin_teff(te)] += wfx;
            if (t->hist_r) t->hist_r[bin_r(s->ex_r[k], s->op.r_det)] += wfx;
        }
    }
    t->emitted_n = s->emitted_n;
    t->emitted_w = s->emitted_w;
    t->n_cand = s->n_cand;
    t->n_coll = s->n_coll;
    t->n_cap = s->n_cap;
    t->n_clamp = s->n_clamp;
    t->n_langevin = s->n_lang;
    t->n_exchange = s->n_exch;
    return 0;
}

int64_t orc_read_exits(const orc_sim *s, orc_exit *buf, int64_t cap) {
    int64_t m = 0;
    for (int64_t k = 0; k < s->n; ++k) {
        if (s->status[k] == ORC_ACTIVE) continue;
        if (m < cap && buf) {
            const ion_t *I = &s->ion[s->tag[k]];
            orc_exit *e = &buf[m];
            double v2 = s->vx[k] * s->vx[k] + s->vy[k] * s->vy[k] + s->vz[k] * s->vz[k];
            e->id = s->id[k]; e->step = s->ex_step[k]; e->cls = s->status[k];
            e->inode = s->ex_i[k]; e->jnode = s->ex_j[k]; e->tag = s->tag[k];
            e->x = s->x[k]; e->y = s->y[k]; e->z = s->z[k];
            e->vx = s->vx[k]; e->vy = s->vy[k]; e->vz = s->vz[k];
            e->t_cross = s->ex_t[k]; e->r_cross = s->ex_r[k];
            e->ke_ev = 0.5 * I->m * v2 / QE;
            e->t_eff = orc_einstein_t(s->eint[k], I->in.n_atoms, I->in.theta_e);
            e->h = s->h[k]; e->w = s->w[k];
        }
        ++m;
    }
    return m;
}

int32_t orc_read_charge(const orc_sim *s, int64_t *q) {
    memcpy(q, s->qgrid, sizeof(int64_t) * (size_t)s->nr * s->nz);
    return 0;
}

int32_t orc_read_sc(const orc_sim *s, double *phi, double *er, double *ez) {
    size_t nn = (size_t)s->nr * s->nz;
    if (phi) memcpy(phi, s->phi_sc, nn * sizeof(double));
    if (er) memcpy(er, s->er_sc, nn * sizeof(double));
    if (ez) memcpy(ez, s->ez_sc, nn * sizeof(double));
    return 0;
}

int32_t orc_read_hit(const orc_sim *s, uint8_t *hit) {
    if (!s->hit) return -2;
    memcpy(hit, s->hit, (size_t)s->nr * s->nz);
    return 0;
}

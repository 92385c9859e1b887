/*
 * oracle.c -- plain FP64 CPU oracle for the GSCL stencil hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the HIP library it checks.
 *
 * Every function is the plain definition of what it computes: one direct loop
 * nest over the grid points, every neighbour fetched through the boundary rule,
 * every floating-point value in FP64 (inputs are exact upcasts of their stored
 * type), terms accumulated in the order the formula lists them.  Build with
 * -ffp-contract=off so no multiply-add is fused.  OpenMP only splits the
 * outermost loop; each point is computed independently, so thread count does
 * not change any result.  Reductions use pairwise summation.
 *
 * Layout: a grid with extents (nx, ny, nz) is a dense array indexed
 * [k][j][i] = k*ny*nx + j*nx + i, x (index i) unit-stride.  A 2D grid is one
 * plane (nz = 1), or a stack of nz independent planes ("layers") that no stencil
 * crosses.
 *
 * Boundary rule (the halo the stencil shape allows an operator to read around
 * the core element, Section 3): a read outside the interior returns
 *   DIRICHLET (0): a constant boundary value,
 *   PERIODIC  (1): the interior point at the index taken modulo the extent,
 *   CLAMP     (2): the nearest interior point (clamp-to-edge).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_DIRICHLET = 0, ORC_PERIODIC = 1, ORC_CLAMP = 2 };

static long wrap_index(long i, long n, int bc)
{
    if (bc == ORC_PERIODIC) {
        long m = i % n;
        return m < 0 ? m + n : m;
    }
    if (i < 0) return 0;
    if (i >= n) return n - 1;
    return i;
}

/* Value of grid a at interior-relative index (i, j, k) under boundary rule bc. */
static double fetch3(const double *a, long nx, long ny, long nz, long i, long j,
                     long k, int bc, double bcv)
{
    int outside = (i < 0 || i >= nx || j < 0 || j >= ny || k < 0 || k >= nz);
    if (outside) {
        if (bc == ORC_DIRICHLET) return bcv;
        i = wrap_index(i, nx, bc);
        j = wrap_index(j, ny, bc);
        k = wrap_index(k, nz, bc);
    }
    return a[(k * ny + j) * nx + i];
}

/* Same for a stack of independent 2D planes: the layer index k is never
 * shifted, only (i, j) pass through the boundary rule. */
static double fetch2(const double *a, long nx, long ny, long i, long j, long layer,
                     int bc, double bcv)
{
    int outside = (i < 0 || i >= nx || j < 0 || j >= ny);
    if (outside) {
        if (bc == ORC_DIRICHLET) return bcv;
        i = wrap_index(i, nx, bc);
        j = wrap_index(j, ny, bc);
    }
    return a[(layer * ny + j) * nx + i];
}

/* ------------------------------------------------------------------------ */
/* do_all with a generic linear stencil operator (Section 3: an operator reads
 * grids at fixed offsets from the core element and writes the core element of
 * its output grids; Fig. 1b is one instance).
 *
 *   out[o](p) = sum over terms t with tout[t] == o, in list order, of
 *               tw[t] * (tcoef[t] >= 0 ? in[tcoef[t]](p) : 1) * in[tg[t]](p + d_t)
 *
 * in:  nin grids packed back to back, each nx*ny*nz doubles.
 * out: nout grids packed the same way (fully overwritten).
 * A coefficient grid is read at the core element only.                      */
void oracle_linear(int ndim, long nx, long ny, long nz, int nin, const double *in,
                   const int *bc, const double *bcv, int nterms, const int *tg,
                   const int *tdx, const int *tdy, const int *tdz, const double *tw,
                   const int *tcoef, const int *tout, int nout, double *out)
{
    long npts = nx * ny * nz;
    (void)nin;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long p = (k * ny + j) * nx + i;
                for (int o = 0; o < nout; ++o) {
                    double acc = 0.0;
                    for (int t = 0; t < nterms; ++t) {
                        if (tout[t] != o) continue;
                        const double *g = in + (long)tg[t] * npts;
                        double v;
                        if (ndim == 3)
                            v = fetch3(g, nx, ny, nz, i + tdx[t], j + tdy[t], k + tdz[t],
                                       bc[tg[t]], bcv[tg[t]]);
                        else
                            v = fetch2(g, nx, ny, i + tdx[t], j + tdy[t], k, bc[tg[t]],
                                       bcv[tg[t]]);
                        double c = 1.0;
                        if (tcoef[t] >= 0) c = in[(long)tcoef[t] * npts + p];
                        acc = acc + tw[t] * c * v;
                    }
                    out[(long)o * npts + p] = acc;
                }
            }
}

/* ------------------------------------------------------------------------ */
/* One weighted-Jacobi sweep of the constant-coefficient Laplacian (the
 * averaging iteration of Section 5.2, with a right-hand side):
 *
 *   S    = neighbour sum in the order +x, -x, +y, -y [, +z, -z]
 *   avg  = (S - h2 * f) / (2 ndim)
 *   unew = (1 - omega) * u + omega * avg
 *   upd  = unew - u                         (the update, nullable)
 *   res  = f - (S - 2 ndim u) / h2           (residual of the input u, nullable)
 *
 * f may be NULL (f = 0).  ndim = 2 treats the nz planes as independent layers. */
void oracle_wjacobi(int ndim, long nx, long ny, long nz, const double *u,
                    const double *f, double omega, double h2, int bc, double bcv,
                    double *unew, double *upd, double *res)
{
    double nnb = 2.0 * ndim;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long p = (k * ny + j) * nx + i;
                double s;
                if (ndim == 3) {
                    s = fetch3(u, nx, ny, nz, i + 1, j, k, bc, bcv);
                    s = s + fetch3(u, nx, ny, nz, i - 1, j, k, bc, bcv);
                    s = s + fetch3(u, nx, ny, nz, i, j + 1, k, bc, bcv);
                    s = s + fetch3(u, nx, ny, nz, i, j - 1, k, bc, bcv);
                    s = s + fetch3(u, nx, ny, nz, i, j, k + 1, bc, bcv);
                    s = s + fetch3(u, nx, ny, nz, i, j, k - 1, bc, bcv);
                } else {
                    s = fetch2(u, nx, ny, i + 1, j, k, bc, bcv);
                    s = s + fetch2(u, nx, ny, i - 1, j, k, bc, bcv);
                    s = s + fetch2(u, nx, ny, i, j + 1, k, bc, bcv);
                    s = s + fetch2(u, nx, ny, i, j - 1, k, bc, bcv);
                }
                double fv = f ? f[p] : 0.0;
                double avg = (s - h2 * fv) / nnb;
                double un = (1.0 - omega) * u[p] + omega * avg;
                unew[p] = un;
                if (upd) upd[p] = un - u[p];
                if (res) res[p] = fv - (s - nnb * u[p]) / h2;
            }
}

/* ------------------------------------------------------------------------ */
/* One colour pass of red-black (over-)relaxation on the 3D Poisson problem
 * Lap_h u = f (the stateful-stencil use of Section 3: the operator queries
 * the index of the point it updates).  A point (i, j, k) has colour
 * (i + j + k) mod 2; the pass updates the points of colour `colour` in place,
 *   u(p) <- (1 - omega) u(p) + omega (S - h2 f(p)) / 6,
 * S the sum of the 6 neighbours, reads outside the interior giving the
 * Dirichlet value bcv.  Every new value is computed from the values at the
 * start of the pass (the neighbours of a point all have the other colour, so
 * the order of the updates within a colour does not matter).  Nullable
 * outputs at the updated points (0 elsewhere):
 *   upd = new - old,  res = f - (S - 6 u_old) / h2  (residual before the update). */
void oracle_rbgs_pass(long nx, long ny, long nz, double *u, const double *f, double omega,
                      double h2, double bcv, int colour, double *upd, double *res)
{
    long n = nx * ny * nz;
    double *nu = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long p = (k * ny + j) * nx + i;
                nu[p] = u[p];
                if (upd) upd[p] = 0.0;
                if (res) res[p] = 0.0;
                if ((i + j + k) % 2 != colour) continue;
                double s = fetch3(u, nx, ny, nz, i + 1, j, k, ORC_DIRICHLET, bcv);
                s = s + fetch3(u, nx, ny, nz, i - 1, j, k, ORC_DIRICHLET, bcv);
                s = s + fetch3(u, nx, ny, nz, i, j + 1, k, ORC_DIRICHLET, bcv);
                s = s + fetch3(u, nx, ny, nz, i, j - 1, k, ORC_DIRICHLET, bcv);
                s = s + fetch3(u, nx, ny, nz, i, j, k + 1, ORC_DIRICHLET, bcv);
                s = s + fetch3(u, nx, ny, nz, i, j, k - 1, ORC_DIRICHLET, bcv);
                double fv = f ? f[p] : 0.0;
                double avg = (s - h2 * fv) / 6.0;
                double un = (1.0 - omega) * u[p] + omega * avg;
                nu[p] = un;
                if (upd) upd[p] = un - u[p];
                if (res) res[p] = fv - (s - 6.0 * u[p]) / h2;
            }
    memcpy(u, nu, sizeof(double) * (size_t)n);
    free(nu);
}

/* ------------------------------------------------------------------------ */
/* Ordered line iteration spaces (Section 3: do_i_inc ... do_k_dec): along
 * axis `axis` (0 = i, 1 = j, 2 = k) every line is processed cell by cell, in
 * increasing index order for dir = +1 (cell c-1 before c) and decreasing for
 * dir = -1 (cell c+1 before c); different lines are independent.  The
 * element at position c of line (p, q) has the grid offset of (i, j, k) with
 * the axis coordinate c.  `prev` below is the value the operator wrote at the
 * previously processed cell of the line, or the seed before the first cell.
 *
 * oracle_line_recur:   out(c) = a(c) * prev + b(c),   seed = `seed`.
 * oracle_tridiag_fwd:  forward elimination of the Thomas algorithm,
 *   den = di(c) - lo(c) * cp_prev,  cp(c) = up(c) / den,
 *   dp(c) = (rhs(c) - lo(c) * dp_prev) / den,   cp, dp seeded with 0.
 * oracle_tridiag_back: back substitution, x(c) = dp(c) - cp(c) * x_prev,
 *   x seeded with 0 (run in the opposite direction of the elimination). */
static long line_offset(long nx, long ny, int axis, long c, long p, long q)
{
    /* (p, q) are the two other coordinates in (i, j, k) order */
    long i, j, k;
    if (axis == 0) { i = c; j = p; k = q; }
    else if (axis == 1) { i = p; j = c; k = q; }
    else { i = p; j = q; k = c; }
    return (k * ny + j) * nx + i;
}

static void line_extents(long nx, long ny, long nz, int axis, long *len, long *np, long *nq)
{
    if (axis == 0) { *len = nx; *np = ny; *nq = nz; }
    else if (axis == 1) { *len = ny; *np = nx; *nq = nz; }
    else { *len = nz; *np = nx; *nq = ny; }
}

void oracle_line_recur(long nx, long ny, long nz, int axis, int dir, const double *a,
                       const double *b, double seed, double *out)
{
    long len, np, nq;
    line_extents(nx, ny, nz, axis, &len, &np, &nq);
#pragma omp parallel for schedule(static)
    for (long q = 0; q < nq; ++q)
        for (long p = 0; p < np; ++p) {
            double prev = seed;
            for (long s = 0; s < len; ++s) {
                long c = dir > 0 ? s : len - 1 - s;
                long o = line_offset(nx, ny, axis, c, p, q);
                double v = a[o] * prev + b[o];
                out[o] = v;
                prev = v;
            }
        }
}

void oracle_tridiag_fwd(long nx, long ny, long nz, int axis, int dir, const double *lo,
                        const double *di, const double *up, const double *rhs, double *cp,
                        double *dp)
{
    long len, np, nq;
    line_extents(nx, ny, nz, axis, &len, &np, &nq);
#pragma omp parallel for schedule(static)
    for (long q = 0; q < nq; ++q)
        for (long p = 0; p < np; ++p) {
            double cprev = 0.0, dprev = 0.0;
            for (long s = 0; s < len; ++s) {
                long c = dir > 0 ? s : len - 1 - s;
                long o = line_offset(nx, ny, axis, c, p, q);
                double den = di[o] - lo[o] * cprev;
                double cv = up[o] / den;
                double dv = (rhs[o] - lo[o] * dprev) / den;
                cp[o] = cv;
                dp[o] = dv;
                cprev = cv;
                dprev = dv;
            }
        }
}

void oracle_tridiag_back(long nx, long ny, long nz, int axis, int dir, const double *cp,
                         const double *dp, double *x)
{
    long len, np, nq;
    line_extents(nx, ny, nz, axis, &len, &np, &nq);
#pragma omp parallel for schedule(static)
    for (long q = 0; q < nq; ++q)
        for (long p = 0; p < np; ++p) {
            double prev = 0.0;
            for (long s = 0; s < len; ++s) {
                long c = dir > 0 ? s : len - 1 - s;
                long o = line_offset(nx, ny, axis, c, p, q);
                double v = dp[o] - cp[o] * prev;
                x[o] = v;
                prev = v;
            }
        }
}

/* ------------------------------------------------------------------------ */
/* The diamond iteration space (Section 3: cells (i-1, j) and (i, j-1) are
 * processed before cell (i, j); 2D, every layer independent).  Row-major
 * order (j outer, i inner) is one order that respects it, and the operators
 * below read only those two predecessors' new values, so every order that
 * respects it gives these results.
 *
 * oracle_diamond_recur: out(i,j) = a(i,j) out(i-1,j) + b(i,j) out(i,j-1)
 *   + c(i,j), reads before the first row or column giving `seed`.
 * oracle_gs2d: one lexicographic Gauss-Seidel / SOR sweep in place on the 2D
 *   5-point Poisson problem Lap_h u = f with Dirichlet value bcv:
 *   u(i,j) <- (1 - omega) u(i,j) + omega (W + S + E + N - h2 f) / 4, where
 *   W = u(i-1,j) and S = u(i,j-1) are already updated and E = u(i+1,j),
 *   N = u(i,j+1) are not. */
void oracle_diamond_recur(long nx, long ny, long nl, const double *a, const double *b,
                          const double *c, double seed, double *out)
{
#pragma omp parallel for schedule(static)
    for (long l = 0; l < nl; ++l)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long p = (l * ny + j) * nx + i;
                double w = i > 0 ? out[p - 1] : seed;
                double s = j > 0 ? out[p - nx] : seed;
                out[p] = a[p] * w + b[p] * s + c[p];
            }
}

void oracle_gs2d(long nx, long ny, long nl, double *u, const double *f, double omega, double h2,
                 double bcv)
{
#pragma omp parallel for schedule(static)
    for (long l = 0; l < nl; ++l)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long p = (l * ny + j) * nx + i;
                double w = i > 0 ? u[p - 1] : bcv;
                double s = j > 0 ? u[p - nx] : bcv;
                double e = i + 1 < nx ? u[p + 1] : bcv;
                double n = j + 1 < ny ? u[p + nx] : bcv;
                double sum = w + s;
                sum = sum + e;
                sum = sum + n;
                double fv = f ? f[p] : 0.0;
                u[p] = (1.0 - omega) * u[p] + omega * ((sum - h2 * fv) / 4.0);
            }
}

/* ------------------------------------------------------------------------ */
/* One sweep of the variable-coefficient 7-point operator over 9 input grids
 * (u, c0..c6, s) writing 3 output grids (Section 2: real codes take 5 to 15
 * grids at once).  Offsets e0 = 0, e1..e6 = +x, -x, +y, -y, +z, -z; c_k is
 * paired with e_k.  All outputs are functions of the input u:
 *
 *   out  = sum_{k=0..6} c_k u(p + e_k)
 *   C    = sum_{k=0..6} c_k
 *   unew = (out + s) / C
 *   r    = s + out - C u
 *   F_d  = ( c_{+d} (u(p+e_d) - u) + c_{-d} (u - u(p-e_d)) ) / 2,  d = x, y, z
 *   Fmag = sqrt(F_x^2 + F_y^2 + F_z^2)
 *
 * c: 7 grids packed back to back.                                           */
void oracle_varcoef7(long nx, long ny, long nz, const double *u, const double *c,
                     const double *s, int bc, double bcv, double *unew, double *r,
                     double *fmag)
{
    long npts = nx * ny * nz;
    static const int ex[7] = {0, 1, -1, 0, 0, 0, 0};
    static const int ey[7] = {0, 0, 0, 1, -1, 0, 0};
    static const int ez[7] = {0, 0, 0, 0, 0, 1, -1};
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long p = (k * ny + j) * nx + i;
                double un[7], ck[7];
                for (int q = 0; q < 7; ++q) {
                    un[q] = fetch3(u, nx, ny, nz, i + ex[q], j + ey[q], k + ez[q], bc, bcv);
                    ck[q] = c[(long)q * npts + p];
                }
                double out = 0.0, csum = 0.0;
                for (int q = 0; q < 7; ++q) {
                    out = out + ck[q] * un[q];
                    csum = csum + ck[q];
                }
                double u0 = un[0];
                unew[p] = (out + s[p]) / csum;
                r[p] = s[p] + out - csum * u0;
                double fx = 0.5 * (ck[1] * (un[1] - u0) + ck[2] * (u0 - un[2]));
                double fy = 0.5 * (ck[3] * (un[3] - u0) + ck[4] * (u0 - un[4]));
                double fz = 0.5 * (ck[5] * (un[5] - u0) + ck[6] * (u0 - un[6]));
                fmag[p] = sqrt(fx * fx + fy * fy + fz * fz);
            }
}

/* ------------------------------------------------------------------------ */
/* Integer image filters on a stack of independent uint8 planes, clamp-to-edge
 * (Section 1: basic image-processing filters are stencil computations):
 *
 *   S   = sum of the 5x5 window centred on the pixel (exact integer)
 *   box = S / 25 rounded to nearest = floor((S + 12) / 25)   (25 is odd, so
 *         S / 25 is never a tie and every round-to-nearest rule agrees)
 *   lap = N + S + E + W - 4 C   (lap_kind 4)   or
 *         sum of the 8 neighbours - 8 C        (lap_kind 8), as int16
 * Both filters read the same raw input.                                     */
void oracle_img(long nlayers, long ny, long nx, const uint8_t *img, int lap_kind,
                uint8_t *box, int16_t *lap)
{
#pragma omp parallel for schedule(static)
    for (long l = 0; l < nlayers; ++l)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                const uint8_t *pl = img + l * ny * nx;
                uint32_t s = 0;
                for (long dj = -2; dj <= 2; ++dj)
                    for (long di = -2; di <= 2; ++di) {
                        long jj = wrap_index(j + dj, ny, ORC_CLAMP);
                        long ii = wrap_index(i + di, nx, ORC_CLAMP);
                        s += pl[jj * nx + ii];
                    }
                box[(l * ny + j) * nx + i] = (uint8_t)((s + 12u) / 25u);
                int32_t c = pl[j * nx + i];
                int32_t acc = 0;
                if (lap_kind == 8) {
                    for (long dj = -1; dj <= 1; ++dj)
                        for (long di = -1; di <= 1; ++di) {
                            if (dj == 0 && di == 0) continue;
                            long jj = wrap_index(j + dj, ny, ORC_CLAMP);
                            long ii = wrap_index(i + di, nx, ORC_CLAMP);
                            acc += pl[jj * nx + ii];
                        }
                    acc -= 8 * c;
                } else {
                    acc += pl[wrap_index(j - 1, ny, ORC_CLAMP) * nx + i];
                    acc += pl[wrap_index(j + 1, ny, ORC_CLAMP) * nx + i];
                    acc += pl[j * nx + wrap_index(i + 1, nx, ORC_CLAMP)];
                    acc += pl[j * nx + wrap_index(i - 1, nx, ORC_CLAMP)];
                    acc -= 4 * c;
                }
                lap[(l * ny + j) * nx + i] = (int16_t)acc;
            }
}

/* ------------------------------------------------------------------------ */
/* Fourth-order 13-point variable-coefficient operator (Section 2: climate and
 * seismic codes combine 5 to 15 grids).  Ten coefficient grids, packed:
 *   c[0] = c0 (mass), c[1..6] = c_{x+}, c_{x-}, c_{y+}, c_{y-}, c_{z+}, c_{z-},
 *   c[7..9] = c_{x2}, c_{y2}, c_{z2} (shared by the +2 and -2 points).
 *
 *   (A u)(p) = c0 u - kappa * sum_{d=x,y,z} [ (4/3) ( c_{d+} (u(p+e_d) - u)
 *                                                   + c_{d-} (u(p-e_d) - u) )
 *                                          - (1/12) c_{d2} (u(p+2e_d) + u(p-2e_d) - 2u) ]
 *
 * Dirichlet boundary (value bcv, normally 0) with halo 2.  With every c = 1
 * this is u - kappa * L4 u, L4 the standard fourth-order Laplacian.          */
void oracle_vc13_apply(long nx, long ny, long nz, const double *u, const double *c,
                       double kappa, double bcv, double *out)
{
    long npts = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nz; ++k)
        for (long j = 0; j < ny; ++j)
            for (long i = 0; i < nx; ++i) {
                long p = (k * ny + j) * nx + i;
                double uc = u[p];
                double sum = 0.0;
                for (int d = 0; d < 3; ++d) {
                    long dx = d == 0, dy = d == 1, dz = d == 2;
                    double up1 = fetch3(u, nx, ny, nz, i + dx, j + dy, k + dz, ORC_DIRICHLET, bcv);
                    double um1 = fetch3(u, nx, ny, nz, i - dx, j - dy, k - dz, ORC_DIRICHLET, bcv);
                    double up2 = fetch3(u, nx, ny, nz, i + 2 * dx, j + 2 * dy, k + 2 * dz,
                                        ORC_DIRICHLET, bcv);
                    double um2 = fetch3(u, nx, ny, nz, i - 2 * dx, j - 2 * dy, k - 2 * dz,
                                        ORC_DIRICHLET, bcv);
                    double cp = c[(long)(1 + 2 * d) * npts + p];
                    double cm = c[(long)(2 + 2 * d) * npts + p];
                    double c2 = c[(long)(7 + d) * npts + p];
                    double near = cp * (up1 - uc) + cm * (um1 - uc);
                    double far = c2 * (up2 + um2 - 2.0 * uc);
                    sum = sum + ((4.0 / 3.0) * near - (1.0 / 12.0) * far);
                }
                out[p] = c[p] * uc - kappa * sum;
            }
}

/* Diagonal of the operator above: the coefficient of u(p) in (A u)(p),
 *   D = c0 + kappa * sum_d [ (4/3) (c_{d+} + c_{d-}) - (1/6) c_{d2} ].      */
void oracle_vc13_diag(long nx, long ny, long nz, const double *c, double kappa,
                      double *diag)
{
    long npts = nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < npts; ++p) {
        double sum = 0.0;
        for (int d = 0; d < 3; ++d) {
            double cp = c[(long)(1 + 2 * d) * npts + p];
            double cm = c[(long)(2 + 2 * d) * npts + p];
            double c2 = c[(long)(7 + d) * npts + p];
            sum = sum + ((4.0 / 3.0) * (cp + cm) - (1.0 / 6.0) * c2);
        }
        diag[p] = c[p] + kappa * sum;
    }
}

/* ------------------------------------------------------------------------ */
/* Reductions (do_reduce, Section 3: operator values combined by a commutative
 * operator).  Pairwise summation keeps the rounding error near log2(n) ulps. */
static double pairwise_sum(const double *x, long n, int square)
{
    if (n <= 16) {
        double s = 0.0;
        for (long i = 0; i < n; ++i) s = s + (square ? x[i] * x[i] : x[i]);
        return s;
    }
    long h = n / 2;
    return pairwise_sum(x, h, square) + pairwise_sum(x + h, n - h, square);
}

double oracle_sum(const double *x, long n) { return pairwise_sum(x, n, 0); }
double oracle_sumsq(const double *x, long n) { return pairwise_sum(x, n, 1); }

/* Largest |x|; a NaN anywhere makes the result NaN. */
double oracle_maxabs(const double *x, long n)
{
    double m = 0.0;
    for (long i = 0; i < n; ++i) {
        double a = fabs(x[i]);
        if (a != a) return a;
        if (a > m) m = a;
    }
    return m;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

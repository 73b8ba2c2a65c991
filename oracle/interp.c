/*
 * Oracle (test infrastructure only): plain FP64 off-grid interpolation on a
 * periodic 3D grid.  Only tests/, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library; the product path never does.
 *
 * The paper evaluates every off-grid value in its semi-Lagrangian scheme with
 * third-degree polynomials in Lagrange form: four nodes per axis, twelve basis
 * polynomials, a 4x4x4 support (Sec. 2.3.1 "Discretization" and Sec. 3.4
 * "Parallel Algorithms and Computational Kernels").  A trilinear variant
 * (two nodes per axis) is provided as well.
 *
 * Positions are given in cell units: xi = i + disp, where i is the integer
 * grid index and disp the displacement stored per grid point.  The base node
 * is i0 = floor(xi), the local coordinate t = xi - i0 lies in [0,1), and node
 * indices wrap periodically (Euclidean remainder).
 */
#include <math.h>
#include <stddef.h>

static long wrap_index(long i, long n)
{
    long r = i % n;
    return r < 0 ? r + n : r;
}

/* Cubic Lagrange basis on the nodes {-1, 0, 1, 2}, evaluated at t. */
static void cubic_lagrange(double t, double w[4])
{
    w[0] = -t * (t - 1.0) * (t - 2.0) / 6.0;
    w[1] = (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0;
    w[2] = -(t + 1.0) * t * (t - 2.0) / 2.0;
    w[3] = (t + 1.0) * t * (t - 1.0) / 6.0;
}

/* Linear Lagrange basis on the nodes {0, 1}. */
static void linear_lagrange(double t, double w[2])
{
    w[0] = 1.0 - t;
    w[1] = t;
}

/* Value of the periodic interpolant of f at the cell-unit position xi. */
double orc_interp_point(const double *f, const int n[3], const double xi[3], int order)
{
    long base[3];
    double w[3][4];
    int nn, first;
    if (order == 3) {
        nn = 4;
        first = -1;
    } else {
        nn = 2;
        first = 0;
    }
    for (int a = 0; a < 3; ++a) {
        double fl = floor(xi[a]);
        double t = xi[a] - fl;
        base[a] = (long)fl;
        if (order == 3)
            cubic_lagrange(t, w[a]);
        else
            linear_lagrange(t, w[a]);
    }
    double acc = 0.0;
    for (int p = 0; p < nn; ++p) {
        long i1 = wrap_index(base[0] + first + p, n[0]);
        for (int q = 0; q < nn; ++q) {
            long i2 = wrap_index(base[1] + first + q, n[1]);
            for (int r = 0; r < nn; ++r) {
                long i3 = wrap_index(base[2] + first + r, n[2]);
                double wt = w[0][p] * w[1][q] * w[2][r];
                acc += wt * f[(i1 * n[1] + i2) * (long)n[2] + i3];
            }
        }
    }
    return acc;
}

/*
 * out[x] = I[f](x + disp(x)) for every grid point x; disp is a vector field
 * laid out [3][n1][n2][n3] in cell units.
 */
void orc_interp_field(const double *f, const int n[3], const double *disp, int order, double *out)
{
    long N = (long)n[0] * n[1] * n[2];
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < N; ++idx) {
        long i3 = idx % n[2];
        long i2 = (idx / n[2]) % n[1];
        long i1 = idx / ((long)n[1] * n[2]);
        double xi[3] = {(double)i1 + disp[idx], (double)i2 + disp[N + idx],
                        (double)i3 + disp[2 * N + idx]};
        out[idx] = orc_interp_point(f, n, xi, order);
    }
}

/* out[p] = I[f](xi_p) for M arbitrary cell-unit positions xi laid out [M][3]. */
void orc_interp_points(const double *f, const int n[3], const double *xi, long M, int order,
                       double *out)
{
#pragma omp parallel for schedule(static)
    for (long p = 0; p < M; ++p)
        out[p] = orc_interp_point(f, n, xi + 3 * p, order);
}

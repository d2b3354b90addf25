/*
 * Oracle -- TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call,
 * link or load this file; only tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.
 *
 * Plain FP64 direct evaluation of the retarded Lorenz-gauge 4-potential of one
 * source sub-domain at a list of target points:
 *
 *   P(r, t) = sum_{r' in d_n} h^3 S^I(r', t - |r - r'|/c) / |r - r'|
 *
 * This is the quadrature of the 4-potential integral (Eq. "4v potential" and
 * its per-domain form "4v potential multi"; grid quadrature with weight h^3 as
 * in the space-time sampled form of the method, Sec. III).  S^I is the
 * piecewise-linear-in-time interpolant of the samples S(r', j dt): the sum of
 * triangle basis functions of the source interpolation (Eq. "space-time sampled
 * four vector sources") is exactly linear interpolation between the two
 * neighbouring samples, and the source equals its ground state S(0) for all
 * times t <= 0.
 *
 * Self cell (target point coincides with a source point, same domain): the
 * paper leaves the singular point to a smoothed Green's function it does not
 * print.  Here the cell of side h around the point is integrated exactly for a
 * source that is constant in space over the cell and linear in time:
 *   int_cell S^I(t_l - |u|/c)/|u| d^3u = w0 S(l) + w1 S(l-1),
 *   w0 = h^2 C1 - h^3/(c dt),  w1 = h^3/(c dt),  S(-1) := S(0),
 * with C1 = int_{[-1/2,1/2]^3} d^3u/|u| supplied by the caller (computed by the
 * oracle's own cubature).  It needs the whole cell inside one time step,
 * h sqrt(3)/2 < c dt.
 *
 * dynamic_only != 0 evaluates the same sum with Delta S = S - S(0) in place of
 * S (the dynamic part of the static + dynamic split, Sec. III).
 *
 * Return: 0 ok; 1 a needed sample lies outside [j0, j1]; 2 self cell with
 * h sqrt(3)/2 >= c dt; 3 self cell requested at a time that is not a step.
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>

static const double *sample_ptr(const double *samples, const double *s0,
                                long j, long j0, long j1, long n4, int *err)
{
    if (j <= 0)
        return s0;
    if (j < j0 || j > j1) {
        *err = 1;
        return s0;
    }
    return samples + (size_t)(j - j0) * (size_t)n4;
}

int rpo_contrib(int n_pts, const double *pts, const long *self_idx,
                int nx, int ny, int nz, const double *origin, double h,
                const double *samples, long j0, long j1, const double *s0,
                double t, double dt, double c, int dynamic_only, double c1,
                double *out)
{
    const long n = (long)nx * ny * nz;
    const long n4 = 4 * n;
    const double h3 = h * h * h;
    const int finite_c = isfinite(c);
    int status = 0;

    /* evaluation time in units of dt; a time within rounding of a step is that
       step exactly, so that with c = inf the samples are hit without
       interpolation */
    double tu = t / dt;
    if (fabs(tu - floor(tu + 0.5)) <= 1e-9 * (fabs(tu) > 1.0 ? fabs(tu) : 1.0))
        tu = floor(tu + 0.5);

    /* self-cell weights */
    double w0 = h * h * c1, w1 = 0.0;
    long lstep = 0;
    if (self_idx) {
        int any_self = 0;
        for (int p = 0; p < n_pts; ++p)
            if (self_idx[p] >= 0)
                any_self = 1;
        if (any_self) {
            if (finite_c) {
                if (h * sqrt(3.0) / 2.0 >= c * dt)
                    return 2;
                w0 = h * h * c1 - h3 / (c * dt);
                w1 = h3 / (c * dt);
            }
            if (tu != floor(tu))
                return 3;
            lstep = (long)tu;
        }
    }

#pragma omp parallel for schedule(dynamic, 1) reduction(max : status)
    for (int p = 0; p < n_pts; ++p) {
        const double px = pts[3 * p], py = pts[3 * p + 1], pz = pts[3 * p + 2];
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        int err = 0;
        const long self = self_idx ? self_idx[p] : -1;
        for (int ix = 0; ix < nx; ++ix) {
            const double dx = px - (origin[0] + h * ix);
            for (int iy = 0; iy < ny; ++iy) {
                const double dy = py - (origin[1] + h * iy);
                for (int iz = 0; iz < nz; ++iz) {
                    const long q = ((long)ix * ny + iy) * nz + iz;
                    if (q == self)
                        continue;
                    const double dz = pz - (origin[2] + h * iz);
                    const double R = sqrt(dx * dx + dy * dy + dz * dz);
                    /* retarded time in units of dt */
                    const double u = finite_c ? tu - R / (c * dt) : tu;
                    double v[4];
                    if (u <= 0.0) {
                        for (int mu = 0; mu < 4; ++mu)
                            v[mu] = dynamic_only ? 0.0 : s0[mu * n + q];
                    } else {
                        const long j = (long)floor(u);
                        const double f = u - (double)j;
                        const double *a = sample_ptr(samples, s0, j, j0, j1, n4, &err);
                        if (f == 0.0) {
                            for (int mu = 0; mu < 4; ++mu)
                                v[mu] = a[mu * n + q] - (dynamic_only ? s0[mu * n + q] : 0.0);
                        } else {
                            const double *b = sample_ptr(samples, s0, j + 1, j0, j1, n4, &err);
                            for (int mu = 0; mu < 4; ++mu)
                                v[mu] = (1.0 - f) * a[mu * n + q] + f * b[mu * n + q]
                                        - (dynamic_only ? s0[mu * n + q] : 0.0);
                        }
                    }
                    for (int mu = 0; mu < 4; ++mu)
                        acc[mu] += h3 * v[mu] / R;
                }
            }
        }
        if (self >= 0) {
            const double *a = sample_ptr(samples, s0, lstep, j0, j1, n4, &err);
            const double *b = sample_ptr(samples, s0, lstep - 1, j0, j1, n4, &err);
            for (int mu = 0; mu < 4; ++mu) {
                double sa = a[mu * n + self], sb = b[mu * n + self];
                if (dynamic_only) {
                    sa -= s0[mu * n + self];
                    sb -= s0[mu * n + self];
                }
                acc[mu] += w0 * sa + w1 * sb;
            }
        }
        for (int mu = 0; mu < 4; ++mu)
            out[4 * p + mu] += acc[mu];
        if (err > status)
            status = err;
    }
    return status;
}

/* Threads used by rpo_contrib (timing control only): n >= 1 sets the count,
 * the return value is the count now in effect. */
int rpo_threads(int n)
{
    if (n >= 1)
        omp_set_num_threads(n);
    return omp_get_max_threads();
}

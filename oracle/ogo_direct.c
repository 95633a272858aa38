/*
 * ORACLE — test infrastructure only.
 *
 * Brute-force direct sum of the short-range TreePM force (paper, "Force
 * evaluation" and "Particle Mesh": the tree side carries the erfc part of
 * the split 1/r = erfc(r/2A)/r + erf(r/2A)/r).  It is the exact result the
 * tree walk approximates.  Written independently of ogo_tree.c: no shared
 * helper, header or table.
 *
 * For target i and every j != i with d = minimg(x_j - x_i), r = |d|:
 *   cutoff mode (r_s > 0): only r^2 < r_cut^2 contributes, and
 *     a_i += G m_j d (r^2 + eps^2)^(-3/2) [erfc(u) + 2u/sqrt(pi) exp(-u^2)]
 *     phi_i -= G m_j erfc(u) / sqrt(r^2 + eps^2),   u = r / (2 r_s);
 *   Newtonian mode (r_s <= 0): every j contributes, with the bracket = 1 and
 *     erfc(u) replaced by 1, and no minimum image.
 * With spline softening (paper, "Force evaluation": the point mass becomes
 * the cubic spline density of support h = 2.8 eps) the factors
 * (r^2 + eps^2)^(-3/2) and (r^2 + eps^2)^(-1/2) become q(r/h)/r^3 and
 * q(r/h)/r + t(r/h)/h, where q is the spline's enclosed mass fraction and
 * t(u) = 32 int_u^1 s f(s) ds its outer shells' potential (f the profile
 * 1 - 6s^2 + 6s^3 below 1/2 and 2(1-s)^3 above, 32 = 4 pi * 8/pi).
 * With per-particle softening lengths (peps, caller order) a pair uses the
 * larger of its two lengths in place of eps.
 */
#include <math.h>
#include <stdint.h>

/* Enclosed mass fraction q(u) = 32 int_0^u s^2 f(s) ds and outer term t(u). */
static void ogo_spline_shells(double u, double *q, double *t)
{
    if (u >= 1.0) {
        *q = 1.0;
        *t = 0.0;
    } else if (u < 0.5) {
        *q = 32.0 / 3.0 * pow(u, 3) - 192.0 / 5.0 * pow(u, 5) + 32.0 * pow(u, 6);
        *t = 14.0 / 5.0 - 16.0 * pow(u, 2) + 48.0 * pow(u, 4) - 192.0 / 5.0 * pow(u, 5);
    } else {
        *q = -1.0 / 15.0 + 64.0 / 3.0 * pow(u, 3) - 48.0 * pow(u, 4) + 192.0 / 5.0 * pow(u, 5)
             - 32.0 / 3.0 * pow(u, 6);
        *t = 16.0 / 5.0 - 32.0 * pow(u, 2) + 64.0 * pow(u, 3) - 48.0 * pow(u, 4)
             + 64.0 / 5.0 * pow(u, 5);
    }
}

void ogo_direct(const double *pos, const double *mass, int64_t n, double box,
                int periodic, double G, double eps, double r_s, double r_cut,
                int softening, const double *peps, const int64_t *targets, int64_t M,
                double *acc3, double *pot, int64_t *nint)
{
    const int cut = r_s > 0.0;
    const double half = 0.5 * box, rc2 = r_cut * r_cut;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < M; ++t) {
        int64_t i = targets[t];
        double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
        int64_t cnt = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = pos[3 * j] - pos[3 * i];
            double dy = pos[3 * j + 1] - pos[3 * i + 1];
            double dz = pos[3 * j + 2] - pos[3 * i + 2];
            if (periodic) {
                dx = dx > half ? dx - box : (dx < -half ? dx + box : dx);
                dy = dy > half ? dy - box : (dy < -half ? dy + box : dy);
                dz = dz > half ? dz - box : (dz < -half ? dz + box : dz);
            }
            double rr = dx * dx + dy * dy + dz * dz;
            double w = 1.0, wp = 1.0;
            if (cut) {
                if (!(rr < rc2)) continue;
                double u = sqrt(rr) / (2.0 * r_s);
                wp = erfc(u);
                w = wp + 2.0 * u / sqrt(M_PI) * exp(-u * u);
            }
            double el = eps;
            if (peps) el = peps[i] > peps[j] ? peps[i] : peps[j];
            const double hs = 2.8 * el;
            double f3, f1; /* softened 1/r^3 and 1/r */
            if (softening == 1 && rr < hs * hs) {
                double r = sqrt(rr), qm, tm;
                ogo_spline_shells(r / hs, &qm, &tm);
                f3 = r > 0.0 ? qm / (rr * r) : 32.0 / 3.0 / (hs * hs * hs);
                f1 = (r > 0.0 ? qm / r : 0.0) + tm / hs;
            } else if (softening == 1) {
                f1 = 1.0 / sqrt(rr);
                f3 = f1 * f1 * f1;
            } else {
                double q = 1.0 / sqrt(rr + el * el);
                f3 = q * q * q;
                f1 = q;
            }
            double g = G * mass[j] * f3 * w;
            ax += g * dx;
            ay += g * dy;
            az += g * dz;
            ph -= G * mass[j] * wp * f1;
            ++cnt;
        }
        acc3[3 * t] = ax;
        acc3[3 * t + 1] = ay;
        acc3[3 * t + 2] = az;
        pot[t] = ph;
        if (nint) nint[t] = cnt;
    }
}

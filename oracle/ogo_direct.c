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
 */
#include <math.h>
#include <stdint.h>

void ogo_direct(const double *pos, const double *mass, int64_t n, double box,
                int periodic, double G, double eps, double r_s, double r_cut,
                const int64_t *targets, int64_t M, double *acc3, double *pot,
                int64_t *nint)
{
    const int cut = r_s > 0.0;
    const double half = 0.5 * box, e2 = eps * eps, rc2 = r_cut * r_cut;
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
            double q = 1.0 / sqrt(rr + e2);
            double g = G * mass[j] * q * q * q * w;
            ax += g * dx;
            ay += g * dy;
            az += g * dz;
            ph -= G * mass[j] * wp * q;
            ++cnt;
        }
        acc3[3 * t] = ax;
        acc3[3 * t + 1] = ay;
        acc3[3 * t + 2] = az;
        pot[t] = ph;
        if (nint) nint[t] = cnt;
    }
}

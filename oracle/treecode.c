/*
 * Kernel sums for the treecode oracle -- TEST INFRASTRUCTURE ONLY (loaded by
 * oracle/treecode.py; shares no code with the HIP library).
 *
 * A treecode replaces the sources of a well-separated cluster by proxy
 * points carrying "generalised" weights: a scalar s and a vector m.  For a
 * real element j the weights are s_j = W_j psi_j and m_j = W_j phi_j nu_j,
 * and the terms of the product (Geng & Jacob, arXiv:1301.5885, Section 2.2,
 * eqs. (eqdbef1)/(eqdbef2)) are
 *     top += K1(x, y) s + K2(x, y; m),   bot += K3(x, y) s + K4(x, y; m),
 * where K2 and K4 depend on the source normal linearly, so
 *     K2(x, y; m) = sum_d K2(x, y; e_d) m_d   (likewise K4)
 * with e_d the unit vectors: the kernels are evaluated with the oracle's own
 * definitions (oracle.c, oracle_pair_kernels) at nu_y = e_x, e_y, e_z.  For a
 * real element this is exactly K2(x, y; nu_j) W_j phi_j.
 */
#include <stdint.h>

void oracle_pair_kernels(const double x[3], const double nux[3],
                         const double y[3], const double nuy[3],
                         double kappa, double eps, double K[4]);

/* For each target t (position tx, normal tn): the sums over sources k of the
 * generalised terms, skipping source k when skip[t] == sid[k] (the self
 * term; pass sid = NULL to skip nothing).  Sources: ys (3 per source),
 * weights s, m (3 per source).  Sums in source order.                      */
void oracle_general_sums(int64_t nt, const double *tx, const double *tn,
                         const int64_t *skip, int64_t ns, const double *ys,
                         const double *s, const double *m, const int64_t *sid,
                         double kappa, double eps, double *top, double *bot)
{
    static const double E[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t t = 0; t < nt; ++t) {
        double st = 0.0, sb = 0.0;
        for (int64_t k = 0; k < ns; ++k) {
            if (sid && skip && sid[k] == skip[t]) continue;
            double K[4];
            double k1 = 0.0, k3 = 0.0, k2m = 0.0, k4m = 0.0;
            for (int d = 0; d < 3; ++d) {
                oracle_pair_kernels(tx + 3 * t, tn + 3 * t, ys + 3 * k, E[d], kappa,
                                    eps, K);
                k1 = K[0];
                k3 = K[2];
                k2m += K[1] * m[3 * k + d];
                k4m += K[3] * m[3 * k + d];
            }
            st += k1 * s[k] + k2m;
            sb += k3 * s[k] + k4m;
        }
        top[t] = st;
        bot[t] = sb;
    }
}

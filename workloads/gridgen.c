/*
 * Input construction for the synthetic workloads: atom-local Becke partition
 * weights and a Gaussian-sum potential sampled at the grid points.
 *
 * Neither routine is part of the integration method itself.  The grid weights
 * w(r) and the potential on the points are inputs of the method (the paper
 * computes w(r) from a partition of unity, Section "Computational Choices in
 * FHI-aims", Becke's scheme; v_eff is produced by the SCF code).  This file
 * exists only because a plain numpy version is too slow for ten million
 * points.  Built with gcc (OpenMP) into workloads/_gridgen.so.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Becke's smoothed step: p(mu) = 1.5 mu - 0.5 mu^3 applied three times,
 * s(mu) = (1 - p(p(p(mu)))) / 2. */
static double becke_step(double mu)
{
    for (int k = 0; k < 3; ++k) mu = 1.5 * mu - 0.5 * mu * mu * mu;
    return 0.5 * (1.0 - mu);
}

/*
 * Atom-local Becke weight of each point's owning atom.
 *   N(r) = { B : |r - R_B| < rp }
 *   P_B  = prod_{C in N(r), C != B} s(mu_BC),  mu_BC = (|r-R_B| - |r-R_C|) / |R_B - R_C|
 *   w_A  = P_A / sum_{B in N(r)} P_B   (0 if A is not in N(r) or the sum is 0)
 * atom_xyz [n_atoms][3], pts [n_points][3], owner [n_points] -> out [n_points].
 * Returns 0 on success, -1 on allocation failure, -2 on coincident atoms.
 */
int gg_becke_owner_weight(int64_t n_atoms, const double* atom_xyz, double rp,
                          int64_t n_points, const double* pts, const int32_t* owner,
                          double* out)
{
    if (n_atoms <= 0) return 0;
    /* inverse inter-atomic distances */
    double* inv_r = (double*)malloc(sizeof(double) * (size_t)n_atoms * (size_t)n_atoms);
    if (!inv_r) return -1;
    int bad = 0;
    for (int64_t b = 0; b < n_atoms; ++b)
        for (int64_t c = 0; c < n_atoms; ++c) {
            double dx = atom_xyz[3 * b] - atom_xyz[3 * c];
            double dy = atom_xyz[3 * b + 1] - atom_xyz[3 * c + 1];
            double dz = atom_xyz[3 * b + 2] - atom_xyz[3 * c + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (b != c && r == 0.0) bad = 1;
            inv_r[b * n_atoms + c] = (b == c) ? 0.0 : 1.0 / r;
        }
    if (bad) { free(inv_r); return -2; }

    /* uniform cell list over the atoms, cell edge rp */
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) { lo[d] = atom_xyz[d]; hi[d] = atom_xyz[d]; }
    for (int64_t a = 0; a < n_atoms; ++a)
        for (int d = 0; d < 3; ++d) {
            double x = atom_xyz[3 * a + d];
            if (x < lo[d]) lo[d] = x;
            if (x > hi[d]) hi[d] = x;
        }
    int64_t nc[3];
    for (int d = 0; d < 3; ++d) {
        nc[d] = (int64_t)floor((hi[d] - lo[d]) / rp) + 1;
        if (nc[d] < 1) nc[d] = 1;
    }
    int64_t ncell = nc[0] * nc[1] * nc[2];
    int64_t* cell_ptr = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    int64_t* cell_atoms = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_atoms);
    int64_t* fill = (int64_t*)calloc((size_t)ncell, sizeof(int64_t));
    if (!cell_ptr || !cell_atoms || !fill) {
        free(inv_r); free(cell_ptr); free(cell_atoms); free(fill); return -1;
    }
    for (int64_t a = 0; a < n_atoms; ++a) {
        int64_t ci[3];
        for (int d = 0; d < 3; ++d) {
            ci[d] = (int64_t)floor((atom_xyz[3 * a + d] - lo[d]) / rp);
            if (ci[d] >= nc[d]) ci[d] = nc[d] - 1;
        }
        cell_ptr[(ci[2] * nc[1] + ci[1]) * nc[0] + ci[0] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) cell_ptr[c + 1] += cell_ptr[c];
    for (int64_t a = 0; a < n_atoms; ++a) {
        int64_t ci[3];
        for (int d = 0; d < 3; ++d) {
            ci[d] = (int64_t)floor((atom_xyz[3 * a + d] - lo[d]) / rp);
            if (ci[d] >= nc[d]) ci[d] = nc[d] - 1;
        }
        int64_t c = (ci[2] * nc[1] + ci[1]) * nc[0] + ci[0];
        cell_atoms[cell_ptr[c] + fill[c]++] = a;
    }
    free(fill);

    int err = 0;
#pragma omp parallel
    {
        int64_t* nb = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_atoms);
        double* dist = (double*)malloc(sizeof(double) * (size_t)n_atoms);
        if (!nb || !dist) {
#pragma omp atomic write
            err = -1;
        }
#pragma omp for schedule(dynamic, 4096)
        for (int64_t p = 0; p < n_points; ++p) {
            if (!nb || !dist) continue;
            const double* r = pts + 3 * p;
            int64_t c0[3], c1[3];
            int empty = 0;
            for (int d = 0; d < 3; ++d) {
                double a0 = floor((r[d] - rp - lo[d]) / rp);
                double a1 = floor((r[d] + rp - lo[d]) / rp);
                if (a1 < 0.0 || a0 > (double)(nc[d] - 1)) { empty = 1; break; }
                c0[d] = a0 < 0.0 ? 0 : (int64_t)a0;
                c1[d] = a1 > (double)(nc[d] - 1) ? nc[d] - 1 : (int64_t)a1;
            }
            double wA = 0.0;
            if (!empty) {
                int64_t cnt = 0, own_slot = -1;
                for (int64_t z = c0[2]; z <= c1[2]; ++z)
                    for (int64_t y = c0[1]; y <= c1[1]; ++y)
                        for (int64_t x = c0[0]; x <= c1[0]; ++x) {
                            int64_t c = (z * nc[1] + y) * nc[0] + x;
                            for (int64_t q = cell_ptr[c]; q < cell_ptr[c + 1]; ++q) {
                                int64_t b = cell_atoms[q];
                                double dx = r[0] - atom_xyz[3 * b];
                                double dy = r[1] - atom_xyz[3 * b + 1];
                                double dz = r[2] - atom_xyz[3 * b + 2];
                                double d = sqrt(dx * dx + dy * dy + dz * dz);
                                if (d < rp) {
                                    if (b == owner[p]) own_slot = cnt;
                                    nb[cnt] = b;
                                    dist[cnt] = d;
                                    ++cnt;
                                }
                            }
                        }
                if (own_slot >= 0) {
                    double sum = 0.0, pown = 0.0;
                    for (int64_t i = 0; i < cnt; ++i) {
                        double prod = 1.0;
                        const double* ir = inv_r + nb[i] * n_atoms;
                        for (int64_t j = 0; j < cnt && prod != 0.0; ++j) {
                            if (j == i) continue;
                            prod *= becke_step((dist[i] - dist[j]) * ir[nb[j]]);
                        }
                        sum += prod;
                        if (i == own_slot) pown = prod;
                    }
                    wA = sum > 0.0 ? pown / sum : 0.0;
                }
            }
            out[p] = wA;
        }
        free(nb);
        free(dist);
    }
    free(inv_r);
    free(cell_ptr);
    free(cell_atoms);
    return err;
}

/* v(r) = sum_g a_g exp(-|r - c_g|^2 / (2 sigma_g^2)); centres [n_g][3]. */
void gg_gaussian_sum(int64_t n_g, const double* amp, const double* centre, const double* sigma,
                     int64_t n_points, const double* pts, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n_points; ++p) {
        const double* r = pts + 3 * p;
        double v = 0.0;
        for (int64_t g = 0; g < n_g; ++g) {
            double dx = r[0] - centre[3 * g];
            double dy = r[1] - centre[3 * g + 1];
            double dz = r[2] - centre[3 * g + 2];
            double s = sigma[g];
            v += amp[g] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * s * s));
        }
        out[p] = v;
    }
}

// CPU check of the host planning code (plan.cpp) for sanitizer builds: descriptor validation,
// octree and cut-plane batches, relevance lists (against brute force), list expansion, spline
// coefficients and execution groups on seeded random point clouds, including coincident points
// and clouds that force the degenerate octree cut.  Built with ASan/UBSan and with TSan (the
// relevance pass runs threads) by tests/test_host_native.py; exits non-zero on a failed check.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "plan.h"

using namespace nao;

#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            std::fprintf(stderr, "CHECK failed at %s:%d: %s\n", __FILE__, __LINE__, #cond); \
            std::exit(1);                                                            \
        }                                                                            \
    } while (0)

struct Desc {
    std::vector<double> axyz, rmin, rcut, samples;
    std::vector<int32_t> spc, shell_ptr, shell_l, shell_rad;
    nao_basis_desc d{};
    void seat()
    {
        d.n_atoms = (int64_t)spc.size();
        d.atom_xyz = axyz.data();
        d.atom_species = spc.data();
        d.n_species = (int32_t)shell_ptr.size() - 1;
        d.species_shell_ptr = shell_ptr.data();
        d.shell_l = shell_l.data();
        d.shell_radial = shell_rad.data();
        d.n_radial = (int32_t)rmin.size();
        d.radial_rmin = rmin.data();
        d.radial_rcut = rcut.data();
        d.radial_samples = samples.data();
    }
};

// Two species: (s, p, d) on radial 0..2 with cutoff 3, (s, f) on radial 3..4 with cutoff 2.
Desc make_desc(std::mt19937_64& rng, int n_atoms, double box)
{
    Desc D;
    std::uniform_real_distribution<double> u(0.0, box);
    for (int a = 0; a < n_atoms; ++a) {
        for (int k = 0; k < 3; ++k) D.axyz.push_back(u(rng));
        D.spc.push_back(a % 2);
    }
    D.shell_ptr = {0, 3, 5};
    D.shell_l = {0, 1, 2, 0, 3};
    D.shell_rad = {0, 1, 2, 3, 4};
    const int nk = 12;
    D.d.n_knots = nk;
    for (int r = 0; r < 5; ++r) {
        D.rmin.push_back(1e-4);
        D.rcut.push_back(r < 3 ? 3.0 : 2.0);
        for (int k = 0; k < nk; ++k) D.samples.push_back(std::cos(0.3 * k + r) * (nk - 1 - k));
    }
    D.seat();
    return D;
}

void check_validation()
{
    std::mt19937_64 rng(1);
    Desc D = make_desc(rng, 3, 4.0);
    HostBasis hb;
    CHECK(load_basis(&D.d, hb).empty());
    CHECK(hb.n_basis == 9 + 8 + 9);  // species 0, 1, 0
    CHECK(!load_basis(nullptr, hb).empty());
    {
        Desc E = D;
        E.shell_l[1] = 4;
        E.seat();
        CHECK(!load_basis(&E.d, hb).empty());
    }
    {
        Desc E = D;
        E.d.n_knots = 3;
        CHECK(!load_basis(&E.d, hb).empty());
    }
    {
        Desc E = D;
        E.rmin[2] = 0.0;
        E.seat();
        CHECK(!load_basis(&E.d, hb).empty());
    }
    {
        Desc E = D;
        E.rcut[0] = 1e-5;
        E.seat();
        CHECK(!load_basis(&E.d, hb).empty());
    }
    {
        Desc E = D;
        E.samples[7] = NAN;
        E.seat();
        CHECK(!load_basis(&E.d, hb).empty());
    }
    {
        Desc E = D;
        E.spc[1] = 2;
        E.seat();
        CHECK(!load_basis(&E.d, hb).empty());
    }
    {
        Desc E = D;
        E.shell_rad[0] = 5;
        E.seat();
        CHECK(!load_basis(&E.d, hb).empty());
    }
    {
        Desc E = D;  // 17 shells in one species
        E.shell_ptr = {0, 17, 17};
        E.shell_l.assign(17, 0);
        E.shell_rad.assign(17, 0);
        E.seat();
        CHECK(!load_basis(&E.d, hb).empty());
    }
    std::printf("validation: ok\n");
}

void check_partition(int64_t n, int32_t max_batch, const std::vector<int64_t>& perm, const std::vector<int64_t>& bp,
                     bool exact_count)
{
    CHECK((int64_t)perm.size() == n);
    CHECK(!bp.empty() && bp.front() == 0 && bp.back() == n);
    std::vector<char> seen(n, 0);
    for (int64_t p : perm) {
        CHECK(p >= 0 && p < n && !seen[p]);
        seen[p] = 1;
    }
    for (size_t b = 0; b + 1 < bp.size(); ++b) {
        CHECK(bp[b + 1] > bp[b] && bp[b + 1] - bp[b] <= max_batch);
        for (int64_t k = bp[b] + 1; k < bp[b + 1]; ++k) CHECK(perm[k] > perm[k - 1]);  // ascending in a batch
    }
    if (exact_count && max_batch >= 2) CHECK((int64_t)bp.size() - 1 == (n + max_batch - 1) / max_batch);
}

void check_plan(int seed, int n_atoms, int64_t n, double box, bool coincident)
{
    std::mt19937_64 rng(seed);
    Desc D = make_desc(rng, n_atoms, box);
    HostBasis hb;
    CHECK(load_basis(&D.d, hb).empty());
    std::uniform_real_distribution<double> u(-1.0, box + 1.0);
    std::vector<double> xyz(3 * n);
    for (int64_t p = 0; p < n; ++p)
        for (int k = 0; k < 3; ++k) xyz[3 * p + k] = coincident && p % 3 ? xyz[3 * (p - p % 3) + k] : u(rng);
    for (int32_t batcher : {0, 1})
        for (int32_t mb : {1, 7, 64, 256}) {
            std::vector<int64_t> perm, bp, ap, lp;
            std::vector<int32_t> at, li;
            make_batches(batcher, xyz.data(), n, mb, perm, bp);
            check_partition(n, mb, perm, bp, batcher == 1);
            relevant_atoms(hb, xyz.data(), perm, bp, ap, at);
            CHECK(ap.size() == bp.size());
            // relevance against brute force
            for (size_t b = 0; b + 1 < bp.size(); ++b) {
                std::vector<int32_t> ref;
                for (int a = 0; a < n_atoms; ++a) {
                    bool rel = false;
                    for (int64_t k = bp[b]; k < bp[b + 1] && !rel; ++k) {
                        const double* p = &xyz[3 * perm[k]];
                        const double dx = p[0] - D.axyz[3 * a], dy = p[1] - D.axyz[3 * a + 1], dz = p[2] - D.axyz[3 * a + 2];
                        const double xx = dx * dx, yy = dy * dy, zz = dz * dz;
                        rel = (xx + yy) + zz < hb.atom_rcut[a] * hb.atom_rcut[a];
                    }
                    if (rel) ref.push_back(a);
                }
                CHECK(std::equal(ref.begin(), ref.end(), at.begin() + ap[b], at.begin() + ap[b + 1]) &&
                      (int64_t)ref.size() == ap[b + 1] - ap[b]);
            }
            expand_lists(hb, ap, at, lp, li);
            for (size_t b = 0; b + 1 < lp.size(); ++b)
                for (int64_t k = lp[b] + 1; k < lp[b + 1]; ++k) CHECK(li[k] > li[k - 1]);
            for (int32_t gm : {0, 16, 100, 256}) {
                std::vector<Unit> units;
                std::vector<int32_t> uat, ucol;
                make_groups(hb, bp, ap, at, gm, units, uat, ucol);
                // every point of a batch with a non-empty list is in exactly one unit whose atoms
                // include the batch's atoms
                std::vector<int> cover(n, 0);
                for (const Unit& un : units) {
                    CHECK(un.n_points >= 1 && un.n_points <= (gm ? gm : 256));
                    std::set<int32_t> ua(uat.begin() + un.atom_begin, uat.begin() + un.atom_begin + un.n_atoms);
                    int32_t col = 0;
                    for (int32_t q = 0; q < un.n_atoms; ++q) {
                        CHECK(ucol[un.atom_begin + q] == col);
                        const int32_t a = uat[un.atom_begin + q];
                        col += (int32_t)(hb.atom_first[a + 1] - hb.atom_first[a]);
                    }
                    CHECK(col == un.m);
                    for (int64_t k = un.point_begin; k < un.point_begin + un.n_points; ++k) {
                        cover[k]++;
                        const int64_t b = std::upper_bound(bp.begin(), bp.end(), k) - bp.begin() - 1;
                        for (int64_t q = ap[b]; q < ap[b + 1]; ++q) CHECK(ua.count(at[q]));
                    }
                }
                for (size_t b = 0; b + 1 < bp.size(); ++b)
                    for (int64_t k = bp[b]; k < bp[b + 1]; ++k) CHECK(cover[k] == (ap[b + 1] > ap[b] ? 1 : 0));
                std::vector<Unit> bu;
                std::vector<int32_t> bat, bcol;
                batch_units(hb, bp, ap, at, 0, (int64_t)bp.size() - 1, bu, bat, bcol);
                CHECK(bu.size() == bp.size() - 1);
            }
        }
    // the knot table holds the samples and the natural spline's M_k / 6: M_0 = M_{N-1} = 0 and
    // M_{k-1} + 4 M_k + M_{k+1} = 6 (y_{k-1} - 2 y_k + y_{k+1}) at every interior knot
    const std::vector<double> c = spline_knots(hb);
    const int nk = hb.n_knots;
    CHECK((int)c.size() == hb.n_radial * nk * 2);
    for (int r = 0; r < hb.n_radial; ++r) {
        const double* q = &c[(size_t)r * nk * 2];
        const double* y = &hb.samples[(size_t)r * nk];
        CHECK(q[1] == 0.0 && q[2 * (nk - 1) + 1] == 0.0);
        for (int k = 0; k < nk; ++k) CHECK(q[2 * k] == y[k]);
        for (int k = 1; k + 1 < nk; ++k) {
            const double lhs = 6.0 * (q[2 * k - 1] + 4.0 * q[2 * k + 1] + q[2 * k + 3]);
            const double rhs = 6.0 * (y[k - 1] - 2.0 * y[k] + y[k + 1]);
            CHECK(std::fabs(lhs - rhs) <= 1e-9 * (1 + std::fabs(rhs)));
        }
    }
}

int main()
{
    check_validation();
    check_plan(11, 5, 900, 6.0, false);
    check_plan(12, 9, 3000, 8.0, true);        // coincident triples: degenerate octree cells
    check_plan(13, 2, 0, 4.0, false);          // no points
    check_plan(14, 40, 20000, 12.0, false);    // enough batches for the threaded relevance pass
    std::printf("plan check: all ok\n");
    return 0;
}

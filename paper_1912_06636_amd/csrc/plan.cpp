// Host-side planning (see plan.h).  Built with -ffp-contract=off: the relevance test
// (dx*dx + dy*dy) + dz*dz < rc*rc must be evaluated exactly in this order, unfused.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

namespace nao {

std::string load_basis(const nao_basis_desc* d, HostBasis& o)
{
    if (!d) return "basis descriptor is NULL";
    if (d->n_atoms < 0) return "n_atoms < 0";
    if (d->n_species < 1) return "n_species < 1";
    if (d->n_radial < 1) return "n_radial < 1";
    if (d->n_knots < 4) return "n_knots < 4";
    if (d->n_atoms > 0 && (!d->atom_xyz || !d->atom_species)) return "atom arrays are NULL";
    if (!d->species_shell_ptr || !d->shell_l || !d->shell_radial || !d->radial_rmin ||
        !d->radial_rcut || !d->radial_samples)
        return "basis arrays are NULL";
    o = HostBasis();
    o.n_atoms = d->n_atoms;
    o.n_species = d->n_species;
    o.n_radial = d->n_radial;
    o.n_knots = d->n_knots;
    o.shell_ptr.assign(d->species_shell_ptr, d->species_shell_ptr + d->n_species + 1);
    if (o.shell_ptr[0] != 0) return "species_shell_ptr[0] != 0";
    for (int32_t s = 0; s < d->n_species; ++s) {
        if (o.shell_ptr[s + 1] < o.shell_ptr[s]) return "species_shell_ptr not non-decreasing";
        if (o.shell_ptr[s + 1] - o.shell_ptr[s] > 16) return "more than 16 shells in a species";
    }
    const int32_t n_shells = o.shell_ptr[d->n_species];
    o.shell_l.assign(d->shell_l, d->shell_l + n_shells);
    o.shell_radial.assign(d->shell_radial, d->shell_radial + n_shells);
    for (int32_t j = 0; j < n_shells; ++j) {
        if (o.shell_l[j] < 0 || o.shell_l[j] > 3) return "shell l outside [0, 3]";
        if (o.shell_radial[j] < 0 || o.shell_radial[j] >= d->n_radial) return "shell radial id out of range";
        o.max_l = std::max(o.max_l, o.shell_l[j]);
    }
    o.rmin.assign(d->radial_rmin, d->radial_rmin + d->n_radial);
    o.rcut.assign(d->radial_rcut, d->radial_rcut + d->n_radial);
    for (int32_t r = 0; r < d->n_radial; ++r) {
        if (!(std::isfinite(o.rmin[r]) && std::isfinite(o.rcut[r]))) return "non-finite rmin/rcut";
        if (!(o.rmin[r] > 0.0)) return "rmin <= 0";
        if (!(o.rcut[r] > o.rmin[r])) return "rcut <= rmin";
    }
    const size_t ns = (size_t)d->n_radial * (size_t)d->n_knots;
    o.samples.assign(d->radial_samples, d->radial_samples + ns);
    for (size_t k = 0; k < ns; ++k)
        if (!std::isfinite(o.samples[k])) return "non-finite radial sample";
    o.atom_xyz.assign(d->atom_xyz, d->atom_xyz + 3 * d->n_atoms);
    o.atom_species.assign(d->atom_species, d->atom_species + d->n_atoms);
    for (double x : o.atom_xyz)
        if (!std::isfinite(x)) return "non-finite atom coordinate";
    o.species_nfn.assign(d->n_species, 0);
    for (int32_t s = 0; s < d->n_species; ++s)
        for (int32_t j = o.shell_ptr[s]; j < o.shell_ptr[s + 1]; ++j) o.species_nfn[s] += 2 * o.shell_l[j] + 1;
    o.atom_first.assign(d->n_atoms + 1, 0);
    o.atom_rcut.assign(d->n_atoms, 0.0);
    for (int64_t a = 0; a < d->n_atoms; ++a) {
        const int32_t s = o.atom_species[a];
        if (s < 0 || s >= d->n_species) return "atom species out of range";
        o.atom_first[a + 1] = o.atom_first[a] + o.species_nfn[s];
        double rc = 0.0;
        for (int32_t j = o.shell_ptr[s]; j < o.shell_ptr[s + 1]; ++j) rc = std::max(rc, o.rcut[o.shell_radial[j]]);
        o.atom_rcut[a] = rc;
    }
    o.n_basis = o.atom_first[d->n_atoms];
    if (o.n_basis > (int64_t)INT32_MAX) return "too many basis functions";
    return "";
}

// ------------------------------------------------------------------------------------------
// octree

namespace {

struct OctreeBuilder {
    const double* xyz;
    int32_t max_batch;
    std::vector<int64_t>& perm;      // working index array (ascending inside every node)
    std::vector<int64_t> tmp;
    std::vector<int64_t>& batch_ptr;

    void emit(int64_t lo, int64_t hi) { (void)lo; batch_ptr.push_back(hi); }

    void node(int64_t lo, int64_t hi, const double* blo, const double* bhi, int depth)
    {
        const int64_t cnt = hi - lo;
        if (cnt <= max_batch) {
            emit(lo, hi);
            return;
        }
        double mid[3];
        bool degenerate = true;
        for (int d = 0; d < 3; ++d) {
            mid[d] = 0.5 * (blo[d] + bhi[d]);
            if (!(mid[d] == blo[d] || mid[d] == bhi[d])) degenerate = false;
        }
        if (depth >= 60 || degenerate) {
            for (int64_t s = lo; s < hi; s += max_batch) emit(s, std::min<int64_t>(s + max_batch, hi));
            return;
        }
        int64_t count[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t k = lo; k < hi; ++k) {
            const double* p = xyz + 3 * perm[k];
            const int c = (p[0] >= mid[0] ? 1 : 0) + (p[1] >= mid[1] ? 2 : 0) + (p[2] >= mid[2] ? 4 : 0);
            ++count[c];
        }
        int64_t off[9];
        off[0] = lo;
        for (int c = 0; c < 8; ++c) off[c + 1] = off[c] + count[c];
        int64_t fill[8];
        for (int c = 0; c < 8; ++c) fill[c] = off[c];
        for (int64_t k = lo; k < hi; ++k) {
            const double* p = xyz + 3 * perm[k];
            const int c = (p[0] >= mid[0] ? 1 : 0) + (p[1] >= mid[1] ? 2 : 0) + (p[2] >= mid[2] ? 4 : 0);
            tmp[fill[c]++] = perm[k];
        }
        std::memcpy(perm.data() + lo, tmp.data() + lo, sizeof(int64_t) * (size_t)cnt);
        for (int c = 0; c < 8; ++c) {
            if (count[c] == 0) continue;
            double clo[3], chi[3];
            for (int d = 0; d < 3; ++d) {
                const bool high = (c >> d) & 1;
                clo[d] = high ? mid[d] : blo[d];
                chi[d] = high ? bhi[d] : mid[d];
            }
            node(off[c], off[c + 1], clo, chi, depth + 1);
        }
    }
};

}  // namespace

void octree_batches(const double* xyz, int64_t n, int32_t max_batch, std::vector<int64_t>& perm,
                    std::vector<int64_t>& batch_ptr)
{
    perm.resize(n);
    for (int64_t k = 0; k < n; ++k) perm[k] = k;
    batch_ptr.assign(1, 0);
    if (n == 0) return;
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) lo[d] = hi[d] = xyz[d];
    for (int64_t k = 0; k < n; ++k)
        for (int d = 0; d < 3; ++d) {
            const double x = xyz[3 * k + d];
            if (x < lo[d]) lo[d] = x;
            if (x > hi[d]) hi[d] = x;
        }
    OctreeBuilder b{xyz, max_batch, perm, std::vector<int64_t>(n), batch_ptr};
    b.node(0, n, lo, hi, 0);
}

namespace {

// Grid-adapted cut-plane partition: a range with more than max_batch points is meant to end
// as k = ceil(count / max_batch) batches; it is cut by the plane normal to its axis of largest
// extent at the point quantile floor(count floor(k/2) / k) under the order (coordinate, index),
// the lower side first.  The lower set is unique under that total order, so nth_element gives
// the same partition as a full sort.
struct CutPlaneBuilder {
    const double* xyz;
    int32_t max_batch;
    std::vector<int64_t>& perm;
    std::vector<int64_t>& batch_ptr;

    void node(int64_t lo, int64_t hi)
    {
        const int64_t m = hi - lo;
        if (m <= max_batch) {
            std::sort(perm.begin() + lo, perm.begin() + hi);
            batch_ptr.push_back(hi);
            return;
        }
        const int64_t k = (m + max_batch - 1) / max_batch;
        double mn[3], mx[3];
        for (int d = 0; d < 3; ++d) mn[d] = mx[d] = xyz[3 * perm[lo] + d];
        for (int64_t q = lo + 1; q < hi; ++q)
            for (int d = 0; d < 3; ++d) {
                const double x = xyz[3 * perm[q] + d];
                if (x < mn[d]) mn[d] = x;
                if (x > mx[d]) mx[d] = x;
            }
        int d = 0;
        double best = mx[0] - mn[0];
        for (int e = 1; e < 3; ++e)
            if (mx[e] - mn[e] > best) {
                best = mx[e] - mn[e];
                d = e;
            }
        const int64_t n_lo = (m * (k / 2)) / k;
        const double* X = xyz;
        std::nth_element(perm.begin() + lo, perm.begin() + lo + n_lo, perm.begin() + hi,
                         [X, d](int64_t a, int64_t b) {
                             const double xa = X[3 * a + d], xb = X[3 * b + d];
                             return xa < xb || (xa == xb && a < b);
                         });
        node(lo, lo + n_lo);
        node(lo + n_lo, hi);
    }
};

}  // namespace

void cutplane_batches(const double* xyz, int64_t n, int32_t max_batch, std::vector<int64_t>& perm,
                      std::vector<int64_t>& batch_ptr)
{
    perm.resize(n);
    for (int64_t k = 0; k < n; ++k) perm[k] = k;
    batch_ptr.assign(1, 0);
    if (n == 0) return;
    CutPlaneBuilder b{xyz, max_batch, perm, batch_ptr};
    b.node(0, n);
}

void make_batches(int32_t batcher, const double* xyz, int64_t n, int32_t max_batch, std::vector<int64_t>& perm,
                  std::vector<int64_t>& batch_ptr)
{
    if (batcher == NAO_BATCH_CUTPLANE) cutplane_batches(xyz, n, max_batch, perm, batch_ptr);
    else octree_batches(xyz, n, max_batch, perm, batch_ptr);
}

// ------------------------------------------------------------------------------------------
// relevance

void relevant_atoms(const HostBasis& b, const double* xyz, const std::vector<int64_t>& perm,
                    const std::vector<int64_t>& batch_ptr, std::vector<int64_t>& atom_ptr,
                    std::vector<int32_t>& atoms)
{
    const int64_t nb = (int64_t)batch_ptr.size() - 1;
    atom_ptr.assign(nb + 1, 0);
    atoms.clear();
    if (nb <= 0 || b.n_atoms == 0) return;

    // uniform cell list over atoms, edge = largest cutoff
    double rcmax = 0.0;
    for (double r : b.atom_rcut) rcmax = std::max(rcmax, r);
    double alo[3], ahi[3];
    for (int d = 0; d < 3; ++d) alo[d] = ahi[d] = b.atom_xyz[d];
    for (int64_t a = 0; a < b.n_atoms; ++a)
        for (int d = 0; d < 3; ++d) {
            alo[d] = std::min(alo[d], b.atom_xyz[3 * a + d]);
            ahi[d] = std::max(ahi[d], b.atom_xyz[3 * a + d]);
        }
    int64_t nc[3];
    for (int d = 0; d < 3; ++d) nc[d] = std::max<int64_t>(1, (int64_t)std::floor((ahi[d] - alo[d]) / rcmax) + 1);
    auto cell_of = [&](int64_t a, int d) {
        int64_t c = (int64_t)std::floor((b.atom_xyz[3 * a + d] - alo[d]) / rcmax);
        return std::min(std::max<int64_t>(c, 0), nc[d] - 1);
    };
    std::vector<int64_t> cell_ptr(nc[0] * nc[1] * nc[2] + 1, 0), cell_atoms(b.n_atoms);
    for (int64_t a = 0; a < b.n_atoms; ++a) ++cell_ptr[(cell_of(a, 2) * nc[1] + cell_of(a, 1)) * nc[0] + cell_of(a, 0) + 1];
    for (size_t c = 1; c < cell_ptr.size(); ++c) cell_ptr[c] += cell_ptr[c - 1];
    {
        std::vector<int64_t> fill(cell_ptr.begin(), cell_ptr.end() - 1);
        for (int64_t a = 0; a < b.n_atoms; ++a)
            cell_atoms[fill[(cell_of(a, 2) * nc[1] + cell_of(a, 1)) * nc[0] + cell_of(a, 0)]++] = a;
    }

    unsigned nthreads = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (nb < 256) nthreads = 1;
    std::vector<std::vector<int32_t>> part_atoms(nthreads);
    std::vector<std::vector<int64_t>> part_cnt(nthreads);
    auto work = [&](unsigned t) {
        const int64_t b0 = nb * t / nthreads, b1 = nb * (t + 1) / nthreads;
        std::vector<int32_t>& out = part_atoms[t];
        std::vector<int64_t>& cnt = part_cnt[t];
        std::vector<int32_t> cand;
        for (int64_t bi = b0; bi < b1; ++bi) {
            const int64_t p0 = batch_ptr[bi], p1 = batch_ptr[bi + 1];
            double lo[3], hi[3];
            for (int d = 0; d < 3; ++d) lo[d] = hi[d] = xyz[3 * perm[p0] + d];
            for (int64_t k = p0; k < p1; ++k)
                for (int d = 0; d < 3; ++d) {
                    const double x = xyz[3 * perm[k] + d];
                    lo[d] = std::min(lo[d], x);
                    hi[d] = std::max(hi[d], x);
                }
            double c[3], rad = 0.0;
            for (int d = 0; d < 3; ++d) c[d] = 0.5 * (lo[d] + hi[d]);
            for (int64_t k = p0; k < p1; ++k) {
                const double* p = xyz + 3 * perm[k];
                const double ex = p[0] - c[0], ey = p[1] - c[1], ez = p[2] - c[2];
                rad = std::max(rad, std::sqrt(ex * ex + ey * ey + ez * ez));
            }
            // candidate cells: those that may hold an atom within rad + rcmax of the centre
            const double reach = rad + rcmax + 1e-9 * (1.0 + rad + rcmax);
            int64_t c0[3], c1[3];
            bool none = false;
            for (int d = 0; d < 3; ++d) {
                const double f0 = std::floor((c[d] - reach - alo[d]) / rcmax);
                const double f1 = std::floor((c[d] + reach - alo[d]) / rcmax);
                if (f1 < 0.0 || f0 > (double)(nc[d] - 1)) none = true;
                c0[d] = f0 < 0.0 ? 0 : (int64_t)f0;
                c1[d] = f1 > (double)(nc[d] - 1) ? nc[d] - 1 : (int64_t)f1;
            }
            cand.clear();
            if (!none)
                for (int64_t z = c0[2]; z <= c1[2]; ++z)
                    for (int64_t y = c0[1]; y <= c1[1]; ++y)
                        for (int64_t x = c0[0]; x <= c1[0]; ++x) {
                            const int64_t cc = (z * nc[1] + y) * nc[0] + x;
                            for (int64_t q = cell_ptr[cc]; q < cell_ptr[cc + 1]; ++q) cand.push_back((int32_t)cell_atoms[q]);
                        }
            std::sort(cand.begin(), cand.end());
            int64_t n_rel = 0;
            for (int32_t a : cand) {
                const double X = b.atom_xyz[3 * a], Y = b.atom_xyz[3 * a + 1], Z = b.atom_xyz[3 * a + 2];
                const double rc = b.atom_rcut[a];
                // bounding-sphere prefilter: may only skip atoms that cannot be relevant
                const double ex = X - c[0], ey = Y - c[1], ez = Z - c[2];
                const double dc = std::sqrt(ex * ex + ey * ey + ez * ez);
                if (dc > rad + rc + 1e-9 * (1.0 + rad + rc)) continue;
                const double rc2 = rc * rc;
                bool rel = false;
                for (int64_t k = p0; k < p1 && !rel; ++k) {
                    const double* p = xyz + 3 * perm[k];
                    const double dx = p[0] - X;
                    const double dy = p[1] - Y;
                    const double dz = p[2] - Z;
                    const double d2 = (dx * dx + dy * dy) + dz * dz;
                    rel = d2 < rc2;
                }
                if (rel) {
                    out.push_back(a);
                    ++n_rel;
                }
            }
            cnt.push_back(n_rel);
        }
    };
    if (nthreads == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nthreads; ++t) th.emplace_back(work, t);
        for (auto& t : th) t.join();
    }
    int64_t bi = 0;
    for (unsigned t = 0; t < nthreads; ++t) {
        for (int64_t c : part_cnt[t]) {
            atom_ptr[bi + 1] = atom_ptr[bi] + c;
            ++bi;
        }
        atoms.insert(atoms.end(), part_atoms[t].begin(), part_atoms[t].end());
    }
}

void expand_lists(const HostBasis& b, const std::vector<int64_t>& atom_ptr,
                  const std::vector<int32_t>& atoms, std::vector<int64_t>& basis_ptr,
                  std::vector<int32_t>& basis_idx)
{
    const int64_t nb = (int64_t)atom_ptr.size() - 1;
    basis_ptr.assign(nb + 1, 0);
    basis_idx.clear();
    for (int64_t bi = 0; bi < nb; ++bi) {
        for (int64_t q = atom_ptr[bi]; q < atom_ptr[bi + 1]; ++q) {
            const int32_t a = atoms[q];
            for (int64_t f = b.atom_first[a]; f < b.atom_first[a + 1]; ++f) basis_idx.push_back((int32_t)f);
        }
        basis_ptr[bi + 1] = (int64_t)basis_idx.size();
    }
}

// ------------------------------------------------------------------------------------------
// splines

std::vector<double> spline_knots(const HostBasis& b)
{
    const int N = b.n_knots;
    std::vector<double> out((size_t)b.n_radial * N * 2);
    std::vector<double> M(N), diag(N), rhs(N);
    for (int32_t r = 0; r < b.n_radial; ++r) {
        const double* y = b.samples.data() + (size_t)r * N;
        // natural spline, unit spacing: M_{k-1} + 4 M_k + M_{k+1} = 6 (y_{k-1} - 2 y_k + y_{k+1})
        for (int k = 1; k < N - 1; ++k) {
            diag[k] = 4.0;
            rhs[k] = 6.0 * (y[k - 1] - 2.0 * y[k] + y[k + 1]);
        }
        for (int k = 2; k < N - 1; ++k) {
            const double f = 1.0 / diag[k - 1];
            diag[k] -= f;
            rhs[k] -= f * rhs[k - 1];
        }
        M[0] = 0.0;
        M[N - 1] = 0.0;
        M[N - 2] = rhs[N - 2] / diag[N - 2];
        for (int k = N - 3; k >= 1; --k) M[k] = (rhs[k] - M[k + 1]) / diag[k];
        // per knot (y_k, M_k / 6): on [k, k+1], with v = 1 - u,
        //   R = v (y_k + (v^2 - 1) M_k / 6) + u (y_{k+1} + (u^2 - 1) M_{k+1} / 6)
        for (int k = 0; k < N; ++k) {
            out[((size_t)r * N + k) * 2] = y[k];
            out[((size_t)r * N + k) * 2 + 1] = M[k] / 6.0;
        }
    }
    return out;
}

// ------------------------------------------------------------------------------------------
// execution units

namespace {

void push_unit(const HostBasis& b, int64_t p0, int32_t np, int32_t batch, const std::vector<int32_t>& at,
               std::vector<Unit>& units, std::vector<int32_t>& unit_atoms, std::vector<int32_t>& unit_cols)
{
    Unit u;
    u.point_begin = p0;
    u.n_points = np;
    u.n_atoms = (int32_t)at.size();
    u.atom_begin = (int64_t)unit_atoms.size();
    u.batch = batch;
    int32_t col = 0;
    for (int32_t a : at) {
        unit_atoms.push_back(a);
        unit_cols.push_back(col);
        col += (int32_t)(b.atom_first[a + 1] - b.atom_first[a]);
    }
    u.m = col;
    units.push_back(u);
}

int64_t list_size(const HostBasis& b, const std::vector<int32_t>& at)
{
    int64_t m = 0;
    for (int32_t a : at) m += b.atom_first[a + 1] - b.atom_first[a];
    return m;
}

}  // namespace

void make_groups(const HostBasis& b, const std::vector<int64_t>& batch_ptr,
                 const std::vector<int64_t>& atom_ptr, const std::vector<int32_t>& atoms,
                 int32_t group_max, std::vector<Unit>& units, std::vector<int32_t>& unit_atoms,
                 std::vector<int32_t>& unit_cols)
{
    units.clear();
    unit_atoms.clear();
    unit_cols.clear();
    const int64_t nb = (int64_t)batch_ptr.size() - 1;
    std::vector<int32_t> cur, merged;
    int64_t cur_p0 = 0, cur_np = 0;
    int32_t cur_batch = 0;
    double cur_cost = 0.0;  // sum over members of |B| m^2
    auto flush = [&]() {
        if (cur_np > 0 && !cur.empty()) push_unit(b, cur_p0, (int32_t)cur_np, cur_batch, cur, units, unit_atoms, unit_cols);
        cur.clear();
        cur_np = 0;
        cur_cost = 0.0;
    };
    for (int64_t bi = 0; bi < nb; ++bi) {
        const int64_t p0 = batch_ptr[bi], np = batch_ptr[bi + 1] - p0;
        if (atom_ptr[bi + 1] == atom_ptr[bi] || np == 0) {  // no basis function reaches it
            flush();
            continue;
        }
        std::vector<int32_t> at(atoms.begin() + atom_ptr[bi], atoms.begin() + atom_ptr[bi + 1]);
        const double m_b = (double)list_size(b, at);
        const int32_t cap = group_max > 0 ? group_max : 256;
        if (group_max == 0 || np > cap) {  // no grouping, or a batch larger than a group
            flush();
            for (int64_t s = 0; s < np; s += cap)
                push_unit(b, p0 + s, (int32_t)std::min<int64_t>(cap, np - s), (int32_t)bi, at, units,
                          unit_atoms, unit_cols);
            continue;
        }
        if (np > group_max) {
            flush();
            for (int64_t s = 0; s < np; s += group_max)
                push_unit(b, p0 + s, (int32_t)std::min<int64_t>(group_max, np - s), (int32_t)bi, at, units,
                          unit_atoms, unit_cols);
            continue;
        }
        if (cur_np > 0 && p0 == cur_p0 + cur_np && cur_np + np <= group_max) {
            merged.clear();
            std::set_union(cur.begin(), cur.end(), at.begin(), at.end(), std::back_inserter(merged));
            const double mu = (double)list_size(b, merged);
            const double joined = (double)(cur_np + np) * mu * mu;
            const double apart = cur_cost + (double)np * m_b * m_b;
            if (joined <= 1.6 * apart) {
                cur.swap(merged);
                cur_np += np;
                cur_cost = apart;
                continue;
            }
        }
        flush();
        cur = at;
        cur_p0 = p0;
        cur_np = np;
        cur_batch = (int32_t)bi;
        cur_cost = (double)np * m_b * m_b;
    }
    flush();
}

void batch_units(const HostBasis& b, const std::vector<int64_t>& batch_ptr,
                 const std::vector<int64_t>& atom_ptr, const std::vector<int32_t>& atoms,
                 int64_t batch_begin, int64_t batch_end, std::vector<Unit>& units,
                 std::vector<int32_t>& unit_atoms, std::vector<int32_t>& unit_cols)
{
    units.clear();
    unit_atoms.clear();
    unit_cols.clear();
    for (int64_t bi = batch_begin; bi < batch_end; ++bi) {
        std::vector<int32_t> at(atoms.begin() + atom_ptr[bi], atoms.begin() + atom_ptr[bi + 1]);
        push_unit(b, batch_ptr[bi], (int32_t)(batch_ptr[bi + 1] - batch_ptr[bi]), (int32_t)bi, at, units,
                  unit_atoms, unit_cols);
    }
}

}  // namespace nao

// HIP kernels for gfx950 (CDNA4): basis evaluation, the two batch contractions on FP64
// MFMA, and the small elementwise / reduction / mirror kernels around them.
//
// Data layout (device memory):
//   - points, weights and w*v in batch order (structure of arrays, FP64);
//   - basis values of an execution unit: [n_points][ld] FP64, point-major, ld a multiple of
//     the 64-wide basis tile, padding columns zero;
//   - D and H dense row-major [N_b][N_b] FP64; n in the caller's point order.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <type_traits>

#include <hip/hip_runtime.h>

#include "devtypes.h"

namespace nao {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// Pointers into device memory read from the segment tables are generic to the compiler;
// casting them to the global address space makes it emit global (not flat) loads, stores and
// atomics, which are counted by vmcnt only and do not hold up waits for LDS results.
template <typename T> using gp = __attribute__((address_space(1))) T*;
template <typename T> __device__ inline gp<T> gptr(T* p) { return (gp<T>)p; }
__device__ inline void gadd(gp<double> p, double v)
{
    (void)__hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------------------------------
// helpers

template <typename F>
__device__ inline int find_segment(const DevSeg* segs, int n_segs, int64_t b, F prefix_of)
{
    int lo = 0, hi = n_segs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix_of(segs[mid]) <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Workgroup ids are dealt round-robin to the 8 XCDs (each with its own L2).  Virtual index
// v in [0, 8 ceil(total/8)) maps to item (v % 8) * ceil(total/8) + v / 8, so XCD x works through
// the contiguous eighth [x ceil(total/8), (x+1) ceil(total/8)) of the item list and the tiles of
// one execution unit share one L2.  Items >= total are skipped.
constexpr int N_XCD = 8;
__host__ __device__ inline int64_t xcd_span(int64_t total) { return N_XCD * ((total + N_XCD - 1) / N_XCD); }
__device__ inline int64_t xcd_item(int64_t v, int64_t total)
{
    const int64_t per = (total + N_XCD - 1) / N_XCD;
    return (v % N_XCD) * per + v / N_XCD;
}

// (dx*dx + dy*dy) + dz*dz without contraction: the same arithmetic that decides relevance.
__device__ inline double dist2_exact(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    const double xx = dx * dx;
    const double yy = dy * dy;
    const double zz = dz * dz;
    return (xx + yy) + zz;
}

// Real orthonormal spherical harmonics of degree L (<= 3) of a unit vector, m = -L..L, into
// Y[0 .. 2L]; Y_11 ~ +x.
template <int L>
__device__ inline void ylm_l(double x, double y, double z, double* Y)
{
    if constexpr (L == 0) {
        Y[0] = 0.28209479177387814;  // 1 / (2 sqrt(pi))
    } else if constexpr (L == 1) {
        const double c1 = 0.48860251190291992;  // sqrt(3 / (4 pi))
        Y[0] = c1 * y;
        Y[1] = c1 * z;
        Y[2] = c1 * x;
    } else if constexpr (L == 2) {
        const double c2a = 1.0925484305920792;   // sqrt(15 / pi) / 2
        const double c2b = 0.31539156525252005;  // sqrt(5 / pi) / 4
        const double c2c = 0.54627421529603959;  // sqrt(15 / pi) / 4
        Y[0] = c2a * x * y;
        Y[1] = c2a * y * z;
        Y[2] = c2b * (3.0 * z * z - 1.0);
        Y[3] = c2a * x * z;
        Y[4] = c2c * (x * x - y * y);
    } else {
        const double c3a = 0.59004358992664352;  // sqrt(35 / (2 pi)) / 4
        const double c3b = 2.8906114426405538;   // sqrt(105 / pi) / 2
        const double c3c = 0.45704579946446572;  // sqrt(21 / (2 pi)) / 4
        const double c3d = 0.37317633259011546;  // sqrt(7 / pi) / 4
        const double c3e = 1.4453057213202769;   // sqrt(105 / pi) / 4
        Y[0] = c3a * y * (3.0 * x * x - y * y);
        Y[1] = c3b * x * y * z;
        Y[2] = c3c * y * (5.0 * z * z - 1.0);
        Y[3] = c3d * (5.0 * z * z * z - 3.0 * z);
        Y[4] = c3c * x * (5.0 * z * z - 1.0);
        Y[5] = c3e * z * (x * x - y * y);
        Y[6] = c3a * x * (x * x - 3.0 * y * y);
    }
}

// All harmonics up to lmax (<= 3), index l^2 + l + m.
__device__ inline void real_ylm(double x, double y, double z, int lmax, double* Y)
{
    ylm_l<0>(x, y, z, Y);
    if (lmax >= 1) ylm_l<1>(x, y, z, Y + 1);
    if (lmax >= 2) ylm_l<2>(x, y, z, Y + 4);
    if (lmax >= 3) ylm_l<3>(x, y, z, Y + 9);
}

// Partial derivatives of the harmonic polynomials of real_ylm (index lm) with respect to the
// three components of the unit vector, taken as independent variables.
__device__ inline void ylm_grad_one(int lm, double x, double y, double z, double* g)
{
    const double c1 = 0.48860251190291992, c2a = 1.0925484305920792, c2b = 0.31539156525252005;
    const double c2c = 0.54627421529603959, c3a = 0.59004358992664352, c3b = 2.8906114426405538;
    const double c3c = 0.45704579946446572, c3d = 0.37317633259011546, c3e = 1.4453057213202769;
    double gx = 0.0, gy = 0.0, gz = 0.0;
    switch (lm) {
    case 1: gy = c1; break;
    case 2: gz = c1; break;
    case 3: gx = c1; break;
    case 4: gx = c2a * y; gy = c2a * x; break;
    case 5: gy = c2a * z; gz = c2a * y; break;
    case 6: gz = 6.0 * c2b * z; break;
    case 7: gx = c2a * z; gz = c2a * x; break;
    case 8: gx = 2.0 * c2c * x; gy = -2.0 * c2c * y; break;
    case 9: gx = 6.0 * c3a * x * y; gy = 3.0 * c3a * (x * x - y * y); break;
    case 10: gx = c3b * y * z; gy = c3b * x * z; gz = c3b * x * y; break;
    case 11: gy = c3c * (5.0 * z * z - 1.0); gz = 10.0 * c3c * y * z; break;
    case 12: gz = c3d * (15.0 * z * z - 3.0); break;
    case 13: gx = c3c * (5.0 * z * z - 1.0); gz = 10.0 * c3c * x * z; break;
    case 14: gx = 2.0 * c3e * x * z; gy = -2.0 * c3e * y * z; gz = c3e * (x * x - y * y); break;
    case 15: gx = 3.0 * c3a * (x * x - y * y); gy = -6.0 * c3a * x * y; break;
    default: break;
    }
    g[0] = gx;
    g[1] = gy;
    g[2] = gz;
}

// ------------------------------------------------------------------------------------------
// Basis evaluation
constexpr size_t BASIS_LDS_BYTES = (size_t)MAX_SPLINE_LDS * sizeof(double);

constexpr int BASIS_ATOMS = 192;   // atoms of a unit staged in LDS
constexpr int BASIS_SHELLS = 128;  // shells of a system staged in LDS
constexpr int BASIS_SLICES = 4;    // work items per unit (point slices) of the basis kernel
constexpr int BASIS_WIN = 16;      // values per pair staged at a time for the row writes

// Basis values of execution units: BASIS_SLICES workgroups per unit, each taking a contiguous
// slice of the unit's points (more workgroups in flight than one per unit, and shorter tails);
// threads over (point, atom) pairs with the atom fastest, each writing all functions of its atom.  The unit's atoms (position,
// cutoff, species, first column) and the system's shell tables (l, radial function and its
// parameters) are staged in LDS first, so that a pair's chain of table lookups stays on chip;
// a unit or system larger than the staging arrays reads them from global memory instead.
template <typename T, bool SPLINE_LDS, int EX>
__global__ __launch_bounds__(256, 2) void basis_kernel(const DevSeg* __restrict__ segs, int n_segs, int64_t total,
                                                       int spline_lds)
{
    extern __shared__ double lds_spline[];
    // plain FP64 basis values (EX = EXTRA_NONE): per wave, BASIS_WIN values of each of its 64
    // pairs, and per pair the unit-local offset of its first value and its value count (FP32
    // values, half the bytes, are faster stored per pair directly)
    constexpr bool STAGE = EX == EXTRA_NONE && sizeof(T) == 8;
    __shared__ double s_win[STAGE ? 4 * 64 * (BASIS_WIN + 1) : 1];
    __shared__ __align__(8) int32_t s_pair[STAGE ? 4 * 64 * 2 : 2];
    constexpr int SPT = MAX_UNIT_POINTS / BASIS_SLICES;  // points of a slice staged at a time
    __shared__ double s_pt[STAGE ? SPT : 1][3];  // the slice's points (a run of SPT at a time)
    __shared__ double s_atom[BASIS_ATOMS][4];  // x, y, z, (largest cutoff)^2
    __shared__ int32_t s_aspc[BASIS_ATOMS][2];  // species, first column in the unit
    __shared__ double s_par[BASIS_SHELLS][4];  // rmin, rcut^2, 1/Delta, ln rmin of the shell's radial
    __shared__ int32_t s_shell[BASIS_SHELLS][2];  // l, radial function
    __shared__ int32_t s_shptr[BASIS_SHELLS + 1];
    (void)spline_lds;  // the launcher sized the dynamic LDS for the table
    const int tid = threadIdx.x;
    const DevSys* table_of = nullptr;  // the system whose spline table is in LDS
    for (int64_t v_ = blockIdx.x; v_ < xcd_span(total); v_ += gridDim.x) {
        const int64_t bi = xcd_item(v_, total);
        if (bi >= total) continue;
        // item = (unit, slice): BASIS_SLICES consecutive items split one unit's points
        const int64_t b = bi / BASIS_SLICES;
        const int slice = (int)(bi - b * BASIS_SLICES);
        __syncthreads();  // the previous item may still read LDS
        const int s = find_segment(segs, n_segs, b, [](const DevSeg& g) { return g.unit_prefix; });
        const DevSeg& sg = segs[s];
        const DevUnit u = sg.units[sg.unit_begin + (b - sg.unit_prefix)];
        const int row0 = (int)(((int64_t)u.n_points * slice) / BASIS_SLICES);
        const int row1 = (int)(((int64_t)u.n_points * (slice + 1)) / BASIS_SLICES);
        if (row1 <= row0) continue;
        const DevSys* S = sg.sys;
        const int nk = S->n_knots;
        const int na = u.n_atoms, n_sp = S->n_species, n_sh = S->n_shells;
        gp<const double> spl = gptr(S->spline);
        gp<const int32_t> uat = gptr(sg.unit_atoms) + u.atom_begin;
        gp<const int32_t> ucol = gptr(sg.unit_cols) + u.atom_begin;
        gp<const double> axyz = gptr(S->atom_xyzr);
        gp<const int32_t> aspecies = gptr(S->atom_species);
        gp<const int32_t> shell_ptr = gptr(S->species_shell_ptr);
        gp<const int32_t> shell_l = gptr(S->shell_l);
        gp<const int32_t> shell_rad = gptr(S->shell_radial);
        gp<const double> rpar = gptr(S->radial_par);
        const bool staged = na <= BASIS_ATOMS && n_sh <= BASIS_SHELLS && n_sp <= BASIS_SHELLS;  // uniform
        // the table is staged once per workgroup and system (the grid is capped, so that a
        // workgroup takes many items)
        const bool restage = SPLINE_LDS && S != table_of;  // uniform
        if (restage) {
            const int nsp = S->n_radial * nk * 2;
            for (int i = tid; i < nsp; i += blockDim.x) lds_spline[i] = spl[i];
            table_of = S;
        }
        // points of rows r0 .. r1 - 1 of the unit into s_pt
        auto stage_points = [&](int r0, int r1) {
            for (int i = tid; i < r1 - r0; i += blockDim.x) {
                const int64_t p = u.point_begin + r0 + i;
                s_pt[i][0] = gptr(S->px)[p];
                s_pt[i][1] = gptr(S->py)[p];
                s_pt[i][2] = gptr(S->pz)[p];
            }
        };
        if (STAGE) stage_points(row0, min(row1, row0 + SPT));
        if (staged) {
            for (int ai = tid; ai < na; ai += blockDim.x) {
                const int atom = uat[ai];
#pragma unroll
                for (int k = 0; k < 4; ++k) s_atom[ai][k] = axyz[4 * (int64_t)atom + k];
                s_aspc[ai][0] = aspecies[atom];
                s_aspc[ai][1] = ucol[ai];
            }
            for (int j = tid; j < n_sh; j += blockDim.x) {
                const int rr = shell_rad[j];
                s_shell[j][0] = shell_l[j];
                s_shell[j][1] = rr;
#pragma unroll
                for (int k = 0; k < 4; ++k) s_par[j][k] = rpar[4 * rr + k];
            }
            for (int k = tid; k <= n_sp; k += blockDim.x) s_shptr[k] = shell_ptr[k];
        }
        if (restage || staged || STAGE) __syncthreads();
        gp<T> __restrict__ out = gptr(static_cast<T*>(sg.phi) + u.out_offset);
        // EX = EXTRA_GRAD: 3 gradient values per basis value; EX = EXTRA_GGA_L: L = (w v / 2) phi +
        // (w a) . grad phi, one per basis value; EX = EXTRA_KS_L: L = (w v / 2) phi - (w / 4) lap phi
        // (+ (w a) . grad phi when the segment has a field); same element order as the basis values
        // EX = EXTRA_GRAD_H: the 3 gradient values and w h_KS phi = (w v) phi - (w / 2) lap phi, 4 per
        // basis value
        constexpr bool LAPL = EX == EXTRA_GRAD_H;
        constexpr bool GRAD = EX == EXTRA_GRAD || LAPL, GGA = EX == EXTRA_GGA_L, KS = EX == EXTRA_KS_L;
        const bool field = GGA || (KS && sg.wa != nullptr);  // uniform
        constexpr int XW = GRAD ? (LAPL ? 4 : 3) : 1;  // extra values per basis value
        gp<T> __restrict__ gout = EX != EXTRA_NONE ? gptr(static_cast<T*>(sg.gphi) + XW * u.out_offset) : nullptr;
        const int64_t npairs = (int64_t)(row1 - row0) * na;
        const double tmax = (double)(nk - 1);

        // Gradient and L values (EX != EXTRA_NONE): threads over (point, atom) pairs, each writing
        // every value of its pair directly.
        auto pairs = [&](auto on_chip) {
            constexpr bool ST = decltype(on_chip)::value;
            for (int64_t q = tid; q < npairs; q += blockDim.x) {
                const int ql = (int)q;
                const int pq = ql / na;
                const int ai = ql - pq * na;
                const int pl = row0 + pq;
                const int atom = ST ? 0 : uat[ai];
                int col = ST ? s_aspc[ai][1] : ucol[ai];
                const int64_t p = u.point_begin + pl;
                const double ax = ST ? s_atom[ai][0] : axyz[4 * (int64_t)atom];
                const double ay = ST ? s_atom[ai][1] : axyz[4 * (int64_t)atom + 1];
                const double az = ST ? s_atom[ai][2] : axyz[4 * (int64_t)atom + 2];
                const double arc2 = ST ? s_atom[ai][3] : axyz[4 * (int64_t)atom + 3];
                const double dx = gptr(S->px)[p] - ax;
                const double dy = gptr(S->py)[p] - ay;
                const double dz = gptr(S->pz)[p] - az;
                const double d2 = dist2_exact(dx, dy, dz);
                const int sp = ST ? s_aspc[ai][0] : aspecies[atom];
                const int sh0 = ST ? s_shptr[sp] : shell_ptr[sp];
                const int sh1 = ST ? s_shptr[sp + 1] : shell_ptr[sp + 1];
                gp<T> row = out + (int64_t)pl * u.ld;
                gp<T> grow = EX != EXTRA_NONE ? gout + XW * (int64_t)pl * u.ld : nullptr;
                if (d2 >= arc2) {
                    for (int j = sh0; j < sh1; ++j) {
                        const int nf = 2 * (ST ? s_shell[j][0] : shell_l[j]) + 1;
                        for (int f = 0; f < nf; ++f) row[col + f] = T(0);
                        if (EX != EXTRA_NONE)
                            for (int f = 0; f < XW * nf; ++f) grow[XW * col + f] = T(0);
                        col += nf;
                    }
                    continue;
                }
                const double r = sqrt(d2);
                double ux = 0.0, uy = 0.0, uz = 1.0;
                if (r > 0.0) {
                    const double ir = 1.0 / r;
                    ux = dx * ir;
                    uy = dy * ir;
                    uz = dz * ir;
                }
                double Y[16];
                int lmax = 0;
                for (int j = sh0; j < sh1; ++j) lmax = max(lmax, ST ? s_shell[j][0] : shell_l[j]);
                real_ylm(ux, uy, uz, lmax, Y);
                const double lnr = r > 0.0 ? log(r) : 0.0;
                for (int j = sh0; j < sh1; ++j) {
                    const int l = ST ? s_shell[j][0] : shell_l[j];
                    const int rr = ST ? s_shell[j][1] : shell_rad[j];
                    const double rmin = ST ? s_par[j][0] : rpar[4 * rr];
                    const double rc2 = ST ? s_par[j][1] : rpar[4 * rr + 1];
                    const double idel = ST ? s_par[j][2] : rpar[4 * rr + 2];
                    const double lnmin = ST ? s_par[j][3] : rpar[4 * rr + 3];
                    double R = 0.0, dR = 0.0, dS = 0.0, d2S = 0.0;
                    if (d2 < rc2) {
                        double t = r > rmin ? (lnr - lnmin) * idel : 0.0;
                        t = fmin(fmax(t, 0.0), tmax);
                        const int k = min((int)t, nk - 2);
                        const double w = t - (double)k, v = 1.0 - w;
                        // knots k and k + 1: (y_k, M_k / 6, y_{k+1}, M_{k+1} / 6), 32 contiguous bytes
                        const int64_t ci = ((int64_t)rr * nk + k) * 2;
                        double ya, pa, yb, pb;
                        if (SPLINE_LDS) {
                            ya = lds_spline[ci], pa = lds_spline[ci + 1], yb = lds_spline[ci + 2], pb = lds_spline[ci + 3];
                        } else {
                            gp<const double> c = spl + ci;
                            ya = c[0], pa = c[1], yb = c[2], pb = c[3];
                        }
                        R = v * (ya + (v * v - 1.0) * pa) + w * (yb + (w * w - 1.0) * pb);
                        // dR/dr = dR/dw dt/dr with dt/dr = 1 / (r Delta); the clamped part r <= rmin is constant
                        const double dRdw = (yb - ya) - (3.0 * v * v - 1.0) * pa + (3.0 * w * w - 1.0) * pb;
                        if (EX != EXTRA_NONE && r > rmin) dR = dRdw * idel / r;
                        if (KS || LAPL) {
                            dS = dRdw;                    // dR/dt
                            d2S = 6.0 * (v * pa + w * pb);  // d2R/dt2
                        }
                    }
                    if (EX != EXTRA_NONE) {
                        // grad phi = R'(r) u Y + (R / r) (G - u (u . G)), G = dY/du; zero where the
                        // function is cut off or r <= rmin
                        const bool live = d2 < rc2 && r > rmin;
                        const double ir = live ? 1.0 / r : 0.0;
                        double hwv = 0.0, wax = 0.0, way = 0.0, waz = 0.0, qw = 0.0;
                        if (GGA || KS) hwv = 0.5 * gptr(sg.wv)[p];
                        if (field) {
                            gp<const double> wa = gptr(sg.wa) + 3 * p;
                            wax = wa[0], way = wa[1], waz = wa[2];
                        }
                        // lap phi = (S''/Delta^2 + S'/Delta - l(l+1) S) Y / r^2 in the spline variable
                        double lap = 0.0;
                        if (KS || LAPL)
                            lap = live ? ((d2S * idel + dS) * idel - (double)(l * (l + 1)) * R) * ir * ir : 0.0;
                        if (KS) qw = 0.25 * gptr(S->pw)[p];
                        if (LAPL) {
                            hwv = gptr(sg.wv)[p];
                            qw = 0.5 * gptr(S->pw)[p];
                        }
                        for (int f = 0; f < 2 * l + 1; ++f) {
                            const int lm = l * l + f;
                            const double yv = Y[lm];
                            double g0 = 0.0, g1 = 0.0, g2 = 0.0;
                            if (GRAD || field) {
                                double gv[3];
                                ylm_grad_one(lm, ux, uy, uz, gv);
                                const double ug = (ux * gv[0] + uy * gv[1]) + uz * gv[2];
                                g0 = live ? dR * ux * yv + R * ir * (gv[0] - ux * ug) : 0.0;
                                g1 = live ? dR * uy * yv + R * ir * (gv[1] - uy * ug) : 0.0;
                                g2 = live ? dR * uz * yv + R * ir * (gv[2] - uz * ug) : 0.0;
                            }
                            if (GRAD) {
                                gp<T> dst = grow + XW * (int64_t)(col + f);
                                dst[0] = T(g0);
                                dst[1] = T(g1);
                                dst[2] = T(g2);
                                if (LAPL) dst[3] = T(hwv * (R * yv) - qw * (lap * yv));
                            } else {
                                grow[col + f] = T((hwv * (R * yv) - qw * (lap * yv)) + ((wax * g0 + way * g1) + waz * g2));
                            }
                        }
                    }
                    auto put = [&](auto deg) {
                        constexpr int L = decltype(deg)::value;
#pragma unroll
                        for (int f = 0; f < 2 * L + 1; ++f) row[col + f] = T(R * Y[L * L + f]);
                        col += 2 * L + 1;
                    };
                    switch (l) {
                    case 0: put(std::integral_constant<int, 0>{}); break;
                    case 1: put(std::integral_constant<int, 1>{}); break;
                    case 2: put(std::integral_constant<int, 2>{}); break;
                    default: put(std::integral_constant<int, 3>{}); break;
                    }
                }
            }
        };
        // Plain values: a wave's 64 pairs are consecutive atoms of one or a few points, whose
        // columns are consecutive in the row, so the values are staged in LDS, BASIS_WIN per pair
        // at a time, and written as contiguous runs of the rows (a store per value and lane would
        // touch a separate cache line per lane).
        // the rows of the run in s_pt (a slice longer than SPT rows, which only a unit of more
        // than MAX_UNIT_POINTS points has, is taken in several runs)
        int run_row0 = row0;
        int64_t run_pairs = (int64_t)(min(row1, row0 + SPT) - row0) * na;
        auto pairs_staged = [&](auto on_chip) {
            constexpr bool ST = decltype(on_chip)::value;
            constexpr int BW = BASIS_WIN, BWP = BASIS_WIN + 1;
            const int lane = tid & 63, wave = tid >> 6;
            double* win = &s_win[wave * 64 * BWP];
            int32_t* pinfo = &s_pair[wave * 64 * 2];
            for (int64_t qb = tid - lane; qb < run_pairs; qb += blockDim.x) {  // wave-uniform trip count
                const int64_t q = qb + lane;
                const bool valid = q < run_pairs;
                const int ql = (int)(valid ? q : qb);  // lanes past the end redo the wave's first pair
                const int pq = ql / na;
                const int ai = ql - pq * na;
                const int pl = run_row0 + pq;
                const int atom = ST ? 0 : uat[ai];
                const int col = ST ? s_aspc[ai][1] : ucol[ai];
                const double ax = ST ? s_atom[ai][0] : axyz[4 * (int64_t)atom];
                const double ay = ST ? s_atom[ai][1] : axyz[4 * (int64_t)atom + 1];
                const double az = ST ? s_atom[ai][2] : axyz[4 * (int64_t)atom + 2];
                const double arc2 = ST ? s_atom[ai][3] : axyz[4 * (int64_t)atom + 3];
                const double dx = s_pt[pq][0] - ax;
                const double dy = s_pt[pq][1] - ay;
                const double dz = s_pt[pq][2] - az;
                const double d2 = dist2_exact(dx, dy, dz);
                const int sp = ST ? s_aspc[ai][0] : aspecies[atom];
                const int sh0 = ST ? s_shptr[sp] : shell_ptr[sp];
                const int sh1 = ST ? s_shptr[sp + 1] : shell_ptr[sp + 1];
                const bool near = d2 < arc2;  // else every value of the pair is zero
                const double r = near ? sqrt(d2) : 0.0;
                double ux = 0.0, uy = 0.0, uz = 1.0;
                if (r > 0.0) {
                    const double ir = 1.0 / r;
                    ux = dx * ir;
                    uy = dy * ir;
                    uz = dz * ir;
                }
                const double lnr = r > 0.0 ? log(r) : 0.0;
                int nval = 0;
                for (int j = sh0; j < sh1; ++j) nval += 2 * (ST ? s_shell[j][0] : shell_l[j]) + 1;
                pinfo[2 * lane] = valid ? pl * u.ld + col : -1;
                pinfo[2 * lane + 1] = nval;
                int nmax = valid ? nval : 0;  // the wave's largest value count
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) nmax = max(nmax, __shfl_xor(nmax, o));
                for (int w0 = 0; w0 < nmax; w0 += BW) {
                    // this pair's values w0 .. w0 + BW - 1 into its row of the window
                    int off = 0;
                    for (int j = sh0; j < sh1 && off < w0 + BW; ++j) {
                        const int l = ST ? s_shell[j][0] : shell_l[j];
                        const int nf = 2 * l + 1;
                        if (off + nf > w0) {
                            const int rr = ST ? s_shell[j][1] : shell_rad[j];
                            const double rmin = ST ? s_par[j][0] : rpar[4 * rr];
                            const double rc2 = ST ? s_par[j][1] : rpar[4 * rr + 1];
                            const double idel = ST ? s_par[j][2] : rpar[4 * rr + 2];
                            const double lnmin = ST ? s_par[j][3] : rpar[4 * rr + 3];
                            double R = 0.0;
                            if (near && d2 < rc2) {
                                double t = r > rmin ? (lnr - lnmin) * idel : 0.0;
                                t = fmin(fmax(t, 0.0), tmax);
                                const int k = min((int)t, nk - 2);
                                const double w = t - (double)k, v = 1.0 - w;
                                const int64_t ci = ((int64_t)rr * nk + k) * 2;
                                double ya, pa, yb, pb;
                                if (SPLINE_LDS) {
                                    ya = lds_spline[ci], pa = lds_spline[ci + 1], yb = lds_spline[ci + 2], pb = lds_spline[ci + 3];
                                } else {
                                    gp<const double> c = spl + ci;
                                    ya = c[0], pa = c[1], yb = c[2], pb = c[3];
                                }
                                R = v * (ya + (v * v - 1.0) * pa) + w * (yb + (w * w - 1.0) * pb);
                            }
                            auto put = [&](auto deg) {
                                constexpr int L = decltype(deg)::value;
                                double Yl[2 * L + 1];
                                ylm_l<L>(ux, uy, uz, Yl);
#pragma unroll
                                for (int f = 0; f < 2 * L + 1; ++f) {
                                    const int slot = off + f - w0;
                                    if (slot >= 0 && slot < BW) win[lane * BWP + slot] = R * Yl[f];
                                }
                            };
                            switch (l) {
                            case 0: put(std::integral_constant<int, 0>{}); break;
                            case 1: put(std::integral_constant<int, 1>{}); break;
                            case 2: put(std::integral_constant<int, 2>{}); break;
                            default: put(std::integral_constant<int, 3>{}); break;
                            }
                        }
                        off += nf;
                    }
                    // the wave's own LDS writes are performed before its later reads (in order)
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    // element e = k 64 + lane of the 64 x BW window: pair e / BW, value e % BW;
                    // the LDS reads of four elements are issued before their stores
                    const int2* pinfo2 = reinterpret_cast<const int2*>(pinfo);
#pragma unroll
                    for (int kb = 0; kb < BW; kb += 4) {
                        int2 pi[4];
                        double val[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int e = (kb + j) * 64 + lane;
                            pi[j] = pinfo2[e / BW];
                            val[j] = win[(e / BW) * BWP + e % BW];
                        }
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int f = ((kb + j) * 64 + lane) % BW;
                            if (pi[j].x >= 0 && w0 + f < pi[j].y) out[(int64_t)pi[j].x + w0 + f] = T(val[j]);
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                }
            }
        };
        if constexpr (STAGE) {
            for (int r0 = row0; r0 < row1; r0 += SPT) {
                const int r1 = min(row1, r0 + SPT);
                if (r0 != row0) {
                    __syncthreads();  // every wave is done with the previous run's points
                    stage_points(r0, r1);
                    __syncthreads();
                }
                run_row0 = r0;
                run_pairs = (int64_t)(r1 - r0) * na;
                if (staged) pairs_staged(std::true_type{});
                else pairs_staged(std::false_type{});
            }
        } else {
            if (staged) pairs(std::true_type{});
            else pairs(std::false_type{});
        }
        const int pad = u.ld - u.m;
        if (pad > 0) {
            const int64_t ne = (int64_t)(row1 - row0) * pad;
            for (int64_t q = tid; q < ne; q += blockDim.x) {
                const int64_t pl = row0 + q / pad;
                const int64_t cpad = q - (pl - row0) * pad;
                out[pl * u.ld + u.m + cpad] = T(0);
                if (EX != EXTRA_NONE)
                    for (int c = 0; c < XW; ++c) gout[XW * (pl * u.ld + u.m + cpad) + c] = T(0);
            }
        }
    }
}

static unsigned grid_for(int64_t n, int64_t max_grid)
{
    const int64_t span = xcd_span(n);
    if (max_grid > 0) {
        const int64_t cap = std::max<int64_t>(N_XCD, max_grid / N_XCD * N_XCD);
        if (span > cap) return (unsigned)cap;
    }
    return (unsigned)span;
}

hipError_t launch_basis(const DevSeg* segs_dev, int n_segs, int64_t n_units, int spline_lds, bool fp32_out,
                        hipStream_t st, int64_t max_grid, int extra)
{
    if (n_units <= 0 || n_segs <= 0) return hipSuccess;
    if (n_units > 0x7ffffff0 / BASIS_SLICES || spline_lds < 0 || spline_lds > MAX_SPLINE_LDS) return hipErrorInvalidValue;
    if (extra != EXTRA_NONE && extra != EXTRA_GRAD && extra != EXTRA_GGA_L && extra != EXTRA_KS_L &&
        extra != EXTRA_GRAD_H)
        return hipErrorInvalidValue;
    const int64_t n_items = n_units * BASIS_SLICES;
    // two workgroups per CU fit (LDS); a grid of that size takes many items per workgroup, which
    // stages its spline table once
    if (max_grid <= 0) {
        static std::atomic<int> n_cu{0};
        if (n_cu.load() == 0) {
            int dev = 0, cu = 0;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
                n_cu.store(cu);
        }
        max_grid = 2 * (int64_t)std::max(1, n_cu.load());
    }
    const dim3 g(grid_for(n_items, max_grid)), b(256);
    const bool staged = spline_lds > 0;
    const size_t lds = (size_t)spline_lds * sizeof(double);
    // dynamic LDS above 64 KiB must be allowed per kernel, once per device
    static std::atomic<uint64_t> attrs_set{0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
    const uint64_t bit = 1ull << (dev & 63);
    if (!(attrs_set.load() & bit)) {
#define NAO_BASIS_FNS(TT)                                                                                          \
    reinterpret_cast<const void*>(&basis_kernel<TT, true, EXTRA_NONE>),                                          \
        reinterpret_cast<const void*>(&basis_kernel<TT, false, EXTRA_NONE>),                                     \
        reinterpret_cast<const void*>(&basis_kernel<TT, true, EXTRA_GRAD>),                                      \
        reinterpret_cast<const void*>(&basis_kernel<TT, false, EXTRA_GRAD>),                                     \
        reinterpret_cast<const void*>(&basis_kernel<TT, true, EXTRA_GGA_L>),                                     \
        reinterpret_cast<const void*>(&basis_kernel<TT, false, EXTRA_GGA_L>),                                    \
        reinterpret_cast<const void*>(&basis_kernel<TT, true, EXTRA_KS_L>),                                      \
        reinterpret_cast<const void*>(&basis_kernel<TT, false, EXTRA_KS_L>),                                     \
        reinterpret_cast<const void*>(&basis_kernel<TT, true, EXTRA_GRAD_H>),                                  \
        reinterpret_cast<const void*>(&basis_kernel<TT, false, EXTRA_GRAD_H>)
        const void* fns[] = {NAO_BASIS_FNS(float), NAO_BASIS_FNS(double)};
#undef NAO_BASIS_FNS
        for (const void* f : fns) {
            const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)BASIS_LDS_BYTES);
            if (e != hipSuccess) return e;
        }
        attrs_set.fetch_or(bit);
    }
#define NAO_BASIS_LAUNCH(TT, EE)                                                                                 \
    do {                                                                                                       \
        if (staged) hipLaunchKernelGGL((basis_kernel<TT, true, EE>), g, b, lds, st, segs_dev, n_segs, n_items, spline_lds); \
        else hipLaunchKernelGGL((basis_kernel<TT, false, EE>), g, b, lds, st, segs_dev, n_segs, n_items, 0);  \
    } while (0)
#define NAO_BASIS_EXTRA(TT)                                           \
    do {                                                              \
        if (extra == EXTRA_GRAD) NAO_BASIS_LAUNCH(TT, EXTRA_GRAD);    \
        else if (extra == EXTRA_GGA_L) NAO_BASIS_LAUNCH(TT, EXTRA_GGA_L); \
        else if (extra == EXTRA_KS_L) NAO_BASIS_LAUNCH(TT, EXTRA_KS_L); \
        else if (extra == EXTRA_GRAD_H) NAO_BASIS_LAUNCH(TT, EXTRA_GRAD_H); \
        else NAO_BASIS_LAUNCH(TT, EXTRA_NONE);                        \
    } while (0)
    if (fp32_out) NAO_BASIS_EXTRA(float);
    else NAO_BASIS_EXTRA(double);
#undef NAO_BASIS_EXTRA
#undef NAO_BASIS_LAUNCH
    return hipGetLastError();
}









// ------------------------------------------------------------------------------------------
// Contractions with one value per lane per operand: FP64 (v_mfma_f64_16x16x4f64) and FP32
// (v_mfma_f32_16x16x4f32).  Operand layouts of both: A lane l holds A[l%16][l/16], B lane l
// holds B[l/16][l%16].  The result register r of lane l is D[l/16 + 4r][l%16] for FP64 and
// D[4(l/16) + r][l%16] for FP32 (measured on gfx950).

// Sum over the 16 lanes of each DPP row (lanes 16 r .. 16 r + 15), every lane receiving the sum:
// quad swaps (xor 1, xor 2), then the half-row and row mirrors pair the quads.
template <int CTRL>
__device__ inline double dpp_move(double x)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ inline double row_sum16(double v)
{
    v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141>(v);  // row_half_mirror
    v += dpp_move<0x140>(v);  // row_mirror
    return v;
}

template <typename T> struct Mma;
template <> struct Mma<double> {
    typedef d4 acc_t;
    static __device__ inline acc_t zero() { return d4{0.0, 0.0, 0.0, 0.0}; }
    static __device__ inline acc_t op(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct Mma<float> {
    typedef f4 acc_t;
    static __device__ inline acc_t zero() { return f4{0.f, 0.f, 0.f, 0.f}; }
    static __device__ inline acc_t op(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lk, int r) { return 4 * lk + r; }
};

// Hamiltonian: per work item one 64x64 tile pair (I <= J) of a unit,
//   H[I, J] += (w v Phi[:, I])^T Phi[:, J];
// K loop over the unit's points in double-buffered chunks of 16 (register prefetch of the
// next chunk while the MFMAs of the current one run); four waves, each a 32x32 quarter as
// 2x2 MFMA blocks; FP64 atomics into the upper triangle of H.  T = FP32 accumulates a unit
// (<= 256 points) in FP32 before the FP64 atomics.  The FP32 form (the staging below applies
// w v once per value as it is stashed) is faster than the directly-loaded form; FP64 uses the
// latter.
template <typename T>
__global__ __launch_bounds__(256, 4) void h_kernel(const DevSeg* __restrict__ segs, int n_segs, int64_t total)
{
    typedef Mma<T> M;
    constexpr int HK = KCHUNK;              // points per chunk
    constexpr int HQ = HK * TILE / 256;     // values per thread per chunk and operand
    // rows padded so that two consecutive rows start half a 128-byte bank period apart: the MFMA
    // reads of a wave's first 32 lanes (16 columns of two rows) then fall in distinct banks
    constexpr int PAD = 64 / (int)sizeof(T);
    __shared__ T As[2][HK][TILE + PAD];
    __shared__ T Bs[2][HK][TILE + PAD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    for (int64_t v_ = blockIdx.x; v_ < xcd_span(total); v_ += gridDim.x) {
        const int64_t b = xcd_item(v_, total);
        if (b >= total) continue;
        const int s = find_segment(segs, n_segs, b, [](const DevSeg& g) { return g.item_prefix; });
        const DevSeg& sg = segs[s];
        const HItem it = static_cast<const HItem*>(sg.items)[sg.item_begin + (b - sg.item_prefix)];
        const DevUnit u = sg.units[it.unit];
        gp<const T> __restrict__ phi = gptr(static_cast<const T*>(sg.phi) + u.out_offset);
        gp<const double> __restrict__ wv = gptr(sg.wv + u.point_begin);
        const int np = u.n_points, ld = u.ld;
        const int I0 = it.ti * TILE, J0 = it.tj * TILE;
        const int n_chunks = (np + HK - 1) / HK;

        if (np <= 0) continue;
        // Loads are issued unconditionally (rows clamped into the unit) and only consumed at
        // the stash after the next chunk's MFMAs, so that they stay in flight meanwhile.
        T ra[HQ], rb[HQ];
        double rw[HQ];
        auto fetch = [&](int c) {
#pragma unroll
            for (int q = 0; q < HQ; ++q) {
                const int e = tid + 256 * q;
                const int pc = min(c * HK + (e >> 6), np - 1), col = e & 63;
                gp<const T> rowp = phi + (int64_t)pc * ld;
                ra[q] = rowp[I0 + col];
                rb[q] = rowp[J0 + col];
                rw[q] = wv[pc];
            }
        };
        auto stash = [&](int c, int buf) {
#pragma unroll
            for (int q = 0; q < HQ; ++q) {
                const int e = tid + 256 * q;
                const bool ok = c * HK + (e >> 6) < np;
                As[buf][e >> 6][e & 63] = ok ? T((double)ra[q] * rw[q]) : T(0);
                Bs[buf][e >> 6][e & 63] = ok ? rb[q] : T(0);
            }
        };
        // global indices of this lane's output rows and columns, needed only after the K loop
        gp<const int32_t> __restrict__ fn = gptr(sg.unit_fn + u.fn_begin);
        int32_t gI[2][4], gJ[2];
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
#pragma unroll
            for (int r = 0; r < 4; ++r) gI[ib][r] = fn[min(I0 + wr * 32 + ib * 16 + M::row(lk, r), u.m - 1)];
            gJ[ib] = fn[min(J0 + wc * 32 + ib * 16 + lr, u.m - 1)];
        }

        typename M::acc_t acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = M::zero();
        // On a diagonal tile pair the wave of the strictly lower quarter only stages data.
        auto k_loop = [&](auto with_mfma) {
            fetch(0);
            stash(0, 0);
            __syncthreads();
            for (int c = 0; c < n_chunks; ++c) {
                const int buf = c & 1;
                if (c + 1 < n_chunks) fetch(c + 1);
                if (decltype(with_mfma)::value) {
#pragma unroll
                    for (int kk = 0; kk < HK / 4; ++kk) {
                        const int kr = kk * 4 + lk;
                        const T a0 = As[buf][kr][wr * 32 + lr];
                        const T a1 = As[buf][kr][wr * 32 + 16 + lr];
                        const T b0 = Bs[buf][kr][wc * 32 + lr];
                        const T b1 = Bs[buf][kr][wc * 32 + 16 + lr];
                        acc[0][0] = M::op(a0, b0, acc[0][0]);
                        acc[0][1] = M::op(a0, b1, acc[0][1]);
                        acc[1][0] = M::op(a1, b0, acc[1][0]);
                        acc[1][1] = M::op(a1, b1, acc[1][1]);
                    }
                }
                if (c + 1 < n_chunks) stash(c + 1, buf ^ 1);
                __syncthreads();
            }
        };
        const bool diag = it.ti == it.tj;
        if (diag && wr > wc) {
            k_loop(std::false_type{});
            continue;
        }
        k_loop(std::true_type{});

        gp<double> __restrict__ H = gptr(sg.H);
        const int64_t ldh = sg.ld;
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wr * 32 + ib * 16 + M::row(lk, r);
                    const int col = wc * 32 + jb * 16 + lr;
                    const int ci = I0 + row, cj = J0 + col;
                    if (ci < u.m && cj < u.m && (!diag || row <= col))
                        gadd(H + (int64_t)gI[ib][r] * ldh + gJ[jb], (double)acc[ib][jb][r]);
                }
    }
}

// Hamiltonian, staged by direct global-to-LDS loads: per work item one 64x64 tile pair (I <= J)
// of a unit, H[I, J] += (w v Phi[:, I])^T Phi[:, J].  K = the unit's points in chunks of KC
// held in an S-stage ring in LDS: the loads of chunk c + S - 1 are issued (global_load_lds, 16
// bytes per lane, no registers involved) while the MFMAs of chunk c run, so S - 1 chunks are in
// flight.  w v of the unit's points is staged the same way once per item; the A operand is
// scaled by it as it is read (loads of rows beyond the unit's last point are clamped into the
// unit, and the w v of such rows is taken as zero).  On a diagonal pair (I == J) one tile
// serves both operands.  Four waves, each a 32x32 quarter as 2x2 MFMA blocks; FP64 atomics
// into the upper triangle of H.  The 16-byte loads need 16-byte aligned rows: every
// basis-value block starts on a 64-value boundary of its buffer and ld is a multiple of 64.
template <typename T, int KC, int S>
__global__ __launch_bounds__(256) void h_kernel_dma(const DevSeg* __restrict__ segs, int n_segs, int64_t total)
{
    typedef Mma<T> M;
    constexpr int ROW_SLOTS = TILE * (int)sizeof(T) / 16;     // 16-byte slots per tile row
    constexpr int ROWS_PER_LOAD = 64 / ROW_SLOTS;            // tile rows one wave load covers
    constexpr int LOADS = KC / ROWS_PER_LOAD / 4;            // wave loads per operand and chunk
    static_assert(LOADS >= 1 && KC % 4 == 0 && MAX_UNIT_POINTS % KC == 0, "chunk geometry");
    __shared__ __align__(16) T st[S][2][KC][TILE];           // [stage][operand A, B][point][column]
    __shared__ double wvs[MAX_UNIT_POINTS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    // this lane's slot of every wave load: tile row (within the load's rows) and 16-byte column slot
    const int slot_row = lane / ROW_SLOTS, slot_col = (lane % ROW_SLOTS) * (16 / (int)sizeof(T));
    for (int64_t v_ = blockIdx.x; v_ < xcd_span(total); v_ += gridDim.x) {
        const int64_t b = xcd_item(v_, total);
        if (b >= total) continue;
        const int s = find_segment(segs, n_segs, b, [](const DevSeg& g) { return g.item_prefix; });
        const DevSeg& sg = segs[s];
        const HItem it = static_cast<const HItem*>(sg.items)[sg.item_begin + (b - sg.item_prefix)];
        const DevUnit u = sg.units[it.unit];
        const int np = u.n_points, ld = u.ld;
        if (np <= 0) continue;
        const T* phi = static_cast<const T*>(sg.phi) + u.out_offset;
        const int I0 = it.ti * TILE, J0 = it.tj * TILE;
        const bool diag = it.ti == it.tj;
        const int n_chunks = (np + KC - 1) / KC;
        const int per_chunk = diag ? LOADS : 2 * LOADS;  // wave loads per chunk (wave-uniform)

        // every wave must be done reading the previous item's stages and w v before they are
        // refilled (its loads into them have all completed; its atomics need not)
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        // w v of the unit's points into wvs, 32 per wave load (two 4-byte halves per value), point
        // indices clamped into the unit; rows at and beyond np are masked where they are used
        {
            const double* wv = sg.wv + u.point_begin;
            const int nq = (n_chunks * KC + 31) / 32;
            for (int q = wave; q < nq; q += 4) {
                const int d = min(32 * q + (lane >> 1), np - 1);
                const char* src = reinterpret_cast<const char*>(wv + d) + 4 * (lane & 1);
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                                 (__attribute__((address_space(3))) void*)&wvs[32 * q], 4, 0, 0);
            }
        }
        auto issue = [&](int c) {
            const int stg = c % S;
#pragma unroll
            for (int op = 0; op < 2; ++op) {
                if (op == 1 && diag) break;
                const int col0 = op == 0 ? I0 : J0;
#pragma unroll
                for (int q = 0; q < LOADS; ++q) {
                    const int r0 = (wave * LOADS + q) * ROWS_PER_LOAD;  // first tile row of this load
                    const int p = min(c * KC + r0 + slot_row, np - 1);
                    const T* src = phi + (int64_t)p * ld + col0 + slot_col;
                    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)src,
                                                     (__attribute__((address_space(3))) void*)&st[stg][op][r0][0],
                                                     16, 0, 0);
                }
            }
        };
        // wait until at most `later` chunks' loads of this wave are outstanding (vmcnt counts wave
        // loads in issue order), and for the LDS reads of the last chunk, then barrier
        auto sync_chunk = [&](int later) {
            const int n = __builtin_amdgcn_readfirstlane(later * per_chunk);  // at most (S - 2) * 2 * LOADS
            switch (n) {
#define NAO_VMWAIT(N) \
    case N: __builtin_amdgcn_s_waitcnt(((N) & 0xF) | (((N) >> 4) << 14) | (0x7 << 4)); break;
                NAO_VMWAIT(0) NAO_VMWAIT(1) NAO_VMWAIT(2) NAO_VMWAIT(3) NAO_VMWAIT(4) NAO_VMWAIT(5)
                NAO_VMWAIT(6) NAO_VMWAIT(7) NAO_VMWAIT(8) NAO_VMWAIT(9) NAO_VMWAIT(10) NAO_VMWAIT(11)
                NAO_VMWAIT(12) NAO_VMWAIT(13) NAO_VMWAIT(14) NAO_VMWAIT(15) NAO_VMWAIT(16)
#undef NAO_VMWAIT
            default: __builtin_amdgcn_s_waitcnt(0x7 << 4); break;  // vmcnt(0), lgkmcnt(0)
            }
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
        };

        gp<const int32_t> __restrict__ fn = gptr(sg.unit_fn + u.fn_begin);
        int32_t gI[2][4], gJ[2];
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
#pragma unroll
            for (int r = 0; r < 4; ++r) gI[ib][r] = fn[min(I0 + wr * 32 + ib * 16 + M::row(lk, r), u.m - 1)];
            gJ[ib] = fn[min(J0 + wc * 32 + ib * 16 + lr, u.m - 1)];
        }
        typename M::acc_t acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = M::zero();
        const bool compute = !(diag && wr > wc);  // the strictly lower quarter of a diagonal pair
        const int ob = diag ? 0 : 1;              // operand B's slot in the stages

        for (int c = 0; c < S - 1 && c < n_chunks; ++c) issue(c);
        for (int c = 0; c < n_chunks; ++c) {
            sync_chunk(min(S - 2, n_chunks - 1 - c));
            if (c + S - 1 < n_chunks) issue(c + S - 1);
            if (compute) {
                const int stg = c % S;
#pragma unroll
                for (int kk = 0; kk < KC / 4; ++kk) {
                    const int kr = kk * 4 + lk;
                    const double w = c * KC + kr < np ? wvs[c * KC + kr] : 0.0;
                    const T a0 = T((double)st[stg][0][kr][wr * 32 + lr] * w);
                    const T a1 = T((double)st[stg][0][kr][wr * 32 + 16 + lr] * w);
                    const T b0 = st[stg][ob][kr][wc * 32 + lr];
                    const T b1 = st[stg][ob][kr][wc * 32 + 16 + lr];
                    acc[0][0] = M::op(a0, b0, acc[0][0]);
                    acc[0][1] = M::op(a0, b1, acc[0][1]);
                    acc[1][0] = M::op(a1, b0, acc[1][0]);
                    acc[1][1] = M::op(a1, b1, acc[1][1]);
                }
            }
        }
        if (!compute) continue;
        gp<double> __restrict__ H = gptr(sg.H);
        const int64_t ldh = sg.ld;
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wr * 32 + ib * 16 + M::row(lk, r);
                    const int col = wc * 32 + jb * 16 + lr;
                    const int ci = I0 + row, cj = J0 + col;
                    if (ci < u.m && cj < u.m && (!diag || row <= col))
                        gadd(H + (int64_t)gI[ib][r] * ldh + gJ[jb], (double)acc[ib][jb][r]);
                }
    }
}

// Hamiltonian with a vector field (GGA form of eq. batch_matrix_mult): per item one 64x64 tile
// pair (I <= J) of a unit, H[I, J] += Phi_I^T L_J + L_I^T Phi_J, with L = (w v / 2) Phi +
// (w a) . grad Phi written by the basis launch (or the kinetic L).  Schedule of h_kernel with
// K = points in double-buffered chunks of 8 (two products per chunk), four waves of 32x32, FP64
// atomics into the upper triangle.
template <typename T>
__global__ __launch_bounds__(256, 4) void h_kernel_gga(const DevSeg* __restrict__ segs, int n_segs, int64_t total)
{
    typedef Mma<T> M;
    constexpr int GK = 8;  // points per chunk: half the LDS of 16-point chunks, so that four
                           // workgroups fit a CU (20 % faster than two with 16-point chunks)
    constexpr int HQ = GK * TILE / 256;  // values per thread per chunk and operand
    __shared__ T Ps[2][2][GK][TILE + 2];  // [buffer][I, J] basis values
    __shared__ T Ls[2][2][GK][TILE + 2];  // [buffer][I, J] L values
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    for (int64_t v_ = blockIdx.x; v_ < xcd_span(total); v_ += gridDim.x) {
        const int64_t b = xcd_item(v_, total);
        if (b >= total) continue;
        const int s = find_segment(segs, n_segs, b, [](const DevSeg& g) { return g.item_prefix; });
        const DevSeg& sg = segs[s];
        const HItem it = static_cast<const HItem*>(sg.items)[sg.item_begin + (b - sg.item_prefix)];
        const DevUnit u = sg.units[it.unit];
        gp<const T> __restrict__ phi = gptr(static_cast<const T*>(sg.phi) + u.out_offset);
        gp<const T> __restrict__ lv = gptr(static_cast<const T*>(sg.gphi) + u.out_offset);
        const int np = u.n_points, ld = u.ld;
        if (np <= 0) continue;
        const int I0 = it.ti * TILE, J0 = it.tj * TILE;
        const int n_chunks = (np + GK - 1) / GK;

        T rp[2][HQ], rl[2][HQ];  // [I, J] basis and L values of the next chunk
        auto fetch = [&](int c) {
#pragma unroll
            for (int q = 0; q < HQ; ++q) {
                const int e = tid + 256 * q;
                const int64_t o = (int64_t)min(c * GK + (e >> 6), np - 1) * ld + (e & 63);
                rp[0][q] = phi[o + I0];
                rp[1][q] = phi[o + J0];
                rl[0][q] = lv[o + I0];
                rl[1][q] = lv[o + J0];
            }
        };
        auto stash = [&](int c, int buf) {
#pragma unroll
            for (int q = 0; q < HQ; ++q) {
                const int e = tid + 256 * q;
                const bool ok = c * GK + (e >> 6) < np;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    Ps[buf][t][e >> 6][e & 63] = ok ? rp[t][q] : T(0);
                    Ls[buf][t][e >> 6][e & 63] = ok ? rl[t][q] : T(0);
                }
            }
        };
        gp<const int32_t> __restrict__ fn = gptr(sg.unit_fn + u.fn_begin);
        int32_t gI[2][4], gJ[2];
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
#pragma unroll
            for (int r = 0; r < 4; ++r) gI[ib][r] = fn[min(I0 + wr * 32 + ib * 16 + M::row(lk, r), u.m - 1)];
            gJ[ib] = fn[min(J0 + wc * 32 + ib * 16 + lr, u.m - 1)];
        }

        typename M::acc_t acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = M::zero();
        auto k_loop = [&](auto with_mfma) {
            fetch(0);
            stash(0, 0);
            __syncthreads();
            for (int c = 0; c < n_chunks; ++c) {
                const int buf = c & 1;
                if (c + 1 < n_chunks) fetch(c + 1);
                if (decltype(with_mfma)::value) {
#pragma unroll
                    for (int kk = 0; kk < GK / 4; ++kk) {
                        const int kr = kk * 4 + lk;
                        // Phi_I^T L_J, then L_I^T Phi_J
                        const T a0 = Ps[buf][0][kr][wr * 32 + lr], a1 = Ps[buf][0][kr][wr * 32 + 16 + lr];
                        const T b0 = Ls[buf][1][kr][wc * 32 + lr], b1 = Ls[buf][1][kr][wc * 32 + 16 + lr];
                        acc[0][0] = M::op(a0, b0, acc[0][0]);
                        acc[0][1] = M::op(a0, b1, acc[0][1]);
                        acc[1][0] = M::op(a1, b0, acc[1][0]);
                        acc[1][1] = M::op(a1, b1, acc[1][1]);
                        const T c0 = Ls[buf][0][kr][wr * 32 + lr], c1 = Ls[buf][0][kr][wr * 32 + 16 + lr];
                        const T d0 = Ps[buf][1][kr][wc * 32 + lr], d1 = Ps[buf][1][kr][wc * 32 + 16 + lr];
                        acc[0][0] = M::op(c0, d0, acc[0][0]);
                        acc[0][1] = M::op(c0, d1, acc[0][1]);
                        acc[1][0] = M::op(c1, d0, acc[1][0]);
                        acc[1][1] = M::op(c1, d1, acc[1][1]);
                    }
                }
                if (c + 1 < n_chunks) stash(c + 1, buf ^ 1);
                __syncthreads();
            }
        };
        const bool diag = it.ti == it.tj;
        if (diag && wr > wc) {  // the strictly lower quarter of a diagonal tile pair only stages data
            k_loop(std::false_type{});
            continue;
        }
        k_loop(std::true_type{});

        gp<double> __restrict__ H = gptr(sg.H);
        const int64_t ldh = sg.ld;
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wr * 32 + ib * 16 + M::row(lk, r);
                    const int col = wc * 32 + jb * 16 + lr;
                    const int ci = I0 + row, cj = J0 + col;
                    if (ci < u.m && cj < u.m && (!diag || row <= col))
                        gadd(H + (int64_t)gI[ib][r] * ldh + gJ[jb], (double)acc[ib][jb][r]);
                }
    }
}

// Hamiltonian with 128x128 tile pairs: eight waves, each a 32x64 block (2x4 MFMA blocks), so
// that every staged basis value feeds twice as many MFMAs as in the 64-wide kernel.  Chunks
// of 16 points, double-buffered as above.
constexpr int WTILE = 128;

template <typename T>
__global__ __launch_bounds__(512) void h_kernel_wide(const DevSeg* __restrict__ segs, int n_segs, int64_t total)
{
    typedef Mma<T> M;
    __shared__ T As[2][KCHUNK][WTILE + 2];
    __shared__ T Bs[2][KCHUNK][WTILE + 2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;  // rows 32 wr .. 32 wr + 31, columns 64 wc .. 64 wc + 63
    const int lr = lane & 15, lk = lane >> 4;
    for (int64_t v_ = blockIdx.x; v_ < xcd_span(total); v_ += gridDim.x) {
        const int64_t b = xcd_item(v_, total);
        if (b >= total) continue;
        const int s = find_segment(segs, n_segs, b, [](const DevSeg& g) { return g.item_prefix; });
        const DevSeg& sg = segs[s];
        const HItem it = static_cast<const HItem*>(sg.items)[sg.item_begin + (b - sg.item_prefix)];
        const DevUnit u = sg.units[it.unit];
        gp<const T> __restrict__ phi = gptr(static_cast<const T*>(sg.phi) + u.out_offset);
        gp<const double> __restrict__ wv = gptr(sg.wv + u.point_begin);
        const int np = u.n_points, ld = u.ld;
        const int I0 = it.ti * WTILE, J0 = it.tj * WTILE;
        const int n_chunks = (np + KCHUNK - 1) / KCHUNK;

        if (np <= 0) continue;
        T ra[4], rb[4];
        double rw[4];
        auto fetch = [&](int c) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = tid + 512 * q;
                const int pc = min(c * KCHUNK + (e >> 7), np - 1), col = e & 127;
                gp<const T> rowp = phi + (int64_t)pc * ld;
                ra[q] = rowp[I0 + col];
                rb[q] = rowp[J0 + col];
                rw[q] = wv[pc];
            }
        };
        auto stash = [&](int c, int buf) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = tid + 512 * q;
                const bool ok = c * KCHUNK + (e >> 7) < np;
                As[buf][e >> 7][e & 127] = ok ? T((double)ra[q] * rw[q]) : T(0);
                Bs[buf][e >> 7][e & 127] = ok ? rb[q] : T(0);
            }
        };
        gp<const int32_t> __restrict__ fn = gptr(sg.unit_fn + u.fn_begin);
        int32_t gI[2][4], gJ[4];
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
            for (int r = 0; r < 4; ++r) gI[ib][r] = fn[min(I0 + wr * 32 + ib * 16 + M::row(lk, r), u.m - 1)];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) gJ[jb] = fn[min(J0 + wc * 64 + jb * 16 + lr, u.m - 1)];

        typename M::acc_t acc[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = M::zero();
        fetch(0);
        stash(0, 0);
        __syncthreads();
        for (int c = 0; c < n_chunks; ++c) {
            const int buf = c & 1;
            if (c + 1 < n_chunks) fetch(c + 1);
#pragma unroll
            for (int kk = 0; kk < KCHUNK / 4; ++kk) {
                const int kr = kk * 4 + lk;
                T a[2], bq[4];
#pragma unroll
                for (int i = 0; i < 2; ++i) a[i] = As[buf][kr][wr * 32 + i * 16 + lr];
#pragma unroll
                for (int j = 0; j < 4; ++j) bq[j] = Bs[buf][kr][wc * 64 + j * 16 + lr];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = M::op(a[i], bq[j], acc[i][j]);
            }
            if (c + 1 < n_chunks) stash(c + 1, buf ^ 1);
            __syncthreads();
        }

        gp<double> __restrict__ H = gptr(sg.H);
        const int64_t ldh = sg.ld;
        const bool diag = it.ti == it.tj;
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
            for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wr * 32 + ib * 16 + M::row(lk, r);
                    const int col = wc * 64 + jb * 16 + lr;
                    const int ci = I0 + row, cj = J0 + col;
                    if (ci < u.m && cj < u.m && (!diag || row <= col))
                        gadd(H + (int64_t)gI[ib][r] * ldh + gJ[jb], (double)acc[ib][jb][r]);
                }
    }
}

// Density: per work item one 64-wide column tile J of a unit,
//   T[:, J] = sum_{I <= J} c_IJ Phi[:, I] D[I, J]   (c = 2 off the diagonal tile, 1 on it,
//             the diagonal tile read from the upper triangle of D),
//   n_p += sum_{j in J} T[p, j] Phi[p, j].
// Rows = the unit's points (<= 256: 16 row blocks), K = basis functions in chunks of KC staged
// through LDS (two buffers when DB, else one buffer and a second barrier per chunk); the next
// chunk is prefetched into registers while the MFMAs of the current one run.  NW waves: wave w
// owns column block w % 4 and row blocks w / 4, w / 4 + NW / 4, ...  T = FP32 accumulates the
// whole column tile in FP32; the row dot and the sum over tiles and units are FP64.
//
// KIND = NK_GRADIENT: T[:, J] = Phi D[:, J] over the whole list (coefficient 1, the lower
// triangle read transposed) and four row dots, n and grad n = 2 T . grad Phi.
// KIND = NK_FORCE: the list is walked twice, M[:, J] = diag(w) (h_KS Phi) D[:, J] - diag(w) Phi
// Q[:, J] with h_KS phi = v phi - lap phi / 2 (w h_KS phi written by the basis launch beside the
// gradients, four values per basis value: x, y, z, w h_KS phi), and the epilogue takes column
// sums, f_j += sum_p grad phi_pj M_pj, into the per-function accumulator fb[N_b][3].
enum NKind { NK_DENSITY = 0, NK_GRADIENT = 1, NK_FORCE = 2 };
template <typename T, int NW, int KC, bool DB, int KIND = NK_DENSITY>
__global__ __launch_bounds__(64 * NW) void n_kernel(const DevSeg* __restrict__ segs, int n_segs, int64_t total)
{
    typedef Mma<T> M;
    constexpr bool GRAD = KIND == NK_GRADIENT;
    constexpr bool FORCE = KIND == NK_FORCE;
    constexpr bool FULL = KIND != NK_DENSITY;  // contraction over the whole list
    constexpr int NT = 64 * NW;                              // threads
    constexpr int RB = 64 / NW;                              // row blocks per wave (16 row x 4 column blocks)
    constexpr int RS = NW / 4;                               // row-block stride between the waves of a column
    constexpr int NA = MAX_UNIT_POINTS * KC / NT;            // basis values per thread per chunk
    constexpr int ND = KC * TILE / NT;                       // D values per thread per chunk
    constexpr int NB = DB ? 2 : 1;                           // LDS buffers
    static_assert(ND >= 1 && NA % 2 == 0 && RB % 4 == 0 && NT % TILE == 0 && TILE % KC == 0 && KC % 4 == 0,
                  "tile geometry");
    static_assert(!FORCE || RS * TILE * 3 <= 4 * MAX_UNIT_POINTS, "force partials fit in red");
    // SLOT (density, gradient): basis values move as 16-byte slots (VPS values of one row), are
    // staged in rows of KC values whose slots are XOR-swizzled by row, and are read back a whole
    // slot per lane, so that the rows one 128-byte pass of a read touches fall in distinct banks
    // (the MFMA steps take the chunk's columns in slot order, A and B alike).  The forces, whose D
    // pass stages every fourth value of the basis launch's extra block, keep rows padded to KC + 1,
    // and so does FP32 (faster so: its slots hold four columns, its rows half the bytes).
    constexpr bool SLOT = !FORCE && sizeof(T) == 8;
    constexpr int VPS = 16 / (int)sizeof(T);                 // values per slot
    constexpr int SPR = KC / VPS;                            // slots per staged row
    constexpr int ROWS_128B = 128 / (KC * (int)sizeof(T));   // staged rows per 128 bytes (the bank period)
    constexpr int AW = SLOT ? KC : KC + 1;                   // staged row length
    static_assert(!SLOT || (SPR >= 4 && SPR % 4 == 0 && ROWS_128B >= 1 && (SPR & (SPR - 1)) == 0), "slot geometry");
    typedef T slot_t __attribute__((ext_vector_type(VPS)));
    __shared__ __align__(16) T As[NB][MAX_UNIT_POINTS][AW];
    __shared__ T Bs[NB][KC][TILE + 2];
    constexpr int NQ = GRAD ? 4 : 1;                         // row dots: n, or n and the three gradient components
    __shared__ double red[NQ][4][MAX_UNIT_POINTS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cb = wave & 3, rh = wave >> 2;  // column block; row blocks rh, rh + RS, ...
    const int lr = lane & 15, lk = lane >> 4;
    // staged position of slot j of row `row` within a buffer (SLOT)
    auto a_slot = [](int row, int j) { return row * KC + ((j ^ ((row / ROWS_128B) & (SPR - 1))) * VPS); };
    for (int64_t v_ = blockIdx.x; v_ < xcd_span(total); v_ += gridDim.x) {
        const int64_t b = xcd_item(v_, total);
        if (b >= total) continue;
        const int s = find_segment(segs, n_segs, b, [](const DevSeg& g) { return g.item_prefix; });
        const DevSeg& sg = segs[s];
        const NItem it = static_cast<const NItem*>(sg.items)[sg.item_begin + (b - sg.item_prefix)];
        const DevUnit u = sg.units[it.unit];
        gp<const T> __restrict__ phi = gptr(static_cast<const T*>(sg.phi) + u.out_offset);
        gp<const int32_t> __restrict__ fn = gptr(sg.unit_fn + u.fn_begin);
        gp<const double> __restrict__ D = gptr(sg.D);
        const int64_t ldd = sg.ld;
        const int np = u.n_points, ld = u.ld, m = u.m;
        if (np <= 0 || m <= 0) continue;
        const int P = (np + 15) >> 4;
        const int J0 = it.tj * TILE;
        // this wave's 16 output columns hold list entries (the last tile of a unit is padded)
        const bool col_live = __builtin_amdgcn_readfirstlane(J0 + cb * 16 < m);
        // chunk c covers columns KC c .. KC c + KC - 1: the tiles I <= J, or all tiles for the
        // gradient (T = Phi D over the whole list); the forces walk the list once against D and
        // once against Q (chunk c + half covers the columns of chunk c).  Chunks that start at
        // or beyond m hold only the zero padding of the basis values and are left out.
        const int half = min(FULL ? (m + TILE - 1) / TILE * (TILE / KC) : (it.tj + 1) * (TILE / KC), (m + KC - 1) / KC);
        const int n_chunks = FORCE ? 2 * half : half;
        auto col0 = [&](int c) { return KC * (FORCE && c >= half ? c - half : c); };
        const int cjd = J0 + (tid & (TILE - 1));              // this thread's D column in every chunk
        const int64_t gjd = fn[min(cjd, m - 1)];

        // F = rows staged (RB row blocks per wave's share, or RB / 2 when the unit has at most
        // 128 points); R = this wave's row blocks below the unit's last one (the waves of one
        // SIMD share a column block and split the rows, so a SIMD issues MFMAs for exactly the
        // unit's row blocks).  Loads are issued with clamped (in-bounds) addresses and consumed
        // only at the stash after the current chunk's MFMAs.
        auto run = [&](auto rows_staged, auto rows_own) {
            constexpr int F = decltype(rows_staged)::value;
            constexpr int R = decltype(rows_own)::value;
            constexpr int NAR = NA * F / RB;
            constexpr int ROWS = F * RS * 16;                           // rows staged
            constexpr int NSL = SLOT ? (ROWS * SPR + NT - 1) / NT : 1;  // slots per thread
            constexpr bool SL_ALL = ROWS * SPR % NT == 0;               // every thread takes NSL slots
            T pa[SLOT ? 1 : NAR];
            slot_t ps[NSL];
            double pd[ND];
            // list indices of the D rows: those of chunk c + 1 are loaded during chunk c
            int32_t gcur[ND], gnxt[ND];
            auto load_idx = [&](int c, int32_t* g) {
#pragma unroll
                for (int q = 0; q < ND; ++q) g[q] = fn[min(col0(c) + (tid >> 6) + (NT / TILE) * q, m - 1)];
            };
            // forces: weights of this thread's staged rows, -w for the Q pass
            double sw[FORCE ? NAR : 1];
            if constexpr (FORCE) {
                gp<const double> pw = gptr(sg.sys->pw + u.point_begin);
#pragma unroll
                for (int q = 0; q < NAR; ++q) sw[q] = -pw[min((tid + NT * q) / KC, np - 1)];
            }
            auto fetch = [&](int c) {
                if constexpr (SLOT) {
#pragma unroll
                    for (int q = 0; q < NSL; ++q) {
                        const int e = tid + NT * q;  // slot e % SPR of row e / SPR
                        if (SL_ALL || e < ROWS * SPR)
                            ps[q] = *reinterpret_cast<gp<const slot_t>>(
                                phi + (int64_t)min(e / SPR, np - 1) * ld + col0(c) + (e % SPR) * VPS);
                    }
                }
#pragma unroll
                for (int q = 0; q < (SLOT ? 0 : NAR); ++q) {
                    const int e = tid + NT * q;
                    const int64_t el = (int64_t)min(e / KC, np - 1) * ld + col0(c) + (e % KC);
                    // forces: the D pass takes w h_KS phi (fourth value of the basis launch's
                    // gradient block), the Q pass phi
                    if (FORCE && c < half) pa[q] = gptr(static_cast<const T*>(sg.gphi) + 4 * u.out_offset)[4 * el + 3];
                    else pa[q] = phi[el];
                }
                const bool diag = c / (TILE / KC) == it.tj;
                gp<const double> src = FORCE && c >= half ? gptr(sg.Q) : D;
#pragma unroll
                for (int q = 0; q < ND; ++q) {
                    const int ci = col0(c) + (tid >> 6) + (NT / TILE) * q;
                    // upper triangle only: the diagonal tile's lower part (every tile's, for the
                    // gradient and the forces) is read transposed
                    const bool lower = (FULL || diag) && ci > cjd;
                    pd[q] = src[lower ? gjd * ldd + gcur[q] : (int64_t)gcur[q] * ldd + gjd];
                }
                load_idx(c + 1, gnxt);
            };
            auto stash = [&](int c, int buf) {
#pragma unroll
                for (int q = 0; q < ND; ++q) gcur[q] = gnxt[q];
                const bool diag = c / (TILE / KC) == it.tj;
                if constexpr (SLOT) {
#pragma unroll
                    for (int q = 0; q < NSL; ++q) {
                        const int e = tid + NT * q;
                        if (SL_ALL || e < ROWS * SPR)
                            *reinterpret_cast<slot_t*>(&As[buf][0][0] + a_slot(e / SPR, e % SPR)) =
                                e / SPR < np ? ps[q] : slot_t(T(0));
                    }
                }
#pragma unroll
                for (int q = 0; q < (SLOT ? 0 : NAR); ++q) {
                    const int e = tid + NT * q;
                    T x = pa[q];
                    if constexpr (FORCE) {  // Q pass: -w phi (the D pass staged w h_KS phi as it is)
                        if (c >= half) x = T((double)x * sw[q]);
                    }
                    As[buf][e / KC][e % KC] = (e / KC) < np ? x : T(0);
                }
#pragma unroll
                for (int q = 0; q < ND; ++q) {
                    const int e = tid + NT * q;
                    const bool ok = col0(c) + (e >> 6) < m && cjd < m;
                    Bs[buf][e >> 6][e & 63] = ok ? T((FULL || diag) ? pd[q] : 2.0 * pd[q]) : T(0);
                }
            };

            typename M::acc_t acc[R > 0 ? R : 1];
#pragma unroll
            for (int i = 0; i < R; ++i) acc[i] = M::zero();
            load_idx(0, gcur);
            fetch(0);
            stash(0, 0);
            __syncthreads();
            auto mfma_chunk = [&](int buf) {
                if (!col_live) return;  // this wave's 16 columns lie in the tile's padding
                if constexpr (SLOT) {
                    // lane group lk reads slots lk + 4 h of its rows; step (h, e) takes column
                    // VPS (lk + 4 h) + e of the chunk
#pragma unroll
                    for (int h = 0; h < SPR / 4; ++h) {
                        slot_t a[R > 0 ? R : 1];
#pragma unroll
                        for (int q = 0; q < R; ++q)
                            a[q] = *reinterpret_cast<const slot_t*>(&As[buf][0][0] + a_slot((RS * q + rh) * 16 + lr, lk + 4 * h));
#pragma unroll
                        for (int e = 0; e < VPS; ++e) {
                            const T bv = Bs[buf][VPS * (lk + 4 * h) + e][cb * 16 + lr];
#pragma unroll
                            for (int q = 0; q < R; ++q) acc[q] = M::op(a[q][e], bv, acc[q]);
                        }
                    }
                } else {
#pragma unroll
                    for (int kk = 0; kk < KC / 4; ++kk) {
                        const T bv = Bs[buf][kk * 4 + lk][cb * 16 + lr];
#pragma unroll
                        for (int q = 0; q < R; ++q) acc[q] = M::op(As[buf][(RS * q + rh) * 16 + lr][kk * 4 + lk], bv, acc[q]);
                    }
                }
            };
            // straight-line body (the last chunk peeled off) so that the scheduler can
            // interleave the next chunk's stash with this chunk's MFMAs
            for (int c = 0; c + 1 < n_chunks; ++c) {
                const int buf = DB ? (c & 1) : 0;
                fetch(c + 1);
                mfma_chunk(buf);
                if (!DB) __syncthreads();  // every wave is done with the only buffer
                stash(c + 1, DB ? (buf ^ 1) : 0);
                __syncthreads();
            }
            mfma_chunk(DB ? ((n_chunks - 1) & 1) : 0);

            const int cj = J0 + cb * 16 + lr;
            if constexpr (FORCE) {
                // f_j += sum_p grad phi_pj M_pj: this wave's rows, then the lanes of one column
                gp<const T> gph = gptr(static_cast<const T*>(sg.gphi) + 4 * u.out_offset);  // x, y, z, lap
                double f[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int pblk = RS * q + rh;
                    if (pblk < P) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int p = pblk * 16 + M::row(lk, r);
                            const int64_t e = (int64_t)min(p, np - 1) * ld + cj;
                            const double a = p < np && cj < m ? (double)acc[q][r] : 0.0;
#pragma unroll
                            for (int k = 0; k < 3; ++k) f[k] += a * (double)gph[4 * e + k];
                        }
                    }
                }
                double(*fred)[RS][TILE] = reinterpret_cast<double(*)[RS][TILE]>(&red[0][0][0]);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    double v = f[k];
                    v += __shfl_xor(v, 16);
                    v += __shfl_xor(v, 32);
                    if (lk == 0) fred[k][rh][cb * 16 + lr] = v;
                }
                return;
            }
            // n_p += sum_j T[p][j] Phi[p][j]
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int pblk = RS * q + rh;
                if (pblk < P) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int p = pblk * 16 + M::row(lk, r);
                        const int64_t e = (int64_t)min(p, np - 1) * ld + cj;
                        const bool live = p < np && cj < m;
#pragma unroll
                        for (int qq = 0; qq < NQ; ++qq) {
                            const double f = qq == 0 ? (double)phi[e]
                                                     : (double)gptr(static_cast<const T*>(sg.gphi) + 3 * u.out_offset)[3 * e + qq - 1];
                            const double v = row_sum16(live ? (double)acc[q][r] * f : 0.0);
                            if (lr == 0) red[qq][cb][p] = v;
                        }
                    }
                }
            }
        };
        // R is the smallest of RB, 3 RB / 4, RB / 2, RB / 4, 0 that covers this wave's blocks
        typedef std::integral_constant<int, RB> Full;
        typedef std::integral_constant<int, RB / 2> Half;
        const int own = min(RB, (P - rh + RS - 1) / RS);  // wave-uniform
        if (P > RB / 2 * RS) {  // rows beyond 128: every wave owns more than RB / 2 - 1 blocks
            if (own > RB * 3 / 4) run(Full{}, Full{});
            else if (own > RB / 2) run(Full{}, std::integral_constant<int, RB * 3 / 4>{});
            else run(Full{}, Half{});
        } else {
            if (own > RB / 4) run(Half{}, Half{});
            else if (own > 0) run(Half{}, std::integral_constant<int, RB / 4>{});
            else run(Half{}, std::integral_constant<int, 0>{});
        }
        __syncthreads();
        if constexpr (FORCE) {
            if (tid < 3 * TILE) {
                const int k = tid / TILE, col = tid % TILE;
                if (J0 + col < m) {
                    double(*fred)[RS][TILE] = reinterpret_cast<double(*)[RS][TILE]>(&red[0][0][0]);
                    double v = 0.0;
#pragma unroll
                    for (int h = 0; h < RS; ++h) v += fred[k][h][col];
                    gadd(gptr(sg.fb) + 3 * (int64_t)fn[J0 + col] + k, v);
                }
            }
        } else if (tid < np) {
            const int32_t pc = gptr(sg.sys->perm)[u.point_begin + tid];
            const double v = (red[0][0][tid] + red[0][1][tid]) + (red[0][2][tid] + red[0][3][tid]);
            gadd(gptr(sg.n) + pc, v);
            if (GRAD)  // grad n = 2 sum_j T_pj grad phi_pj
#pragma unroll
                for (int qq = 1; qq < NQ; ++qq)
                    gadd(gptr(sg.gn) + 3 * (int64_t)pc + qq - 1,
                         2.0 * ((red[qq][0][tid] + red[qq][1][tid]) + (red[qq][2][tid] + red[qq][3][tid])));
        }
        __syncthreads();  // red is rewritten by the next item
    }
}

// ------------------------------------------------------------------------------------------
// Reduced-precision contractions.  Basis values arrive as FP32 (rounded from the FP64
// evaluation); w*v and D are rounded from FP64 when staged.  Per-tile results are flushed
// into FP64 accumulators and reach H and n through FP64 atomics.






// Split of an FP32 value into NS bf16 parts: x ~ x0 + x1 (+ x2), each part the rounding to
// nearest of what the previous parts leave.
template <int NS>
__device__ inline void split_bf16(float x, __bf16* part)
{
    float r = x;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const __bf16 h = (__bf16)r;
        part[s] = h;
        r -= (float)h;
    }
}

// Products kept: parts (s, t) with s + t <= NS - 1 (3 terms for NS = 2, 6 terms for NS = 3).
template <int NS>
__device__ inline f4 mfma_split(const bf8* a, const bf8* b, f4 acc)
{
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int t = 0; t < NS; ++t)
            if (s + t <= NS - 1) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s], b[t], acc, 0, 0, 0);
    return acc;
}

constexpr int BK = 32;       // K per bf16 MFMA step
constexpr int BKP = BK + 8;  // padded LDS row (80 bytes: keeps 16-byte alignment)

// Hamiltonian, split-BF16 MFMA (v_mfma_f32_16x16x32_bf16): per item one 64x64 tile pair of a
// unit, K = 32 points per chunk, four waves of 32x32.  LDS holds [buffer][part][column][point]
// so that every lane reads its 8 consecutive points as one 16-byte vector; the next chunk's
// FP32 basis values and FP64 w v are prefetched into registers while the MFMAs of the current
// one run and are split into bf16 parts at the stash.  The FP32 tile sums move into FP64
// after every chunk; FP64 atomics into the upper triangle of H.  At least three waves per SIMD
// (the two-part form then fits three workgroups per CU: 9 % faster than two).
template <int NS>
__global__ __launch_bounds__(256, 3) void h_kernel_bf16(const DevSeg* __restrict__ segs, int n_segs, int64_t total)
{
    constexpr int NQ = BK * TILE / 256;  // values per thread per chunk and operand
    __shared__ __attribute__((aligned(16))) __bf16 As[2][NS][TILE][BKP];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][NS][TILE][BKP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    for (int64_t v_ = blockIdx.x; v_ < xcd_span(total); v_ += gridDim.x) {
        const int64_t b = xcd_item(v_, total);
        if (b >= total) continue;
        const int s = find_segment(segs, n_segs, b, [](const DevSeg& g) { return g.item_prefix; });
        const DevSeg& sg = segs[s];
        const HItem it = static_cast<const HItem*>(sg.items)[sg.item_begin + (b - sg.item_prefix)];
        const DevUnit u = sg.units[it.unit];
        gp<const float> __restrict__ phi = gptr(static_cast<const float*>(sg.phi) + u.out_offset);
        gp<const double> __restrict__ wv = gptr(sg.wv + u.point_begin);
        const int np = u.n_points, ld = u.ld;
        if (np <= 0) continue;
        const int I0 = it.ti * TILE, J0 = it.tj * TILE;
        const int n_chunks = (np + BK - 1) / BK;

        // this thread's column of both operands and its NQ = 8 consecutive points of a chunk, so
        // that every part is stashed as one 16-byte run of a column (loads: a wave reads 64
        // consecutive columns of one point)
        static_assert(NQ == 8, "eight points per thread");
        const int col = tid & 63, p0 = NQ * (tid >> 6);
        float ra[NQ], rb[NQ];
        double rw[NQ];
        auto fetch = [&](int c) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int pc = min(c * BK + p0 + q, np - 1);
                gp<const float> rowp = phi + (int64_t)pc * ld;
                ra[q] = rowp[I0 + col];
                rb[q] = rowp[J0 + col];
                rw[q] = wv[pc];
            }
        };
        auto stash = [&](int c, int buf) {
            bf8 pa[NS], pb[NS];
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const bool ok = c * BK + p0 + q < np;
                __bf16 xa[NS], xb[NS];
                split_bf16<NS>(ok ? (float)((double)ra[q] * rw[q]) : 0.f, xa);
                split_bf16<NS>(ok ? rb[q] : 0.f, xb);
#pragma unroll
                for (int t = 0; t < NS; ++t) {
                    pa[t][q] = xa[t];
                    pb[t][q] = xb[t];
                }
            }
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                *reinterpret_cast<bf8*>(&As[buf][t][col][p0]) = pa[t];
                *reinterpret_cast<bf8*>(&Bs[buf][t][col][p0]) = pb[t];
            }
        };
        gp<const int32_t> __restrict__ fn = gptr(sg.unit_fn + u.fn_begin);
        int32_t gI[2][4], gJ[2];
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
#pragma unroll
            for (int r = 0; r < 4; ++r) gI[ib][r] = fn[min(I0 + wr * 32 + ib * 16 + lk * 4 + r, u.m - 1)];
            gJ[ib] = fn[min(J0 + wc * 32 + ib * 16 + lr, u.m - 1)];
        }

        f4 acc[2][2];
        d4 acc64[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
                acc64[i][j] = d4{0.0, 0.0, 0.0, 0.0};
            }
        auto k_loop = [&](auto with_mfma) {
            fetch(0);
            stash(0, 0);
            __syncthreads();
            for (int c = 0; c < n_chunks; ++c) {
                const int buf = c & 1;
                if (c + 1 < n_chunks) fetch(c + 1);
                if (decltype(with_mfma)::value) {
                    bf8 a0[NS], a1[NS], b0[NS], b1[NS];
#pragma unroll
                    for (int t = 0; t < NS; ++t) {
                        a0[t] = *reinterpret_cast<const bf8*>(&As[buf][t][wr * 32 + lr][lk * 8]);
                        a1[t] = *reinterpret_cast<const bf8*>(&As[buf][t][wr * 32 + 16 + lr][lk * 8]);
                        b0[t] = *reinterpret_cast<const bf8*>(&Bs[buf][t][wc * 32 + lr][lk * 8]);
                        b1[t] = *reinterpret_cast<const bf8*>(&Bs[buf][t][wc * 32 + 16 + lr][lk * 8]);
                    }
                    acc[0][0] = mfma_split<NS>(a0, b0, acc[0][0]);
                    acc[0][1] = mfma_split<NS>(a0, b1, acc[0][1]);
                    acc[1][0] = mfma_split<NS>(a1, b0, acc[1][0]);
                    acc[1][1] = mfma_split<NS>(a1, b1, acc[1][1]);
                    // every chunk of 32 points: move the FP32 sums into FP64
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                acc64[i][j][r] += (double)acc[i][j][r];
                                acc[i][j][r] = 0.f;
                            }
                }
                if (c + 1 < n_chunks) stash(c + 1, buf ^ 1);
                __syncthreads();
            }
        };
        const bool diag = it.ti == it.tj;
        if (diag && wr > wc) {  // the strictly lower quarter of a diagonal tile pair only stages data
            k_loop(std::false_type{});
            continue;
        }
        k_loop(std::true_type{});
        gp<double> __restrict__ H = gptr(sg.H);
        const int64_t ldh = sg.ld;
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wr * 32 + ib * 16 + lk * 4 + r, col = wc * 32 + jb * 16 + lr;
                    const int ci = I0 + row, cj = J0 + col;
                    if (ci < u.m && cj < u.m && (!diag || row <= col))
                        gadd(H + (int64_t)gI[ib][r] * ldh + gJ[jb], acc64[ib][jb][r]);
                }
    }
}

// Density, split-BF16 MFMA: per item one 64-wide column tile J of a unit, K = 32 functions per
// chunk; sixteen waves as in n_kernel (wave w: column block w % 4, row blocks w / 4 + 4 q).  A
// (points x functions) in LDS as [part][point][function], B (functions x columns) as
// [part][column][function]; NB LDS buffers (one buffer adds a barrier per chunk).  The FP32
// sums move into FP64 after every 64-function tile; the row dot and the sums over tiles and
// units are FP64.
template <int NS, int NB>
__global__ __launch_bounds__(1024) void n_kernel_bf16(const DevSeg* __restrict__ segs, int n_segs, int64_t total)
{
    constexpr int NT = 1024, RB = 4, RS = 4;
    constexpr int NA = MAX_UNIT_POINTS * BK / NT;  // basis values per thread per chunk (8)
    constexpr int ND = BK * TILE / NT;             // D values per thread per chunk (2)
    constexpr int CPT = TILE / BK;                 // chunks per tile (2)
    __shared__ __attribute__((aligned(16))) __bf16 As[NB][NS][MAX_UNIT_POINTS][BKP];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[NB][NS][TILE][BKP];
    __shared__ double red[4][MAX_UNIT_POINTS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cb = wave & 3, rh = wave >> 2;
    const int lr = lane & 15, lk = lane >> 4;
    for (int64_t v_ = blockIdx.x; v_ < xcd_span(total); v_ += gridDim.x) {
        const int64_t b = xcd_item(v_, total);
        if (b >= total) continue;
        const int s = find_segment(segs, n_segs, b, [](const DevSeg& g) { return g.item_prefix; });
        const DevSeg& sg = segs[s];
        const NItem it = static_cast<const NItem*>(sg.items)[sg.item_begin + (b - sg.item_prefix)];
        const DevUnit u = sg.units[it.unit];
        gp<const float> __restrict__ phi = gptr(static_cast<const float*>(sg.phi) + u.out_offset);
        gp<const int32_t> __restrict__ fn = gptr(sg.unit_fn + u.fn_begin);
        gp<const double> __restrict__ D = gptr(sg.D);
        const int64_t ldd = sg.ld;
        const int np = u.n_points, ld = u.ld, m = u.m;
        if (np <= 0 || m <= 0) continue;
        const int P = (np + 15) >> 4;
        const int J0 = it.tj * TILE;
        const int n_chunks = (it.tj + 1) * CPT;  // chunk c covers functions 32 c .. 32 c + 31
        const int cjd = J0 + (tid & (TILE - 1));
        const int64_t gjd = fn[min(cjd, m - 1)];

        auto run = [&](auto rows_staged, auto rows_own) {
            constexpr int F = decltype(rows_staged)::value;
            constexpr int R = decltype(rows_own)::value;
            constexpr int NAR = NA * F / RB;
            float pa[NAR];
            double pd[ND];
            int32_t gcur[ND], gnxt[ND];
            auto load_idx = [&](int c, int32_t* g) {
#pragma unroll
                for (int q = 0; q < ND; ++q) g[q] = fn[min(BK * c + (tid >> 6) + (NT / TILE) * q, m - 1)];
            };
            auto fetch = [&](int c) {
#pragma unroll
                for (int q = 0; q < NAR; ++q) {
                    const int e = tid + NT * q;
                    pa[q] = phi[(int64_t)min(e / BK, np - 1) * ld + BK * c + (e % BK)];
                }
                const bool diag = c / CPT == it.tj;
#pragma unroll
                for (int q = 0; q < ND; ++q) {
                    const int ci = BK * c + (tid >> 6) + (NT / TILE) * q;
                    const bool lower = diag && ci > cjd;
                    pd[q] = D[lower ? gjd * ldd + gcur[q] : (int64_t)gcur[q] * ldd + gjd];
                }
                load_idx(c + 1, gnxt);
            };
            auto stash = [&](int c, int buf) {
#pragma unroll
                for (int q = 0; q < ND; ++q) gcur[q] = gnxt[q];
                const bool diag = c / CPT == it.tj;
#pragma unroll
                for (int q = 0; q < NAR; ++q) {
                    const int e = tid + NT * q;
                    __bf16 px[NS];
                    split_bf16<NS>((e / BK) < np ? pa[q] : 0.f, px);
#pragma unroll
                    for (int t = 0; t < NS; ++t) As[buf][t][e / BK][e % BK] = px[t];
                }
#pragma unroll
                for (int q = 0; q < ND; ++q) {
                    const int e = tid + NT * q;
                    const int i = e >> 6, j = e & 63;
                    const bool ok = BK * c + i < m && cjd < m;
                    __bf16 pv[NS];
                    split_bf16<NS>(ok ? (float)(diag ? pd[q] : 2.0 * pd[q]) : 0.f, pv);
#pragma unroll
                    for (int t = 0; t < NS; ++t) Bs[buf][t][j][i] = pv[t];
                }
            };

            f4 acc[R > 0 ? R : 1];
            d4 acc64[R > 0 ? R : 1];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                acc[i] = f4{0.f, 0.f, 0.f, 0.f};
                acc64[i] = d4{0.0, 0.0, 0.0, 0.0};
            }
            load_idx(0, gcur);
            fetch(0);
            stash(0, 0);
            __syncthreads();
            for (int c = 0; c < n_chunks; ++c) {
                const int buf = NB == 2 ? (c & 1) : 0;
                if (c + 1 < n_chunks) fetch(c + 1);
                if (R > 0) {
                    bf8 bv[NS];
#pragma unroll
                    for (int t = 0; t < NS; ++t) bv[t] = *reinterpret_cast<const bf8*>(&Bs[buf][t][cb * 16 + lr][lk * 8]);
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        bf8 av[NS];
#pragma unroll
                        for (int t = 0; t < NS; ++t)
                            av[t] = *reinterpret_cast<const bf8*>(&As[buf][t][(RS * q + rh) * 16 + lr][lk * 8]);
                        acc[q] = mfma_split<NS>(av, bv, acc[q]);
                    }
                    if (c % CPT == CPT - 1) {  // end of a 64-function tile
#pragma unroll
                        for (int q = 0; q < R; ++q)
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                acc64[q][r] += (double)acc[q][r];
                                acc[q][r] = 0.f;
                            }
                    }
                }
                if (NB == 1) __syncthreads();
                if (c + 1 < n_chunks) stash(c + 1, NB == 2 ? (buf ^ 1) : 0);
                __syncthreads();
            }
            const int cj = J0 + cb * 16 + lr;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int pblk = RS * q + rh;
                if (pblk < P) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int p = pblk * 16 + lk * 4 + r;
                        const double f = (double)phi[(int64_t)min(p, np - 1) * ld + cj];
                        const double v = row_sum16((p < np && cj < m) ? acc64[q][r] * f : 0.0);
                        if (lr == 0) red[cb][p] = v;
                    }
                }
            }
        };
        typedef std::integral_constant<int, RB> Full;
        typedef std::integral_constant<int, RB / 2> Half;
        const int own = min(RB, (P - rh + RS - 1) / RS);
        if (P > RB / 2 * RS) {
            if (own > RB * 3 / 4) run(Full{}, Full{});
            else if (own > RB / 2) run(Full{}, std::integral_constant<int, RB * 3 / 4>{});
            else run(Full{}, Half{});
        } else {
            if (own > RB / 4) run(Half{}, Half{});
            else if (own > 0) run(Half{}, std::integral_constant<int, RB / 4>{});
            else run(Half{}, std::integral_constant<int, 0>{});
        }
        __syncthreads();
        if (tid < np) {
            const double v = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
            gadd(gptr(sg.n) + gptr(sg.sys->perm)[u.point_begin + tid], v);
        }
        __syncthreads();  // red is rewritten by the next item
    }
}

hipError_t launch_h(Mode mode, const DevSeg* segs_dev, int n_segs, int64_t n_items, hipStream_t st,
                    int64_t max_grid, int h_tile)
{
    if (h_tile == WTILE && (mode == MODE_FP64 || mode == MODE_FP32)) {
        if (n_items <= 0 || n_segs <= 0) return hipSuccess;
        if (n_items > 0x7ffffff0) return hipErrorInvalidValue;
        const dim3 g(grid_for(n_items, max_grid)), b(512);
        if (mode == MODE_FP64) hipLaunchKernelGGL(h_kernel_wide<double>, g, b, 0, st, segs_dev, n_segs, n_items);
        else hipLaunchKernelGGL(h_kernel_wide<float>, g, b, 0, st, segs_dev, n_segs, n_items);
        return hipGetLastError();
    }
    if (h_tile != TILE) return hipErrorInvalidValue;
    if (n_items <= 0 || n_segs <= 0) return hipSuccess;
    if (n_items > 0x7ffffff0) return hipErrorInvalidValue;
    const dim3 g(grid_for(n_items, max_grid)), b(256);
    switch (mode) {
    case MODE_FP64: hipLaunchKernelGGL((h_kernel_dma<double, 16, 3>), g, b, 0, st, segs_dev, n_segs, n_items); break;
    case MODE_FP32: hipLaunchKernelGGL(h_kernel<float>, g, b, 0, st, segs_dev, n_segs, n_items); break;
    case MODE_BF16X3: hipLaunchKernelGGL(h_kernel_bf16<2>, g, b, 0, st, segs_dev, n_segs, n_items); break;
    case MODE_BF16X6: hipLaunchKernelGGL(h_kernel_bf16<3>, g, b, 0, st, segs_dev, n_segs, n_items); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_n(Mode mode, const DevSeg* segs_dev, int n_segs, int64_t n_items, hipStream_t st,
                    int64_t max_grid)
{
    if (n_items <= 0 || n_segs <= 0) return hipSuccess;
    if (n_items > 0x7ffffff0) return hipErrorInvalidValue;
    const dim3 g(grid_for(n_items, max_grid)), b(1024);
    switch (mode) {
    case MODE_FP64: hipLaunchKernelGGL((n_kernel<double, 16, 16, true>), g, b, 0, st, segs_dev, n_segs, n_items); break;
    case MODE_FP32: hipLaunchKernelGGL((n_kernel<float, 16, 16, true>), g, b, 0, st, segs_dev, n_segs, n_items); break;
    case MODE_BF16X3: hipLaunchKernelGGL((n_kernel_bf16<2, 2>), g, b, 0, st, segs_dev, n_segs, n_items); break;
    case MODE_BF16X6: hipLaunchKernelGGL((n_kernel_bf16<3, 1>), g, b, 0, st, segs_dev, n_segs, n_items); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_n_grad(Mode mode, const DevSeg* segs_dev, int n_segs, int64_t n_items, hipStream_t st)
{
    if (n_items <= 0 || n_segs <= 0) return hipSuccess;
    if (n_items > 0x7ffffff0) return hipErrorInvalidValue;
    const dim3 g(grid_for(n_items, 0)), b(1024);
    switch (mode) {
    case MODE_FP64: hipLaunchKernelGGL((n_kernel<double, 16, 16, true, NK_GRADIENT>), g, b, 0, st, segs_dev, n_segs, n_items); break;
    case MODE_FP32: hipLaunchKernelGGL((n_kernel<float, 16, 16, true, NK_GRADIENT>), g, b, 0, st, segs_dev, n_segs, n_items); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_n_force(Mode mode, const DevSeg* segs_dev, int n_segs, int64_t n_items, hipStream_t st)
{
    if (n_items <= 0 || n_segs <= 0) return hipSuccess;
    if (n_items > 0x7ffffff0) return hipErrorInvalidValue;
    const dim3 g(grid_for(n_items, 0)), b(1024);
    switch (mode) {
    case MODE_FP64: hipLaunchKernelGGL((n_kernel<double, 16, 16, true, NK_FORCE>), g, b, 0, st, segs_dev, n_segs, n_items); break;
    case MODE_FP32: hipLaunchKernelGGL((n_kernel<float, 16, 16, true, NK_FORCE>), g, b, 0, st, segs_dev, n_segs, n_items); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_h_gga(Mode mode, const DevSeg* segs_dev, int n_segs, int64_t n_items, hipStream_t st)
{
    if (n_items <= 0 || n_segs <= 0) return hipSuccess;
    if (n_items > 0x7ffffff0) return hipErrorInvalidValue;
    const dim3 g(grid_for(n_items, 0)), b(256);
    switch (mode) {
    case MODE_FP64: hipLaunchKernelGGL(h_kernel_gga<double>, g, b, 0, st, segs_dev, n_segs, n_items); break;
    case MODE_FP32: hipLaunchKernelGGL(h_kernel_gga<float>, g, b, 0, st, segs_dev, n_segs, n_items); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// small kernels

__global__ void fill_kernel(double* __restrict__ p, int64_t n, double value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void force_atoms_kernel(const double* __restrict__ fb, const int64_t* __restrict__ atom_first,
                                   int64_t n_atoms, double* __restrict__ F)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 3 * n_atoms) return;
    const int64_t a = i / 3, k = i - 3 * a;
    double v = 0.0;
    for (int64_t j = atom_first[a]; j < atom_first[a + 1]; ++j) v += fb[3 * j + k];
    F[i] = 2.0 * v;
}

hipError_t launch_force_atoms(const double* fb, const int64_t* atom_first, int64_t n_atoms, double* F,
                              hipStream_t st)
{
    if (n_atoms <= 0) return hipSuccess;
    const int64_t blocks = (3 * n_atoms + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(force_atoms_kernel, dim3((unsigned)blocks), dim3(256), 0, st, fb, atom_first, n_atoms, F);
    return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double value, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n, value);
    return hipGetLastError();
}

__global__ void wv_kernel(const double* __restrict__ pw, const int32_t* __restrict__ perm,
                          const double* __restrict__ v, double* __restrict__ wv, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        wv[i] = pw[i] * v[perm[i]];
}

hipError_t launch_wv(const double* pw, const int32_t* perm, const double* v_caller, double* wv,
                     int64_t n_points, hipStream_t st)
{
    if (n_points <= 0) return hipSuccess;
    int64_t blocks = (n_points + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(wv_kernel, dim3((unsigned)blocks), dim3(256), 0, st, pw, perm, v_caller, wv, n_points);
    return hipGetLastError();
}

__global__ void wa_kernel(const double* __restrict__ pw, const int32_t* __restrict__ perm,
                          const double* __restrict__ a, double* __restrict__ wa, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = i / 3;
        wa[i] = pw[p] * a[3 * (int64_t)perm[p] + (i - 3 * p)];
    }
}

hipError_t launch_wa(const double* pw, const int32_t* perm, const double* a_caller, double* wa, int64_t n_points,
                     hipStream_t st)
{
    if (n_points <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((3 * n_points + 255) / 256, 65536);
    hipLaunchKernelGGL(wa_kernel, dim3((unsigned)blocks), dim3(256), 0, st, pw, perm, a_caller, wa, n_points);
    return hipGetLastError();
}

// H[j][i] = H[i][j] for i < j, through 32x32 LDS tiles (coalesced on both sides).
__global__ __launch_bounds__(256) void mirror_kernel(double* __restrict__ H, int64_t n)
{
    __shared__ double t[32][33];
    const int64_t bi = blockIdx.y, bj = blockIdx.x;
    if (bi > bj) return;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bi * 32 + r, j = bj * 32 + tx;
        t[r][tx] = (i < n && j < n) ? H[i * n + j] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bj * 32 + r, j = bi * 32 + tx;  // lower-triangle target (i > j)
        if (i < n && j < n && i > j) H[i * n + j] = t[tx][r];
    }
}

hipError_t launch_mirror(double* H, int64_t n, hipStream_t st)
{
    if (n <= 1) return hipSuccess;
    const int64_t nt = (n + 31) / 32;
    if (nt > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mirror_kernel, dim3((unsigned)nt, (unsigned)nt), dim3(256), 0, st, H, n);
    return hipGetLastError();
}

// N_e = sum_p w_p n_p: per-block partial sums, then one block adds them in a fixed order.
__global__ __launch_bounds__(256) void wsum_partial_kernel(const double* __restrict__ pw, const int32_t* __restrict__ perm,
                                                           const double* __restrict__ n, int64_t np,
                                                           double* __restrict__ partial)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x)
        acc += pw[i] * n[perm[i]];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void wsum_final_kernel(const double* __restrict__ partial, int nb, double* out)
{
    __shared__ double s[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += partial[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

hipError_t launch_weighted_sum(const double* pw, const int32_t* perm, const double* n_caller,
                               int64_t n_points, double* partial, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(wsum_partial_kernel, dim3(WSUM_BLOCKS), dim3(256), 0, st, pw, perm, n_caller, n_points,
                       partial);
    hipLaunchKernelGGL(wsum_final_kernel, dim3(1), dim3(256), 0, st, partial, WSUM_BLOCKS, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Scratch of the allocation-free Hamiltonian call.  Every GPU that loads this code object holds
// its own copy of the array until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: the device address is looked up once per device and kept in
// g_noalloc_ptr, and only that address is ever handed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current first
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_noalloc_ptr[device] = ptr;
    return hipSuccess;
}

void* noalloc_scratch(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    return g_noalloc_ptr[device];
}

}  // namespace nao

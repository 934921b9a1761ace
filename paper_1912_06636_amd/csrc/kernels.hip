// HIP kernels for gfx950 (CDNA4): basis evaluation, the two batch contractions on FP64
// MFMA, and the small elementwise / reduction / mirror kernels around them.
//
// Data layout (device memory):
//   - points, weights and w*v in batch order (structure of arrays, FP64);
//   - basis values of an execution unit: [n_points][ld] FP64, point-major, ld a multiple of
//     the 64-wide basis tile, padding columns zero;
//   - D and H dense row-major [N_b][N_b] FP64; n in the caller's point order.
#include <hip/hip_runtime.h>

#include "devtypes.h"

namespace nao {

typedef double d4 __attribute__((ext_vector_type(4)));

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

// (dx*dx + dy*dy) + dz*dz without contraction: the same arithmetic that decides relevance.
__device__ inline double dist2_exact(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    const double xx = dx * dx;
    const double yy = dy * dy;
    const double zz = dz * dz;
    return (xx + yy) + zz;
}

// Real orthonormal spherical harmonics (l <= 3) of a unit vector, m = -l..l; Y_11 ~ +x.
struct Ylm {
    double v[16];
};

__device__ inline void real_ylm(double x, double y, double z, int lmax, double* Y)
{
    const double c00 = 0.28209479177387814;   // 1 / (2 sqrt(pi))
    const double c1 = 0.48860251190291992;    // sqrt(3 / (4 pi))
    const double c2a = 1.0925484305920792;    // sqrt(15 / pi) / 2
    const double c2b = 0.31539156525252005;   // sqrt(5 / pi) / 4
    const double c2c = 0.54627421529603959;   // sqrt(15 / pi) / 4
    const double c3a = 0.59004358992664352;   // sqrt(35 / (2 pi)) / 4
    const double c3b = 2.8906114426405538;    // sqrt(105 / pi) / 2
    const double c3c = 0.45704579946446572;   // sqrt(21 / (2 pi)) / 4
    const double c3d = 0.37317633259011546;   // sqrt(7 / pi) / 4
    const double c3e = 1.4453057213202769;    // sqrt(105 / pi) / 4
    Y[0] = c00;
    if (lmax >= 1) {
        Y[1] = c1 * y;
        Y[2] = c1 * z;
        Y[3] = c1 * x;
    }
    if (lmax >= 2) {
        Y[4] = c2a * x * y;
        Y[5] = c2a * y * z;
        Y[6] = c2b * (3.0 * z * z - 1.0);
        Y[7] = c2a * x * z;
        Y[8] = c2c * (x * x - y * y);
    }
    if (lmax >= 3) {
        Y[9] = c3a * y * (3.0 * x * x - y * y);
        Y[10] = c3b * x * y * z;
        Y[11] = c3c * y * (5.0 * z * z - 1.0);
        Y[12] = c3d * (5.0 * z * z * z - 3.0 * z);
        Y[13] = c3c * x * (5.0 * z * z - 1.0);
        Y[14] = c3e * z * (x * x - y * y);
        Y[15] = c3a * x * (x * x - 3.0 * y * y);
    }
}

// ------------------------------------------------------------------------------------------
// basis evaluation: one workgroup per unit, threads over (point, atom) pairs (atom fastest)

template <bool SPLINE_LDS>
__global__ __launch_bounds__(256) void basis_kernel_f64(const DevSeg* __restrict__ segs, int n_segs)
{
    extern __shared__ double lds_spline[];
    const int64_t b = blockIdx.x;
    const int s = find_segment(segs, n_segs, b, [](const DevSeg& g) { return g.unit_prefix; });
    const DevSeg& sg = segs[s];
    const DevUnit u = sg.units[sg.unit_begin + (b - sg.unit_prefix)];
    const DevSys* S = sg.sys;
    const int nk = S->n_knots;
    const double* spl = S->spline;
    if (SPLINE_LDS) {
        const int nsp = S->n_radial * (nk - 1) * 4;
        for (int i = threadIdx.x; i < nsp; i += blockDim.x) lds_spline[i] = spl[i];
        __syncthreads();
    }
    double* __restrict__ out = sg.phi + u.out_offset;
    const int64_t npairs = (int64_t)u.n_points * u.n_atoms;
    const double tmax = (double)(nk - 1);
    for (int64_t q = threadIdx.x; q < npairs; q += blockDim.x) {
        const int pl = (int)(q / u.n_atoms);
        const int ai = (int)(q - (int64_t)pl * u.n_atoms);
        const int atom = sg.unit_atoms[u.atom_begin + ai];
        int col = sg.unit_cols[u.atom_begin + ai];
        const int64_t p = u.point_begin + pl;
        const double* A = S->atom_xyzr + 4 * (int64_t)atom;
        const double dx = S->px[p] - A[0];
        const double dy = S->py[p] - A[1];
        const double dz = S->pz[p] - A[2];
        const double d2 = dist2_exact(dx, dy, dz);
        const int sp = S->atom_species[atom];
        const int sh0 = S->species_shell_ptr[sp], sh1 = S->species_shell_ptr[sp + 1];
        double* row = out + (int64_t)pl * u.ld;
        if (d2 >= A[3]) {
            for (int j = sh0; j < sh1; ++j) {
                const int nf = 2 * S->shell_l[j] + 1;
                for (int f = 0; f < nf; ++f) row[col + f] = 0.0;
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
        int lmax = 0;
        for (int j = sh0; j < sh1; ++j) lmax = max(lmax, S->shell_l[j]);
        double Y[16];
        real_ylm(ux, uy, uz, lmax, Y);
        const double lnr = r > 0.0 ? log(r) : 0.0;
        for (int j = sh0; j < sh1; ++j) {
            const int l = S->shell_l[j];
            const int rr = S->shell_radial[j];
            const double* par = S->radial_par + 4 * rr;
            double R = 0.0;
            if (d2 < par[1]) {
                double t = r > par[0] ? (lnr - par[3]) * par[2] : 0.0;
                t = fmin(fmax(t, 0.0), tmax);
                const int k = min((int)t, nk - 2);
                const double w = t - (double)k;
                const double* c = (SPLINE_LDS ? lds_spline : spl) + ((int64_t)rr * (nk - 1) + k) * 4;
                R = c[0] + w * (c[1] + w * (c[2] + w * c[3]));
            }
            switch (l) {
            case 0:
                row[col] = R * Y[0];
                col += 1;
                break;
            case 1:
                row[col] = R * Y[1];
                row[col + 1] = R * Y[2];
                row[col + 2] = R * Y[3];
                col += 3;
                break;
            case 2:
#pragma unroll
                for (int f = 0; f < 5; ++f) row[col + f] = R * Y[4 + f];
                col += 5;
                break;
            default:
#pragma unroll
                for (int f = 0; f < 7; ++f) row[col + f] = R * Y[9 + f];
                col += 7;
                break;
            }
        }
    }
    const int pad = u.ld - u.m;
    if (pad > 0) {
        const int64_t np = (int64_t)u.n_points * pad;
        for (int64_t q = threadIdx.x; q < np; q += blockDim.x) {
            const int64_t pl = q / pad;
            out[pl * u.ld + u.m + (q - pl * pad)] = 0.0;
        }
    }
}

hipError_t launch_basis_f64(const DevSeg* segs_dev, int n_segs, int64_t n_units, bool spline_in_lds,
                            hipStream_t st)
{
    if (n_units <= 0 || n_segs <= 0) return hipSuccess;
    if (n_units > 0x7fffffff) return hipErrorInvalidValue;
    if (spline_in_lds)
        hipLaunchKernelGGL(basis_kernel_f64<true>, dim3((unsigned)n_units), dim3(256),
                           MAX_SPLINE_LDS * sizeof(double), st, segs_dev, n_segs);
    else
        hipLaunchKernelGGL(basis_kernel_f64<false>, dim3((unsigned)n_units), dim3(256), 0, st, segs_dev,
                           n_segs);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Hamiltonian: per work item one 64x64 tile pair (I <= J) of a unit,
//   H[I, J] += (w v Phi[:, I])^T Phi[:, J],
// K loop over the unit's points in chunks of 16 staged in LDS; four waves, each a 32x32
// quarter as 2x2 blocks of v_mfma_f64_16x16x4; FP64 atomics into the upper triangle.

__global__ __launch_bounds__(256) void h_kernel_f64(const DevSeg* __restrict__ segs, int n_segs)
{
    __shared__ double As[KCHUNK][TILE + 2];
    __shared__ double Bs[KCHUNK][TILE + 2];
    const int64_t b = blockIdx.x;
    const int s = find_segment(segs, n_segs, b, [](const DevSeg& g) { return g.item_prefix; });
    const DevSeg& sg = segs[s];
    const HItem it = static_cast<const HItem*>(sg.items)[sg.item_begin + (b - sg.item_prefix)];
    const DevUnit u = sg.units[it.unit];
    const double* __restrict__ phi = sg.phi + u.out_offset;
    const double* __restrict__ wv = sg.wv + u.point_begin;
    const int np = u.n_points, ld = u.ld;
    const int I0 = it.ti * TILE, J0 = it.tj * TILE;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;

    d4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    for (int k0 = 0; k0 < np; k0 += KCHUNK) {
#pragma unroll
        for (int e = tid; e < KCHUNK * TILE; e += 256) {
            const int r = e >> 6, c = e & 63;
            const int p = k0 + r;
            double a = 0.0, bb = 0.0;
            if (p < np) {
                const double* rowp = phi + (int64_t)p * ld;
                a = rowp[I0 + c] * wv[p];
                bb = rowp[J0 + c];
            }
            As[r][c] = a;
            Bs[r][c] = bb;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < KCHUNK / 4; ++kk) {
            const int kr = kk * 4 + lk;
            const double a0 = As[kr][wr * 32 + lr];
            const double a1 = As[kr][wr * 32 + 16 + lr];
            const double b0 = Bs[kr][wc * 32 + lr];
            const double b1 = Bs[kr][wc * 32 + 16 + lr];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }

    const int32_t* __restrict__ fn = sg.unit_fn + u.fn_begin;
    double* __restrict__ H = sg.H;
    const int64_t ldh = sg.ld;
    const bool diag = it.ti == it.tj;
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wr * 32 + ib * 16 + lk * 4 + r;
                const int col = wc * 32 + jb * 16 + lr;
                const int ci = I0 + row, cj = J0 + col;
                if (ci < u.m && cj < u.m && (!diag || row <= col)) {
                    const int64_t gi = fn[ci], gj = fn[cj];
                    unsafeAtomicAdd(H + gi * ldh + gj, acc[ib][jb][r]);
                }
            }
}

hipError_t launch_h_f64(const DevSeg* segs_dev, int n_segs, int64_t n_items, hipStream_t st)
{
    if (n_items <= 0 || n_segs <= 0) return hipSuccess;
    if (n_items > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(h_kernel_f64, dim3((unsigned)n_items), dim3(256), 0, st, segs_dev, n_segs);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Density: per work item one 64-wide column tile J of a unit,
//   T[:, J] = sum_{I <= J} c_IJ Phi[:, I] D[I, J]   (c = 2 off the diagonal tile, 1 on it,
//             the diagonal tile read from the upper triangle of D),
//   n_p += sum_{j in J} T[p, j] Phi[p, j].
// Rows = the unit's points (<= 256, 16 row blocks), K = basis functions in chunks of 16;
// wave w owns column block w (16 columns) for all row blocks.

__global__ __launch_bounds__(256) void n_kernel_f64(const DevSeg* __restrict__ segs, int n_segs)
{
    __shared__ double As[MAX_UNIT_POINTS][KCHUNK + 1];
    __shared__ double Bs[KCHUNK][TILE + 2];
    __shared__ double red[4][MAX_UNIT_POINTS];
    const int64_t b = blockIdx.x;
    const int s = find_segment(segs, n_segs, b, [](const DevSeg& g) { return g.item_prefix; });
    const DevSeg& sg = segs[s];
    const NItem it = static_cast<const NItem*>(sg.items)[sg.item_begin + (b - sg.item_prefix)];
    const DevUnit u = sg.units[it.unit];
    const double* __restrict__ phi = sg.phi + u.out_offset;
    const int32_t* __restrict__ fn = sg.unit_fn + u.fn_begin;
    const double* __restrict__ D = sg.D;
    const int64_t ldd = sg.ld;
    const int np = u.n_points, ld = u.ld, m = u.m;
    const int P = (np + 15) >> 4;
    const int J0 = it.tj * TILE;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;

    d4 acc[MAX_UNIT_POINTS / 16];
#pragma unroll
    for (int i = 0; i < MAX_UNIT_POINTS / 16; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};

    for (int ti = 0; ti <= it.tj; ++ti) {
        const bool diag = ti == it.tj;
        for (int i0 = 0; i0 < TILE; i0 += KCHUNK) {
            const int c0 = ti * TILE + i0;
            for (int e = tid; e < MAX_UNIT_POINTS * KCHUNK; e += 256) {
                const int p = e >> 4, i = e & 15;
                As[p][i] = p < np ? phi[(int64_t)p * ld + c0 + i] : 0.0;
            }
#pragma unroll
            for (int e = tid; e < KCHUNK * TILE; e += 256) {
                const int i = e >> 6, j = e & 63;
                const int ci = c0 + i, cj = J0 + j;
                double val = 0.0;
                if (ci < m && cj < m) {
                    const int64_t gi = fn[ci], gj = fn[cj];
                    if (!diag) val = 2.0 * D[gi * ldd + gj];
                    else val = ci <= cj ? D[gi * ldd + gj] : D[gj * ldd + gi];
                }
                Bs[i][j] = val;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < KCHUNK / 4; ++kk) {
                const double bv = Bs[kk * 4 + lk][wave * 16 + lr];
#pragma unroll
                for (int pb = 0; pb < MAX_UNIT_POINTS / 16; ++pb)
                    if (pb < P) {
                        const double av = As[pb * 16 + lr][kk * 4 + lk];
                        acc[pb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[pb], 0, 0, 0);
                    }
            }
            __syncthreads();
        }
    }

    const int cj = J0 + wave * 16 + lr;
#pragma unroll
    for (int pb = 0; pb < MAX_UNIT_POINTS / 16; ++pb) {
        if (pb < P) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = pb * 16 + lk * 4 + r;
                double v = 0.0;
                if (p < np && cj < m) v = acc[pb][r] * phi[(int64_t)p * ld + cj];
                v += __shfl_xor(v, 1);
                v += __shfl_xor(v, 2);
                v += __shfl_xor(v, 4);
                v += __shfl_xor(v, 8);
                if (lr == 0) red[wave][p] = v;
            }
        }
    }
    __syncthreads();
    if (tid < np) {
        const double v = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
        const int64_t pc = sg.sys->perm[u.point_begin + tid];
        unsafeAtomicAdd(sg.n + pc, v);
    }
}

hipError_t launch_n_f64(const DevSeg* segs_dev, int n_segs, int64_t n_items, hipStream_t st)
{
    if (n_items <= 0 || n_segs <= 0) return hipSuccess;
    if (n_items > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(n_kernel_f64, dim3((unsigned)n_items), dim3(256), 0, st, segs_dev, n_segs);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// small kernels

__global__ void fill_kernel(double* __restrict__ p, int64_t n, double value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
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

}  // namespace nao

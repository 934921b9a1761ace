// Types shared by the host runtime (runtime.cpp) and the kernels (kernels.hip).
#pragma once

#include <cstdint>

#include <hip/hip_runtime_api.h>

namespace nao {

constexpr int TILE = 64;              // basis-function tile of the contraction kernels
constexpr int KCHUNK = 16;            // points (Hamiltonian) / functions (density) per LDS stage
constexpr int MAX_UNIT_POINTS = 256;  // largest execution group the contraction kernels take
constexpr int MAX_SPLINE_LDS = 8192;  // doubles of spline table staged in LDS (64 KiB)

// One structure's resident device state, as seen by the kernels.
struct DevSys {
    const double* px;                  // batch-ordered point coordinates [n_points]
    const double* py;
    const double* pz;
    const double* pw;                  // batch-ordered weights
    const int32_t* perm;               // batch order -> caller index
    const double* atom_xyzr;           // [n_atoms][4]: x, y, z, (largest cutoff)^2
    const int32_t* atom_species;       // [n_atoms]
    const int32_t* species_shell_ptr;  // [n_species+1]
    const int32_t* shell_l;            // [n_shells]
    const int32_t* shell_radial;       // [n_shells]
    const double* radial_par;          // [n_radial][4]: rmin, rcut^2, 1/Delta, ln(rmin)
    const double* spline;              // [n_radial][n_knots][2]: y_k, M_k / 6 (plan.h)
    const int32_t* species_fn_ptr;     // [n_species+1] into fn_code
    const int32_t* fn_code;            // per species function: (shell within species << 4) | lm
    int32_t n_species;
    int32_t n_shells;
    int32_t n_radial;
    int32_t n_knots;
    int64_t n_basis;
    int64_t n_points;
};

// A run of batch-ordered points evaluated against one list of atoms.
struct DevUnit {
    int64_t point_begin;  // into the system's batch-ordered points
    int64_t atom_begin;   // into unit_atoms / unit_cols
    int64_t fn_begin;     // into unit_fn (global basis index of every column)
    int64_t out_offset;   // element offset of this unit's [n_points][ld] block within its block
    int32_t n_points;
    int32_t n_atoms;
    int32_t m;            // columns in use
    int32_t ld;           // row stride of the basis block (>= m)
};

// Work item of the Hamiltonian kernel: one tile pair (ti <= tj) of one unit.
struct HItem {
    int32_t unit;  // index into the system's unit array
    int16_t ti;
    int16_t tj;
};

// Work item of the density kernel: one column tile of one unit.
struct NItem {
    int32_t unit;
    int32_t tj;
};

// One segment of a launch: a block of one system's units (and their work items) whose
// basis values live at phi.  A launch covers a list of segments; block b of a launch maps
// to the segment whose prefix range contains it.
struct DevSeg {
    const DevSys* sys;
    const DevUnit* units;
    const int32_t* unit_atoms;
    const int32_t* unit_cols;
    const int32_t* unit_fn;
    const void* items;       // HItem* or NItem*
    void* phi;               // basis values of this block (FP64, or FP32 for the reduced-precision
                             // modes); unit.out_offset is relative to it
    const double* wv;        // batch-ordered w*v (Hamiltonian)
    const double* D;         // density matrix (density), row-major, ld = n_basis
    double* H;               // Hamiltonian, row-major, ld = n_basis
    double* n;               // density, caller order
    void* gphi;              // gradients of the basis values of this block, 3 per value (x, y, z
                             // interleaved; density-gradient launches only)
    double* gn;              // density gradient [n_points][3], caller order
    const double* wa;        // batch-ordered w*a, 3 per point (Hamiltonian with a vector field)
    const double* Q;         // energy-weighted density matrix (forces), row-major, ld = n_basis
    double* fb;              // per-function force accumulator [n_basis][3] (forces)
    int64_t ld;              // n_basis
    int64_t unit_begin, unit_count, unit_prefix;
    int64_t item_begin, item_count, item_prefix;
};

// ------------------------------------------------------------------------------------------
// kernel launchers (kernels.hip).  Every launcher checks its own grid against the segment
// table before launching and returns hipErrorInvalidValue on a mismatch.

// Contraction arithmetic (nao_precision values).
enum Mode { MODE_FP64 = 0, MODE_FP32 = 1, MODE_BF16X3 = 2, MODE_BF16X6 = 3 };

// Basis values as FP64 (fp32_out = false) or rounded to FP32.
// max_grid > 0 caps the grid: workgroups then loop over the items (persistent launch).
// spline_lds: doubles of spline table to stage in LDS (0 = read it through the cache); it must
// cover the largest table of the systems in the segment list.
// extra: also write, to the segments' gphi, the gradient of every basis value (EXTRA_GRAD, 3 per
// value), L = (w v / 2) phi + (w a) . grad phi (EXTRA_GGA_L, 1 per value; needs wv and wa) or
// L = (w v / 2) phi - (w / 4) lap phi [+ (w a) . grad phi when wa is set] (EXTRA_KS_L, 1 per value),
// or the gradient and w h_KS phi = (w v) phi - (w / 2) lap phi (EXTRA_GRAD_H, 4 per value: x, y, z,
// w h_KS phi; needs wv).
enum BasisExtra { EXTRA_NONE = 0, EXTRA_GRAD = 1, EXTRA_GGA_L = 2, EXTRA_KS_L = 3, EXTRA_GRAD_H = 4 };
hipError_t launch_basis(const DevSeg* segs_dev, int n_segs, int64_t n_units, int spline_lds, bool fp32_out,
                        hipStream_t st, int64_t max_grid = 0, int extra = EXTRA_NONE);
// h_tile: 64, or 128 for the wide FP64/FP32 kernels (items then index 128-wide tiles).
hipError_t launch_h(Mode mode, const DevSeg* segs_dev, int n_segs, int64_t n_items, hipStream_t st,
                    int64_t max_grid = 0, int h_tile = TILE);
hipError_t launch_n(Mode mode, const DevSeg* segs_dev, int n_segs, int64_t n_items, hipStream_t st,
                    int64_t max_grid = 0);
// Density and its gradient (FP64 or FP32 modes): every item contracts over all of its unit's
// column tiles, and the row dots take the basis values and their gradients.
hipError_t launch_n_grad(Mode mode, const DevSeg* segs_dev, int n_segs, int64_t n_items, hipStream_t st);
// Hamiltonian with a vector field (FP64 or FP32 modes): H[I, J] += Phi_I^T L_J + L_I^T Phi_J over
// 64-wide tile pairs I <= J, L from the basis launch with EXTRA_GGA_L.
hipError_t launch_h_gga(Mode mode, const DevSeg* segs_dev, int n_segs, int64_t n_items, hipStream_t st);
// Local Pulay forces (FP64 or FP32 modes), density items walked over the whole list twice:
// fb[j] += sum_p grad phi_pj [((w v Phi - w lap Phi / 2) D)_pj - w_p (Phi Q)_pj]; gphi from the
// basis launch with EXTRA_GRAD_H, wv batch-ordered w*v.
hipError_t launch_n_force(Mode mode, const DevSeg* segs_dev, int n_segs, int64_t n_items, hipStream_t st);
// F[a] = 2 sum over the functions i of atom a (atom_first[a] <= i < atom_first[a + 1]) of fb[i].
hipError_t launch_force_atoms(const double* fb, const int64_t* atom_first, int64_t n_atoms, double* F,
                              hipStream_t st);
hipError_t launch_wa(const double* pw, const int32_t* perm, const double* a_caller, double* wa, int64_t n_points,
                     hipStream_t st);
hipError_t launch_fill(double* p, int64_t n, double value, hipStream_t st);
hipError_t launch_wv(const double* pw, const int32_t* perm, const double* v_caller, double* wv,
                     int64_t n_points, hipStream_t st);
hipError_t launch_mirror(double* H, int64_t n, hipStream_t st);
hipError_t launch_weighted_sum(const double* pw, const int32_t* perm, const double* n_caller,
                               int64_t n_points, double* partial, double* out, hipStream_t st);
constexpr int WSUM_BLOCKS = 1024;

// Fixed per-GPU scratch of the allocation-free Hamiltonian call (kernels.hip): a file-scope
// device array of NOALLOC_SCRATCH_BYTES that the library never allocates or frees.  Its head
// (NOALLOC_SEG_BYTES) holds the call's segment table, then w*v, then the basis values of one
// sub-block of execution groups at a time.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)256 << 20;
constexpr size_t NOALLOC_SEG_BYTES = (size_t)1 << 20;
// Look up the array's device address on `device`, which must be the current device; once per
// device (later calls return at once).  Called by nao_ctx_create.
hipError_t noalloc_scratch_init(int device);
// The address found by noalloc_scratch_init on `device`, or nullptr before it succeeded.
void* noalloc_scratch(int device);

}  // namespace nao

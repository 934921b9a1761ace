// Host-side planning: validated basis, octree batches, relevant-basis lists, execution
// groups and spline coefficients.  Pure C++ (no HIP); built with -ffp-contract=off so
// that the relevance test is evaluated exactly as specified.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "nao.h"

namespace nao {

struct HostBasis {
    int64_t n_atoms = 0;
    std::vector<double> atom_xyz;        // [n_atoms][3]
    std::vector<int32_t> atom_species;   // [n_atoms]
    int32_t n_species = 0;
    std::vector<int32_t> shell_ptr;      // [n_species+1]
    std::vector<int32_t> shell_l;        // [n_shells]
    std::vector<int32_t> shell_radial;   // [n_shells]
    int32_t n_radial = 0, n_knots = 0;
    std::vector<double> rmin, rcut;      // [n_radial]
    std::vector<double> samples;         // [n_radial][n_knots]
    // derived
    std::vector<int64_t> atom_first;     // [n_atoms+1] first global basis index
    std::vector<double> atom_rcut;       // [n_atoms] largest cutoff of the atom's radials
    std::vector<int32_t> species_nfn;    // [n_species] basis functions per atom of species
    int64_t n_basis = 0;
    int32_t max_l = 0;
};

// Returns "" on success, otherwise the reason the descriptor is invalid.
std::string load_basis(const nao_basis_desc* d, HostBasis& out);

// Octree batches (see nao.h): perm [n], batch_ptr [n_batches+1].
void octree_batches(const double* xyz, int64_t n, int32_t max_batch, std::vector<int64_t>& perm,
                    std::vector<int64_t>& batch_ptr);
// Grid-adapted cut-plane batches (see nao.h), same output form.
void cutplane_batches(const double* xyz, int64_t n, int32_t max_batch, std::vector<int64_t>& perm,
                      std::vector<int64_t>& batch_ptr);
// Batches by the method nao_batcher names (NAO_BATCH_OCTREE or NAO_BATCH_CUTPLANE).
void make_batches(int32_t batcher, const double* xyz, int64_t n, int32_t max_batch, std::vector<int64_t>& perm,
                  std::vector<int64_t>& batch_ptr);

// Relevant atoms of every batch (ascending), CSR.
void relevant_atoms(const HostBasis& b, const double* xyz, const std::vector<int64_t>& perm,
                    const std::vector<int64_t>& batch_ptr, std::vector<int64_t>& atom_ptr,
                    std::vector<int32_t>& atoms);

// Expands atom lists to basis-function lists.
void expand_lists(const HostBasis& b, const std::vector<int64_t>& atom_ptr,
                  const std::vector<int32_t>& atoms, std::vector<int64_t>& basis_ptr,
                  std::vector<int32_t>& basis_idx);

// Natural cubic spline in the unit-spaced coordinate t, stored per knot as (y_k, M_k / 6) with
// M the second derivative: layout [n_radial][n_knots][2].  On [k, k+1], u = t - k, v = 1 - u:
// R = v (y_k + (v^2 - 1) M_k / 6) + u (y_{k+1} + (u^2 - 1) M_{k+1} / 6).
std::vector<double> spline_knots(const HostBasis& b);

// An execution unit: a run of batch-ordered points with the union of their lists.
struct Unit {
    int64_t point_begin;  // into batch-ordered points
    int32_t n_points;
    int32_t n_atoms;      // relevant atoms
    int64_t atom_begin;   // into unit atom arrays
    int32_t m;            // basis functions (sum over atoms)
    int32_t batch;        // first source batch
};

// Packs consecutive batches (those with non-empty lists) into groups of at most group_max
// points; a batch larger than group_max is cut into pieces.  unit_atoms / unit_cols give
// each unit's atoms and the column where each atom's functions start.
void make_groups(const HostBasis& b, const std::vector<int64_t>& batch_ptr,
                 const std::vector<int64_t>& atom_ptr, const std::vector<int32_t>& atoms,
                 int32_t group_max, std::vector<Unit>& units, std::vector<int32_t>& unit_atoms,
                 std::vector<int32_t>& unit_cols);

// One unit per batch (used for basis output per batch).
void batch_units(const HostBasis& b, const std::vector<int64_t>& batch_ptr,
                 const std::vector<int64_t>& atom_ptr, const std::vector<int32_t>& atoms,
                 int64_t batch_begin, int64_t batch_end, std::vector<Unit>& units,
                 std::vector<int32_t>& unit_atoms, std::vector<int32_t>& unit_cols);

}  // namespace nao

// Host-side atom decomposition (Sec. 3.1): modified recursive bisection along
// inertia-tensor principal axes.
#pragma once

#include <cstdint>

namespace hartree {

// Fills order[natoms] (atom indices grouped by part, parts in tree order),
// part[natoms] (part of each atom; may be NULL) and part_start[nparts + 1]
// (offsets of the parts in `order`; may be NULL).  pos is natoms x 3 host
// doubles; weights is natoms positive host doubles or NULL for unit weights.
// Returns NULL on success, otherwise a description of the invalid argument
// (nothing is written then except possibly `order`).
const char *bisect_atoms(int32_t natoms, const double *pos, const double *weights, int32_t nparts, int32_t *order,
                         int32_t *part, int32_t *part_start);

}  // namespace hartree

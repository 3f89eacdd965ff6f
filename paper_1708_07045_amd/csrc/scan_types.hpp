// Plain-old-data records shared by the host runtime and the kernels.
#pragma once
#include <stdint.h>

namespace fftdg {

// One ligand configuration inside a chunk of work.
// Coordinates are "true" grid indices (may be negative for occupancy balls
// near the corner); the FFT sees them modulo n_fft.
struct CfgDev {
    int32_t u_base;      // first row of this configuration's placed atoms (lattice U table)
    int32_t atom_base;   // first row of its ligand's atom tables (gamma, thr)
    int32_t n_atoms;
    int32_t global_cfg;  // index of the configuration in the batch
    int32_t V[3];        // box-valid translations along x, y, z
    int32_t n_valid;     // V[0]*V[1]*V[2] (0 if the box does not fit)
    int32_t ze0, Le;     // energy channels: first plane (true z) and plane count
    int32_t ye0, Lye;    // energy channels: first row (true y) and row count
    int32_t zo0, Lo;     // occupancy channel: first plane and count
    int32_t yo0, Lyo;    // occupancy channel: first row and count
    int32_t pp_base;     // first plane-partial slot (one per valid z translation)
    int32_t scanned;     // 1 if the configuration is scanned in this call
    int32_t occ_slot0;   // forward-plane slot of the first occupancy plane
    int32_t xo0, Lxo;    // occupancy channel: first column (true x) and count
    // fused path (clash test on bits):
    int32_t run_off;     // first slot of its occupancy runs in the chunk's run buffer
    int32_t run_cap;     // slots reserved for them (an upper bound on the count)
    int32_t free_off;    // first word of its free-translation bits in the chunk
    int32_t item_base;   // first (tz, 64-row group) item of its clash test in the chunk
    int32_t surv_off;    // first slot of its list of undecided rows (Vz * Vy slots)
    int64_t off_fwd;     // complex-element offset of its forward planes
    int64_t off_inv;     // complex-element offset of its inverse planes
};

// Work items are not listed: a chunk carries, per configuration, the
// running count of its forward planes (fwd_off) and of its valid z
// translations (inv_off); a block finds its configuration by binary search.

template <typename T>
struct PlanePartial {
    T m, s, psi_min;
    int32_t n_finite, argmin;
};

// Per-ligand FP64 reduction output (device side).
struct LigRed {
    double dG, v_site, psi_min;
    int64_t n_finite, n_samples;
};

}  // namespace fftdg

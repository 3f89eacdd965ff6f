// Host/device view of the fused scan path: bit tables of the clash test and
// the launchers (one set per precision and FFT edge, N <= 128).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "scan_types.hpp"

namespace fftdg {

__host__ __device__ constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

// Longest run piece of the clash test (its two windows lie within one word
// of each other); runs of 2^k <= len < 2^(k+1) points read level k.
constexpr int RUN_MAX = 63;

// OR-dilated receptor occupancy rows of one snapshot, u32 words
// [k][Z][q][Y]: level k (window 2^k, k = 0 .. log2(RUN_MAX + 1) - 1, the
// levels runs of at most RUN_MAX points read); slice Z = z + M and row
// Y = y + M for true coordinates z, y in [-M, N + M) (row (y, z) holds
// receptor row (y mod N, z mod N): the periodic domain of the FFT with M
// rows continued past each end, so a row index z + t_z or y + t_y of a
// ligand point within M of the box needs no reducing); word q holds the
// row's points x in [32 (q - 1), 32 q), taken mod N, for q in [0, RW), so a
// run starting at x >= -32 reads its words without wrapping; row Y fastest
// (a wavefront's 64 consecutive rows read one contiguous 256-byte run per
// word).  The whole table is 4.0 MB at N = 128, about one XCD's L2.
template <int N>
struct Dil {
    static constexpr int NW = N / 32;
    static constexpr int M = 8;
    static constexpr int E = N + 2 * M;
    static constexpr int RW = NW + 4;
    static constexpr int K = ilog2c(RUN_MAX + 1);
    static_assert((1 << (K - 1)) <= N, "a level's window must fit in a row");
    __host__ __device__ static constexpr int64_t words() { return (int64_t)K * E * RW * E; }
    __host__ __device__ static constexpr int64_t index(int k, int Z, int q, int Y) {
        return (((int64_t)k * E + Z) * RW + q) * E + Y;
    }
};

// LDS budget of the per-block factor table of the fused z kernel.
constexpr size_t FUSED_TABLE_BYTES = 16384;

struct FusedSet {
    int n_fft;
    int64_t dil_words;  // words of one snapshot's dilation table
    int margin;         // Dil<N>::M: occupancy may reach this many points past the box
    // occ [n_rec^3] bytes -> dil (Dil<N> layout)
    hipError_t (*rec_dilate)(hipStream_t, const uint8_t *occ, int n_rec, uint32_t *dil);
    // ligand occupancy runs of the scanned configurations zcfg[0..nz) of a
    // chunk: two words per run from runs[2 run_off], run_count[local index]
    hipError_t (*lig_runs)(hipStream_t, const CfgDev *cfgs, const int32_t *zcfg, int nz, const int32_t *ulat,
                           const double *thr, uint32_t *runs, int32_t *run_count);
    // free bits and live flags: item_off[0..n_cfg] running counts of the
    // phase-1 items (tz, 64-row group), item2_off those of the phase-2 items
    // (64-row slices of a configuration's undecided-row list); surv holds the
    // lists (at surv_off), scnt their lengths (n_cfg ints, cleared here)
    hipError_t (*clash)(hipStream_t, const int32_t *item_off, const int32_t *item2_off, int n_cfg, int n_items,
                        int n_items2, const CfgDev *cfgs, const uint32_t *runs, const int32_t *run_count,
                        const uint32_t *dil, uint32_t *fb, uint8_t *live, uint32_t *surv, int32_t *scnt);
    // per scanned configuration of a chunk: its atoms sorted by plane with
    // their x/y placement and channel weights, and the plane starts
    // (zat: nz x max_atoms records, zbt: nz x (N + 2) ints)
    hipError_t (*zprep)(hipStream_t, const CfgDev *cfgs, const int32_t *zcfg, int nz, int max_atoms,
                        const int32_t *ulat, const void *gam, void *zat, int32_t *zbt);
    size_t zat_bytes;  // bytes of one atom record
    // z pass of one snapshot (spectra rspec, 3 energy channels)
    hipError_t (*zpass)(hipStream_t, bool zhalf, bool clash, const CfgDev *cfgs, const int32_t *zcfg, int nz,
                        int max_atoms, const void *zat, const int32_t *zbt, const void *rspec, const void *tw,
                        void *wsi, const uint8_t *live);
    // z pass of one snapshot from energy planes in ws (direct forward pass)
    hipError_t (*zplanes)(hipStream_t, bool zhalf, bool clash, const CfgDev *cfgs, const int32_t *zcfg, int nz,
                          const void *ws, const void *rspec, const void *tw, void *wsi, const uint8_t *live);
    // inverse xy + Eq. 2 plane partials; e_count (nullable) counts planes read
    hipError_t (*inv)(hipStream_t, bool clash, const int32_t *inv_off, int n_cfg, int n_items, const CfgDev *cfgs,
                      const void *wsi, double beta, const void *tw, const uint32_t *fb, const uint8_t *live,
                      void *pp, void *psi_out, uint8_t *clash_out, unsigned int *e_count);
    // dynamic LDS bytes of the z kernel for ligands of up to max_atoms atoms
    size_t (*z_lds)(int max_atoms);
};

// nullptr where the fused path is not built (N = 256)
const FusedSet *fused_set(int precision, int n_fft);

}  // namespace fftdg

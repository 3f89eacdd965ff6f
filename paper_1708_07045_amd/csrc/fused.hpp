// Host/device view of the fused scan path: bit tables of the clash test and
// the launchers (one set per precision and FFT edge, N <= 128).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "scan_types.hpp"

namespace fftdg {

__host__ __device__ constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

// OR-dilated receptor occupancy rows of one snapshot, u32 words
// [k][Z][q][Y]: level k (window 2^k, k = 0 .. log2 N); slice Z and row Y
// over two periods, 0 .. 2N - 1 (row (Y, Z) is row (Y mod N, Z mod N), so
// a row index y + t_y or z + t_z never needs reducing); word q of the
// periodic row continued for RW = 2 N/32 + 2 words (word q holds the row's
// word q mod N/32, so windows starting anywhere in the first period and
// spanning up to N/32 + 2 words never wrap); row Y fastest (a wavefront's
// 64 consecutive rows read one contiguous 256-byte run per word).
template <int N>
struct Dil {
    static constexpr int NW = N / 32;
    static constexpr int RW = 2 * NW + 2;
    static constexpr int K = ilog2c(N) + 1;
    static constexpr int N2 = 2 * N;
    __host__ __device__ static constexpr int64_t words() { return (int64_t)K * N2 * RW * N2; }
    __host__ __device__ static constexpr int64_t index(int k, int Z, int q, int Y) {
        return (((int64_t)k * N2 + Z) * RW + q) * N2 + Y;
    }
};

// LDS budget of the per-block factor table of the fused z kernel.
constexpr size_t FUSED_TABLE_BYTES = 16384;

struct FusedSet {
    int n_fft;
    int64_t dil_words;  // words of one snapshot's dilation table
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

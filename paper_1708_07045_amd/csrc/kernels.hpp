// Host-side view of the kernel launchers (one set per precision and FFT edge).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fftdg.h"
#include "scan_types.hpp"

namespace fftdg {

struct KernelSet {
    int n_fft;
    int cbytes;   // bytes per complex element
    int ppbytes;  // bytes per plane partial
    int np;       // complex elements per half-plane, n_fft * (n_fft/2 + 1)
    // receptor spectra of one snapshot: grids [3][n_rec^3] (+ occ [n_rec^3])
    // -> rspec [n_ch][N][np]; rxy is scratch [n_ch][n_rec][np]
    hipError_t (*rec_spectra)(hipStream_t, const void *grids, const uint8_t *occ, int n_rec, int n_ch,
                              const void *tw, void *rxy, void *rspec);
    // one block per forward plane (edf: one per energy z-plane for all three
    // channels, evaluated directly, plus one per occupancy plane);
    // fwd_off[0..n_cfg] running item counts
    hipError_t (*fwd)(hipStream_t, bool edf, const int32_t *fwd_off, int n_cfg, int n_items, const CfgDev *cfgs,
                      const int32_t *ulat, const void *gam, const double *thr, const void *tw, void *ws);
    // edirect: energy-channel xy transforms evaluated per atom inside the
    // kernel (else read from forward planes written by fwd)
    // n_snap snapshots per launch: spectra spec_stride and outputs inv_stride
    // complex elements apart
    // zhalf: 1 = every configuration's energy planes lie in [0, n_fft/2);
    // 2 = that, and some occupancy window spans more than n_fft/2 planes
    hipError_t (*zprod)(hipStream_t, bool occ, bool edirect, int zhalf, const CfgDev *cfgs, const int32_t *zcfg, int nz,
                        const void *ws, const void *rspec, const void *tw, void *wsi, const int32_t *ulat,
                        const void *gam, int n_snap, int64_t spec_stride, int64_t inv_stride);
    // e_count (nullable): incremented once per energy plane transformed
    // one block per valid z translation; inv_off[0..n_cfg] running counts
    hipError_t (*inv)(hipStream_t, bool occ, const int32_t *inv_off, int n_cfg, int n_items, const CfgDev *cfgs,
                      const void *wsi, double beta, const void *tw, void *pp, void *psi_out,
                      uint8_t *clash_out, unsigned int *e_count);
    hipError_t (*merge)(hipStream_t, const CfgDev *cfgs, int n_cfg, const void *pp, fftdg_partial *out);
};

const KernelSet *kernel_set(int precision, int n_fft);

hipError_t launch_reduce(hipStream_t st, const fftdg_partial *p, int64_t n_cfg_total, int n_snap, int n_lig,
                         const int32_t *cfg_off, const double *cfg_w, const double *W, double kT, double h3,
                         double c0, double *B, LigRed *res);

hipError_t launch_grid_energies(hipStream_t st, int precision, const void *grids, int n_rec, double h,
                                const double *origin, int n_atoms, const double *lq, const double *ls,
                                const double *le, int n_poses, const double *pose, double *out);
hipError_t launch_pair_energies(hipStream_t st, int n_rec_atoms, const double *rxyz, const double *rq,
                                const double *rs, const double *re, int n_atoms, const double *lq,
                                const double *ls, const double *le, int n_poses, const double *pose, int excl,
                                double *out);

hipError_t launch_sample_translations(hipStream_t st, int precision, const void *psi, const uint8_t *clash, int n,
                                     double beta, const double *u, int nu, int32_t *out_lin, double *out_psi);

hipError_t launch_scan_features(hipStream_t st, const fftdg_partial *p, int64_t n_cfg_total, int n_snap, int n_lig,
                                const int32_t *cfg_off, const double *W, float *feat, int ld, int col0);

hipError_t launch_receptor_grids(hipStream_t st, int precision, int n_atoms, const double *xyz, const double *q,
                                 const double *sg, const double *ep, int n_rec, double h, const double *origin,
                                 int mode, double cap, double occ_f, void *grids, uint8_t *occ);

}  // namespace fftdg

/*
 * fftdg — FFT translational scan for binding potentials of mean force
 * (BPMF) and standard binding free energies on AMD Instinct MI355X (gfx950).
 *
 * Method: Nguyen, Zhou & Minh, "Using the Fast Fourier Transform in Binding
 * Free Energy Calculations".  For every rigid ligand configuration (conformer
 * x random rotation about its centroid), the ligand's electrostatic and
 * Lennard-Jones weights (Eqs. 3-6) and its occupancy (Eq. 10) are spread onto
 * grids, correlated with precomputed receptor grids through the FFT (Eqs.
 * 8-9), giving the interaction energy at every grid translation; translations
 * whose ligand box leaves the receptor grid are discarded and sterically
 * clashing ones are infinite; the energies are exponentially averaged into
 * the BPMF (Eq. 2) and over receptor snapshots into the standard binding
 * free energy (Eqs. 12-13).
 *
 * Conventions (all calls):
 *   - units: Angstrom, elementary charge, kcal/mol, Kelvin; sigma is the
 *     r_min-form Lennard-Jones radius (the pair minimum -eps_ij sits at
 *     r = sigma_ij, Eqs. 5-6);
 *   - 3-D arrays are [z][y][x] with x fastest; grid point (x,y,z) sits at
 *     origin + h*(x,y,z);
 *   - "_dev" pointers are device memory on the context's device, "_host"
 *     pointers are host memory; the caller owns every pointer it passes in;
 *   - device work is ordered on the context's stream and is asynchronous
 *     unless a call says it synchronizes;
 *   - every call returns FFTDG_OK (0) or a negative status; on failure
 *     fftdg_last_error() describes it; no call throws or aborts;
 *   - one context must not be used by two host threads at once.
 */
#ifndef FFTDG_H
#define FFTDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FFTDG_VERSION 10000

/* status codes */
#define FFTDG_OK 0
#define FFTDG_E_INVALID (-1) /* null pointer, bad size/offset, unsupported n_fft, non-finite input, T <= 0, ... */
#define FFTDG_E_NOVALID (-2) /* a ligand has no box-valid translation in any configuration */
#define FFTDG_E_NOMEM (-3)   /* device or host allocation failed, or a workspace limit was exceeded */
#define FFTDG_E_DEVICE (-4)  /* any HIP runtime error, including "no device" */
#define FFTDG_E_STATE (-5)   /* call out of order (e.g. scan before set_receptors) */

/* precision of grids, FFTs and energies */
#define FFTDG_F32 0
#define FFTDG_F64 1

/* clash handling (readings of the exclusion and occupancy rules of the
 * FFT-based BPMF estimation section) */
#define FFTDG_OCC 0 /* three energy grids zeroed inside 2^-1/6 sigma, plus an occupancy grid; clash -> +inf */
#define FFTDG_CAP 1 /* three energy grids, LJ repulsion kept inside 2^-1/6 sigma and clamped; no clash test */

typedef struct fftdg_ctx fftdg_ctx;

/* Grid description (FFT-based BPMF estimation section).
 *   n_rec  receptor grid edge in points (the ligand box must fit inside)
 *   n_fft  FFT edge, n_fft >= n_rec; receptor grids are zero-padded to it.
 *          Supported: 32, 64, 128, 256 (FFTDG_F32); 32, 64 (FFTDG_F64).
 *          At 256 (a 62 A grid at 0.25 A) the xy transforms run as
 *          separate row and column passes over planes in device memory,
 *          and energy_xy_direct = 1 is not available.
 *          In FFTDG_OCC mode choose n_fft >= n_rec + occupancy radius so
 *          that the periodic wrap only meets padding.
 *   h      grid spacing (A), origin position of point (0,0,0) (A)
 *   ljr_cap  FFTDG_CAP only: LJ-repulsive grid values are clamped to it
 *          (kcal/mol per unit ligand weight)
 *   occ_f  FFTDG_OCC only: occupancy radius rho_i = occ_f 2^-1/6 sigma_i
 *          for ligand and receptor atoms (the paper's literal rule is 1). */
typedef struct {
    int32_t n_rec;
    int32_t n_fft;
    double h;
    double origin[3];
    int32_t precision;
    int32_t clash_mode;
    double ljr_cap;
    double occ_f;
} fftdg_grid_desc;

/* A batch of ligands and their rigid configurations (host memory).
 *   ligand l owns atoms atom_off[l] .. atom_off[l+1]-1 (n_l atoms, <= 256),
 *   conformers conf_off[l] .. conf_off[l+1]-1 and configurations
 *   cfg_off[l] .. cfg_off[l+1]-1;
 *   q, sigma, eps: per atom (e, A, kcal/mol);
 *   conf_xyz: the conformers' coordinates, ligand by ligand, conformer by
 *     conformer, atom by atom, [.][3] doubles (A);
 *   cfg_conf[c]: conformer of configuration c, local to its ligand;
 *   cfg_quat[c][4]: rotation (w,x,y,z) about the conformer's unweighted
 *     centroid ("Ligand Sampling"); need not be normalised, must be non-zero;
 *   cfg_select: NULL = scan every configuration; else scan only those with
 *     cfg_select[c] != 0 (the others still count their translations in the
 *     sample size, as importance sampling over configurations needs). */
typedef struct {
    int32_t n_lig;
    const int32_t *atom_off;
    const int32_t *conf_off;
    const int32_t *cfg_off;
    const double *q;
    const double *sigma;
    const double *eps;
    const double *conf_xyz;
    const int32_t *cfg_conf;
    const double *cfg_quat;
    const uint8_t *cfg_select;
} fftdg_batch;

/* Per-(snapshot, configuration) partial of the sample mean of Eq. 2, over
 * the configuration's box-valid translations.  x = -Psi/kT;
 *   m = max x over finite samples (-inf if none), s = sum exp(x - m),
 *   psi_min = min Psi (+inf if none), n_valid = box-valid translations
 *   (clashes included), n_finite = non-clashing ones, argmin = linear index
 *   (tz*Vy + ty)*Vx + tx of psi_min (lowest on ties, -1 if none).
 * m, s, psi_min are computed in the context precision. */
typedef struct {
    double m;
    double s;
    double psi_min;
    int32_t n_valid;
    int32_t n_finite;
    int32_t argmin;
    int32_t scanned; /* 1 if the configuration was scanned */
} fftdg_partial;

/* Per-ligand result of fftdg_reduce. */
typedef struct {
    double dG;        /* Eq. 13, kcal/mol (+inf if every snapshot's BPMF is +inf) */
    double v_site;    /* A^3: h^3 x mean over configurations of box-valid translations */
    double psi_min;   /* min interaction energy over snapshots and configurations */
    int64_t n_finite; /* non-clashing samples over snapshots */
    int64_t n_samples; /* box-valid samples per snapshot (sum over configurations) */
} fftdg_ligand_result;

int fftdg_version(void);
const char *fftdg_status_string(int status);

/* Create a context on HIP device `device`, ordering work on `hip_stream`
 * (a hipStream_t, or NULL for the default stream).  Validates g.
 * Errors: E_INVALID (g), E_DEVICE (no device / HIP error), E_NOMEM. */
int fftdg_create(fftdg_ctx **out, const fftdg_grid_desc *g, int device, void *hip_stream);
void fftdg_destroy(fftdg_ctx *ctx);
const char *fftdg_last_error(const fftdg_ctx *ctx);
int fftdg_set_stream(fftdg_ctx *ctx, void *hip_stream);

/* Receptor grids of Eq. 7 (ELE = 332.05 q/r, LJr = sqrt(eps) sigma^6/r^12,
 * LJa = sqrt(eps) sigma^3/r^6, with the exclusion rule of the clash mode) and
 * the receptor occupancy grid of Eq. 10, built on the GPU in FP64 from
 * receptor atoms (xyz_dev [n_atoms][3], q/sigma/eps_dev [n_atoms], all
 * double, device).  Writes grids_dev [3][n_rec^3] in the context precision
 * and, in FFTDG_OCC mode, occ_dev [n_rec^3] (0/1 bytes; may be NULL in CAP).
 * Asynchronous. */
int fftdg_receptor_grids(fftdg_ctx *ctx, int32_t n_atoms, const double *xyz_dev,
                         const double *q_dev, const double *sigma_dev, const double *eps_dev,
                         void *grids_dev, uint8_t *occ_dev);

/* Precompute the receptor spectra FT(G_R) of Eq. 9 for n_snap snapshots.
 *   grids_dev [n_snap][3][n_rec^3] (context precision, device)
 *   occ_dev   [n_snap][n_rec^3] bytes (device), required in OCC, ignored in CAP
 *   w_host    [n_snap] snapshot weights W of Eq. 13 (normalised internally,
 *             must be >= 0 with a positive sum); NULL = uniform.
 * The library owns the spectra; the caller may free its grids once the
 * stream has passed this call.  Replaces any previous receptor set. */
int fftdg_set_receptors(fftdg_ctx *ctx, int32_t n_snap, const void *grids_dev,
                        const uint8_t *occ_dev, const double *w_host);

/* The scan (Eqs. 2, 8-10): places every configuration of the batch (host,
 * FP64, exact integer box), runs the FFT correlation against every receptor
 * snapshot and writes out_dev[snap * n_cfg_total + c] (device) for all
 * snapshots and configurations.  Temperature T_K > 0.  Asynchronous: keep
 * out_dev alive until the stream passes this call.  Besides the chunk
 * workspaces the context holds one plane partial (20 B in FP32, 32 B in
 * FP64) per valid z-translation of the batch and snapshot until the scan's
 * final merge; E_INVALID if a batch has more than 2^31 of them per snapshot.
 * Errors: E_STATE (no receptors), E_INVALID, E_NOVALID (a ligand without
 * any box-valid translation), E_NOMEM, E_DEVICE. */
int fftdg_scan(fftdg_ctx *ctx, const fftdg_batch *b, double T_K, fftdg_partial *out_dev);

/* Raw interaction energy Psi (Eq. 8, before clash masking) at every
 * box-valid translation of one configuration `cfg` (index into the batch)
 * against snapshot `snap`: psi_dev [Vz][Vy][Vx] in the context precision,
 * clash_dev [Vz][Vy][Vx] bytes (NULL allowed; all 0 in CAP mode).  shape_host
 * receives {Vz, Vy, Vx}; call with psi_dev == NULL to query the shape only.
 * Synchronizes the stream. */
int fftdg_energy_grid(fftdg_ctx *ctx, int32_t snap, const fftdg_batch *b, int32_t cfg,
                      double T_K, void *psi_dev, uint8_t *clash_dev, int32_t *shape_host);

/* Placement of configuration `cfg` as the scan does it: lattice coordinates
 * U_host [n_atoms][3] (grid units x 2^16) and the box extents box_host[3]
 * (x, y, z).  Host only. */
int fftdg_place(fftdg_ctx *ctx, const fftdg_batch *b, int32_t cfg, int32_t *U_host,
                int32_t *box_host);

/* FP64 exponential averages on the GPU (Eqs. 2, 12, 13):
 *   ln Z_{l,s} = LSE over configurations c of ligand l of
 *                ln(w_c) + m_{s,c} + ln s_{s,c}   (w_c = 1 if cfg_weight_dev
 *                is NULL; else cfg_weight_dev[c] >= 0, e.g. multiplicity/(K q_c)
 *                for importance sampling)
 *   B_{l,s}    = -kT (ln Z_{l,s} - ln sum_c n_valid_c)
 *   dG_l       = -kT ln sum_s W_s exp(-B_{l,s}/kT) - kT ln(V_site C0),
 *                V_site = h^3 mean_c n_valid_c, C0 = 1 M.
 * p_dev as written by fftdg_scan for the same batch.  Writes B_host
 * [n_lig][n_snap] and res_host [n_lig] (host).  Synchronizes the stream. */
int fftdg_reduce(fftdg_ctx *ctx, const fftdg_batch *b, const fftdg_partial *p_dev,
                 const double *cfg_weight_dev, double T_K, double *B_host,
                 fftdg_ligand_result *res_host);

/* Bytes of the static device scratch behind fftdg_reduce_static. */
#define FFTDG_REDUCE_STATIC_BYTES (4 << 20)

/* fftdg_reduce for callers that cannot allocate device memory at call time
 * (code between graph captures, tight serving loops, hosts that forbid
 * hipMalloc): same arguments, same kernel, bit-identical B_host and res_host.
 * Its staging buffers (cfg_off, W, B, per-ligand results; 256-byte aligned
 * pieces) live in one static device array of FFTDG_REDUCE_STATIC_BYTES per
 * device, looked up once per device by fftdg_create and held until the
 * process ends; the call makes no hipMalloc, hipFree or other allocation.
 * Batches needing more, about 4 (n_lig + 1) + 8 n_snap + 8 n_lig n_snap +
 * 40 n_lig bytes plus alignment (some 33 000 ligands at 10 snapshots), get
 * E_INVALID with the figures in fftdg_last_error.  Every call on one device
 * shares that device's array and nothing in it must start at zero (the kernel
 * writes every output): calls that overlap in time on one device (other
 * threads, other contexts or streams) race; one call ends with a stream
 * synchronize, so calls made one after the other do not.  Not recorded by
 * fftdg_profile. */
int fftdg_reduce_static(fftdg_ctx *ctx, const fftdg_batch *b, const fftdg_partial *p_dev,
                        const double *cfg_weight_dev, double T_K, double *B_host,
                        fftdg_ligand_result *res_host);

/* Kernel timing with HIP events recorded on the context's stream around
 * every launch the library makes (for benchmarks).  Kernel ids:
 *   0 ligand xy forward   1 z-pencil product   2 inverse xy + log-sum-exp
 *   3 plane merge         4 receptor spectra   5 FP64 reduce
 *   6 ligand occupancy runs (fused path)       7 clash test on bits (fused path)
 * fftdg_profile(ctx, 1) clears the counters and starts recording; 0 stops.
 * fftdg_profile_read synchronizes the stream and returns, for kernel id k,
 * the summed event time (ms), the launch count and the algorithmic HBM
 * bytes those launches must move (inputs read once, outputs written once;
 * the per-launch figures are documented with the kernels). */
#define FFTDG_K_FWD 0
#define FFTDG_K_ZPROD 1
#define FFTDG_K_INV 2
#define FFTDG_K_MERGE 3
#define FFTDG_K_SPECTRA 4
#define FFTDG_K_REDUCE 5
#define FFTDG_K_RUNS 6
#define FFTDG_K_CLASH 7
#define FFTDG_N_KERNELS 8
int fftdg_profile(fftdg_ctx *ctx, int enable);
int fftdg_profile_read(fftdg_ctx *ctx, int32_t kernel_id, double *ms_host, int64_t *launches_host,
                       double *alg_bytes_host);

/* Sampling importance resampling of poses (solvation section: poses for the
 * single-step perturbation, Eq. 11, are drawn from the scanned bound state with
 * weight exp(-Psi/kT)).  For ligand `lig` and snapshot `snap` of a finished
 * scan of batch b (partials p_dev as written by fftdg_scan), draws K poses
 * (configuration c, translation t), with replacement, with probability
 * exp(-Psi_c(t)/kT) / Z over every clash-free box-valid translation of every
 * scanned configuration of the ligand, in two inverse-CDF steps (the random
 * numbers are inputs, u_host [2K] in [0, 1)):
 *   configuration: the running sum over the ligand's configurations in index
 *     order of Z_c = exp(m_c - max m) s_c (FP64, from the partials) is
 *     searched for u_host[2k] times its total (first sum exceeding it);
 *   translation: the configuration's energies are recomputed as
 *     fftdg_energy_grid does and the running sum over its clash-free
 *     translations in linear order (tz, ty, tx) of exp(-(Psi - min Psi)/kT)
 *     (FP64) is searched for u_host[2k+1] times its total.
 * Writes cfg_host [K] (configuration index in the batch), t_host [K][3]
 * (tx, ty, tz, valid-translation indices as in fftdg_energy_grid) and
 * psi_host [K] (the pose's Psi, kcal/mol).  E_NOVALID if the ligand has no
 * clash-free translation in that snapshot.  Synchronizes the stream. */
int fftdg_sample_poses(fftdg_ctx *ctx, const fftdg_batch *b, const fftdg_partial *p_dev, int32_t lig,
                       int32_t snap, double T_K, int32_t K, const double *u_host, int32_t *cfg_host,
                       int32_t *t_host, double *psi_host);

/* ------------------------------------------------------------------------
 * Grid tools without an FFT context, for the accuracy of grid-based energies
 * against direct atom-pair sums as the spacing varies (section on the
 * accuracy of FFT-based interaction energies).  Each call launches on
 * hip_stream of `device`, is asynchronous and returns E_INVALID for bad
 * sizes or NULL pointers, E_DEVICE for HIP errors (no error text: there is
 * no context).  n_fft of the grid description is ignored; any edge
 * 2 <= n_rec <= 1024 is allowed.  All arrays are device arrays.
 * ------------------------------------------------------------------------ */

/* Eq. 7 grids [3][n_rec^3] (context precision of g) and Eq. 10 occupancy
 * [n_rec^3] (OCC mode; NULL in CAP mode), exactly as fftdg_receptor_grids. */
int fftdg_grids_build(int device, void *hip_stream, const fftdg_grid_desc *g, int32_t n_atoms,
                      const double *xyz_dev, const double *q_dev, const double *sigma_dev,
                      const double *eps_dev, void *grids_dev, uint8_t *occ_dev);

/* Interaction energies of n_poses ligand poses (atom coordinates
 * pose_xyz_dev [n_poses][n_atoms][3], Angstrom) from grids of g by trilinear
 * interpolation at each atom (Eqs. 3 and 8 at one position; corners outside
 * the grid read as zero), with the ligand weights of Eqs. 4-6 from the atom
 * parameters q, sigma, eps [n_atoms]; FP64.  out_dev [n_poses][3] =
 * (ELE, LJr, LJa) in kcal/mol.  n_atoms <= 256. */
int fftdg_grid_energies(int device, void *hip_stream, const fftdg_grid_desc *g, const void *grids_dev,
                        int32_t n_poses, int32_t n_atoms, const double *q_dev, const double *sigma_dev,
                        const double *eps_dev, const double *pose_xyz_dev, double *out_dev);

/* Direct atom-pair interaction energies of the same poses with receptor
 * atoms rxyz_dev [n_rec_atoms][3] (Eqs. 4-6 without grids), FP64:
 *   ELE 332.05 q_i q_j / r,  LJr sqrt(eps_i eps_j) (sigma_i sigma_j)^6 / r^12,
 *   LJa -2 sqrt(eps_i eps_j) (sigma_i sigma_j)^3 / r^6;
 * exclusion = 1 drops every term of a pair closer than 2^(-1/6) sigma_j (the
 * receptor atom's, as in the occupancy-mode grids); 0 keeps all pairs.
 * out_dev [n_poses][3].  n_atoms <= 256. */
int fftdg_pair_energies(int device, void *hip_stream, int32_t n_rec_atoms, const double *rxyz_dev,
                        const double *rq_dev, const double *rsigma_dev, const double *reps_dev, int32_t n_poses,
                        int32_t n_atoms, const double *q_dev, const double *sigma_dev, const double *eps_dev,
                        const double *pose_xyz_dev, int32_t exclusion, double *out_dev);

/* Execution schedule (results do not depend on it beyond rounding order of
 * the FP32 transforms):
 *   configs_per_chunk  configurations whose forward and inverse planes share
 *                      device workspace at one time (>= 1, default 256);
 *   energy_xy_direct   how the x/y transforms of the three energy channels
 *                      are done (each is the xy DFT of the trilinearly
 *                      spread plane): 0: the same LDS-staged xy FFT pass as
 *                      the occupancy channel, through HBM (default);
 *                      1: evaluated per atom inside the z-pencil kernel, no
 *                      HBM planes; 2: evaluated per atom in the forward
 *                      pass (one block writes a z-plane of all three
 *                      channels), through HBM;
 *   snapshots_per_pass receptor snapshots handled by one z-pencil launch
 *                      (>= 1, default 1): with more than one, a
 *                      configuration's forward z spectra stay in registers
 *                      while the products and inverse transforms of every
 *                      snapshot of the pass are computed; the inverse planes
 *                      of all of them share device workspace;
 *   use_graph          1: the scan's launch sequence is captured once into a
 *                      hipGraph (kernel nodes only) and replayed by later
 *                      scans whose launch shapes, buffers and temperature
 *                      are unchanged (the new placement tables are uploaded
 *                      first); not used while profiling or exporting
 *                      energies.  Default 0;
 *   fused              1 or 2 (1 is the default where available: n_fft <=
 *                      128): only the three energy channels go through the
 *                      FFT; in OCC mode the clash test of Eq. 10 is made
 *                      exactly on bits (ligand occupancy runs against
 *                      OR-dilated receptor occupancy rows) before the z pass,
 *                      and only z-translations with a clash-free translation
 *                      are stored and inverse-transformed.  1: the energy
 *                      planes' x/y transforms come from the direct per-atom
 *                      forward pass through device memory; 2: the z-pencil
 *                      kernel forms its inputs itself from the per-atom
 *                      factors (no forward planes).  energy_xy_direct and
 *                      snapshots_per_pass are then not used.  0: the
 *                      occupancy channel as a fourth FFT channel thresholded
 *                      at 1/2 (the paper's formulation);
 *   clash_stream       1 (default) uses a second stream of the context
 *                      (default priority, created on first use), its
 *                      buffers double-buffered and the streams ordered by
 *                      events: on the fused path in OCC mode the clash test
 *                      of the next (chunk, snapshot) runs on it beside the z
 *                      pass and inverse of the current one; on the plane
 *                      path (fused = 0) the inverse xy of one z pass runs on
 *                      it beside the next z pass (twice the inverse
 *                      workspace).  0 runs everything on the context's
 *                      stream.  Not used while profiling or exporting
 *                      energies. */
typedef struct {
    int32_t configs_per_chunk;
    int32_t energy_xy_direct;
    int32_t snapshots_per_pass;
    int32_t use_graph;
    int32_t fused;
    int32_t clash_stream;
} fftdg_tuning;
int fftdg_get_tuning(const fftdg_ctx *ctx, fftdg_tuning *out);
int fftdg_set_tuning(fftdg_ctx *ctx, const fftdg_tuning *t);

/* Autotuner: times the candidate schedules (configurations per chunk in
 * {64, 128, 256, 512}, use_graph in {0, 1}, and fused in {1, 2} with
 * clash_stream in {0, 1} (OCC mode) where available or
 * fused = 0 with energy_xy_direct in {0, 1, 2}, clash_stream in {0, 1} and
 * snapshots_per_pass in {1, n_snap} when there are several snapshots) with
 * HIP events, each by the fastest of four runs after a warm-up, on an evenly
 * strided sample of at most max_cfgs configurations of the batch (all
 * receptor snapshots), keeps the fastest in the context and writes it to
 * out (may be NULL); ms_host (may be NULL) receives its time per sampled
 * configuration and snapshot.  Synchronizes the stream.  Results of later
 * scans do not depend on the choice beyond FP rounding order. */
int fftdg_autotune(fftdg_ctx *ctx, const fftdg_batch *b, double T_K, int32_t max_cfgs, fftdg_tuning *out,
                   double *ms_host);

/* ------------------------------------------------------------------------
 * Learned importance-sampling proposal over ligand configurations.
 *
 * Not part of the paper: Eq. 2 is estimated from a subset of configurations
 * drawn from a proposal q built from a small network's prediction of each
 * configuration's log Boltzmann weight, with exact 1/q reweighting through
 * fftdg_reduce's cfg_weight; the exhaustive scan stays the fallback and the
 * reference its error is measured against.
 * ------------------------------------------------------------------------ */

/* Per-configuration input features (host; FFTDG_N_FEATURES floats each):
 *   [0..3]   rotation quaternion, normalised, sign fixed to w >= 0 (q = -q)
 *   [4..11]  one-hot of the conformer index modulo 8
 *   [12]     n_atoms / 40,   [13] ln(n_atoms) / ln(40)
 *   [14..16] placed extent along x, y, z in units of 10 A
 *   [17]     radius of gyration of the conformer in units of 5 A
 * feat_host [n_cfg_total][FFTDG_N_FEATURES]. */
#define FFTDG_N_FEATURES 18
int fftdg_config_features(fftdg_ctx *ctx, const fftdg_batch *b, float *feat_host);

/* Per-configuration descriptors of a finished scan by this context (for
 * instance a coarse-spacing context over the same batch, whose scan is a
 * cheap predictor of the fine one), from partials p_dev [n_snap][n_cfg_total]
 * and the context's snapshot weights W_s, in FP64:
 *   x_c   = ln sum_s W_s Z_{c,s}   (Z as in fftdg_reduce, Eq. 2)
 *   psi_c = min_s psi_min_{c,s},   f_c = sum_s n_finite / sum_s n_valid
 * written as floats into columns col0 .. col0+2 of the row-major device
 * matrix feat_dev [n_cfg_total][ld]:
 *   (max(x_c - max_l x, -25) / 5,  min(psi_c - min_l psi, 50) / 10,  f_c)
 * with max_l / min_l over the configurations of the same ligand; a
 * configuration with nothing finite gets (-5, 5, 0).  Other columns are not
 * touched.  Asynchronous on the context's stream. */
#define FFTDG_N_SCAN_FEATURES 3
int fftdg_scan_features(fftdg_ctx *ctx, const fftdg_batch *b, const fftdg_partial *p_dev, float *feat_dev,
                        int32_t ld, int32_t col0);

/* Stratified importance-sampling plan over each ligand's P configurations
 * (host only).  From predicted log weights yhat_host [n_cfg_total]:
 *   - the n_top = ceil(top_frac P) configurations of largest yhat (ties to
 *     the lower index) are scanned exactly: select 1, weight 1;
 *   - over the other R = P - n_top, taken in increasing index order, the
 *     defensive mixture q_j = (1 - alpha) softmax(yhat / tau)_j + alpha / R
 *     (FP64) is sampled K = ceil(draw_frac P) times (none if R = 0) by
 *     inverse CDF: draw k takes the first j whose running sum of q exceeds
 *     u_k times the total; a drawn configuration gets select 2 and weight
 *     multiplicity / (K q_j);
 *   - all others: select 0, weight 0.
 * Uniforms u_host in [0, 1) are consumed in ligand order (ligand 0's K
 * first); n_u must cover them all.  With these weights fftdg_reduce returns
 *   Z_hat = sum_top Z_c + (1/K) sum_k Z_{c_k} / q_{c_k},
 * an unbiased estimate of sum_c Z_c for any yhat (exact when top_frac = 1).
 * select_host [n_cfg_total] (nonzero = scan; 1 exact stratum, 2 drawn) can
 * be used as the batch's cfg_select and
 * weight_host [n_cfg_total] (upload it) as fftdg_reduce's cfg_weight.
 * n_scan_host (may be NULL) receives the number of selected configurations.
 * Host only: needs no device, and ctx may be NULL (no error text is kept).
 * E_INVALID: NULL pointer, fractions outside [0, 1], alpha outside [0, 1],
 * tau <= 0, non-finite yhat, too few uniforms. */
int fftdg_is_plan(fftdg_ctx *ctx, const fftdg_batch *b, const float *yhat_host, double top_frac,
                  double draw_frac, double alpha, double tau, const double *u_host, int64_t n_u,
                  uint8_t *select_host, double *weight_host, int64_t *n_scan_host);

/* Network: n_in inputs -> 3 hidden layers of `width` SiLU units -> 1 linear
 * output; BF16 MFMA products with FP32 accumulation, FP32 master parameters,
 * Adam (beta 0.9/0.999, eps 1e-8).  Flat FP32 parameter layout (row-major):
 *   W1 [width][n_in], b1 [width], W2 [width][width], b2 [width],
 *   W3 [width][width], b3 [width], W4 [1][width], b4 [1].
 * Loss of a batch: sum_i w_i (y_i - t_i)^2 / sum_i w_i.
 * Requirements: 1 <= n_in <= 64, width a multiple of 64 (<= 1024),
 * batches of at most max_batch rows.  Parameters start at zero: set them. */
typedef struct fftdg_mlp fftdg_mlp;
int fftdg_mlp_create(fftdg_mlp **out, int device, void *hip_stream, int32_t n_in, int32_t width,
                     int32_t max_batch);
/* The same network with a choice of operand type: fp32_operands = 0 is
 * fftdg_mlp_create (BF16 operands and activations); 1 keeps operands and
 * activations in FP32 (GEMMs on FP32 MFMA, FP32 accumulation throughout),
 * for checking gradients against an FP64 reference to FP32 rounding;
 * twice the activation memory.
 * E_INVALID for any other value, as for fftdg_mlp_create's arguments. */
int fftdg_mlp_create_ex(fftdg_mlp **out, int device, void *hip_stream, int32_t n_in, int32_t width,
                        int32_t max_batch, int32_t fp32_operands);
void fftdg_mlp_destroy(fftdg_mlp *m);
const char *fftdg_mlp_last_error(const fftdg_mlp *m);
int64_t fftdg_mlp_num_params(const fftdg_mlp *m);
/* host <-> device parameters (synchronizes; set also resets Adam) */
int fftdg_mlp_set_params(fftdg_mlp *m, const float *params_host, int64_t n);
int fftdg_mlp_get_params(fftdg_mlp *m, float *params_host, int64_t n);
/* Skip connection (the proposal's residual form): with col >= 0 the output
 * becomes net(x) + scale * x[col], in forward, gradients and training alike
 * (the term has no parameters: the network is trained on the residual
 * t - scale * x[col]).  col = -1 removes it (the default).  E_INVALID if col
 * is outside [-1, n_in) or scale is not finite. */
int fftdg_mlp_set_skip(fftdg_mlp *m, int32_t col, float scale);
/* y_dev[i] = net(x_dev[i]) for i < n (device arrays, x [n][n_in]) */
int fftdg_mlp_forward(fftdg_mlp *m, const float *x_dev, int32_t n, float *y_dev);
/* gradient of the loss over the rows idx_dev[0..B-1] (NULL = rows 0..B-1)
 * of x_all_dev [.][n_in], t_all_dev, w_all_dev into grad_dev (flat layout);
 * loss_host may be NULL (else synchronizes) */
int fftdg_mlp_grad(fftdg_mlp *m, const float *x_all_dev, const float *t_all_dev, const float *w_all_dev,
                   const int32_t *idx_dev, int32_t B, float *grad_dev, float *loss_host);
/* one Adam step on that gradient with learning rate lr */
int fftdg_mlp_train_step(fftdg_mlp *m, const float *x_all_dev, const float *t_all_dev,
                         const float *w_all_dev, const int32_t *idx_dev, int32_t B, float lr,
                         float *loss_host);
/* Defensive mixture q_c = (1 - alpha) softmax(yhat / tau)_c + alpha / P over
 * P configurations (FP64, q_dev [P]) and K inverse-CDF draws idx_dev [K] from
 * the given uniforms u_dev [K] in [0, 1) (the random numbers are inputs). */
int fftdg_proposal_sample(fftdg_mlp *m, const float *yhat_dev, int32_t P, double alpha, double tau, int32_t K,
                          const double *u_dev, int32_t *idx_dev, double *q_dev);

#ifdef __cplusplus
}
#endif
#endif /* FFTDG_H */

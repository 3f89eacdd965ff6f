// C-ABI runtime of libfftdg: context, validation, ligand placement, work
// planning and kernel launches.  See include/fftdg.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fftdg.h"
#include "fused.hpp"
#include "kernels.hpp"
#include "scan_types.hpp"

using namespace fftdg;

namespace {

constexpr double kR = 1.987204259e-3;       // kcal mol^-1 K^-1
constexpr double kC0 = 6.02214076e-4;       // 1 mol/L in A^-3
constexpr double kLat = 65536.0;            // placement lattice: 2^16 points per grid unit

struct DevBuf {
    void *p = nullptr;
    size_t n = 0;
};

}  // namespace

// Device scratch of fftdg_reduce_static: one copy per device, held until the
// process ends.  In host code `scratch` names a host-side stand-in, so host
// code never hands it to a kernel or a copy; it uses the device address that
// fftdg_create looks up once per device (static_scratch_ptr).
static __device__ __align__(256) unsigned char scratch[FFTDG_REDUCE_STATIC_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_addr[kMaxDevices] = {};  // device address of `scratch` per device, nullptr until looked up

// Device address of `scratch` on `device` (the current device), looked up
// on the first call for that device; nullptr with *why set on failure.
void *static_scratch_ptr(int device, std::string *why) {
    if (device < 0 || device >= kMaxDevices) {
        *why = "device index beyond the static scratch table";
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            *why = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        scratch_addr[device] = ptr;
    }
    return scratch_addr[device];
}

// The device reduce writes LigRed records that the host copies straight into
// fftdg_ligand_result.
static_assert(sizeof(LigRed) == sizeof(fftdg_ligand_result), "LigRed layout");
static_assert(offsetof(LigRed, dG) == offsetof(fftdg_ligand_result, dG) &&
                  offsetof(LigRed, v_site) == offsetof(fftdg_ligand_result, v_site) &&
                  offsetof(LigRed, psi_min) == offsetof(fftdg_ligand_result, psi_min) &&
                  offsetof(LigRed, n_finite) == offsetof(fftdg_ligand_result, n_finite) &&
                  offsetof(LigRed, n_samples) == offsetof(fftdg_ligand_result, n_samples),
              "LigRed layout");

}  // namespace

struct fftdg_ctx {
    fftdg_grid_desc g{};
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    void *scratch = nullptr;  // device address of the static scratch on `device`
    const KernelSet *ks = nullptr;
    const FusedSet *fs = nullptr;  // fused path (nullptr where not built)
    int n_ch = 3;  // receptor/ligand channels: 3 energy (+1 occupancy)
    DevBuf tw, rspec, rxy, ws_fwd, ws_inv, pp, tables, red_B, red_res, red_off, red_W;
    DevBuf dil, runs, run_cnt, fbits, lives;  // fused path: receptor bit rows, ligand runs, clash results
    DevBuf zat, zbt;                          // fused path: sorted atoms and plane starts per configuration
    DevBuf surv, scnt;                        // fused path: undecided rows of the clash test and their counts
    DevBuf sir_psi, sir_clash, sir_u, sir_lin, sir_psi_out;  // pose resampling
    int n_snap = 0;
    std::vector<double> W;
    void *pinned = nullptr;
    size_t pinned_n = 0;
    hipEvent_t staging_ev = nullptr;
    bool staging_used = false;
    int chunk_cfgs = 256;
    int edirect = 0;  // energy xy transforms: 0 FFT pass, 1 inside the z kernel, 2 direct in the forward pass
    int snap_group = 1;  // snapshots per z launch (limited by workspace)
    bool use_graph = false;
    int fused = 0;  // 0 plane path; fused path with energy planes from the forward pass (1) or built in the z kernel (2)
    // second stream: the fused path (OCC) tests the clash of the next item on
    // `side` beside the current z pass and inverse; the plane path runs the
    // inverse xy of one z pass on `side` beside the next z pass
    bool clash_stream = true;
    hipStream_t side = nullptr;  // second stream (default priority), created on first use
    // buffer set p: work on `side` (ev_side) and on the context's stream
    // (ev_main) that last produced or read it
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_side[2] = {nullptr, nullptr}, ev_main[2] = {nullptr, nullptr};
    hipStream_t cap_stream = nullptr;   // capture only; graphs run on `stream`
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<int64_t> graph_sig;
    DevBuf tune_out;     // partials written while autotuning
    size_t ws_limit = (size_t)24 << 30;
    // profiling
    bool prof = false;
    struct Rec {
        int k;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> ev_pool;
    double prof_ms[FFTDG_N_KERNELS] = {0};
    int64_t prof_n[FFTDG_N_KERNELS] = {0};
    double prof_bytes[FFTDG_N_KERNELS] = {0};
    DevBuf prof_cnt;  // energy planes transformed by the inverse-xy kernel
    bool prof_fused = false;  // the counted planes were also written by the fused z kernel
};

namespace {

int set_err(fftdg_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return set_err(ctx, FFTDG_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

hipEvent_t pool_event(fftdg_ctx *c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Launch `fn` (returning hipError_t) bracketed by profiling events.
template <class F>
hipError_t timed(fftdg_ctx *c, int k, double bytes, F &&fn) {
    if (!c->prof) return fn();
    hipEvent_t a = pool_event(c), b = pool_event(c);
    if (a) (void)hipEventRecord(a, c->stream);
    hipError_t e = fn();
    if (b) (void)hipEventRecord(b, c->stream);
    if (a && b) c->recs.push_back(fftdg_ctx::Rec{k, a, b, bytes});
    return e;
}

int reserve(fftdg_ctx *c, DevBuf &b, size_t bytes) {
    if (bytes <= b.n) return FFTDG_OK;
    if (b.p) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return set_err(c, FFTDG_E_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
        (void)hipFree(b.p);
        b.p = nullptr;
        b.n = 0;
    }
    size_t want = bytes + bytes / 8 + 256;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return set_err(c, FFTDG_E_NOMEM, "device allocation of " + std::to_string(want) + " bytes failed");
    }
    b.n = want;
    return FFTDG_OK;
}

int reserve_pinned(fftdg_ctx *c, size_t bytes) {
    if (c->staging_used) {
        hipError_t e = hipEventSynchronize(c->staging_ev);
        if (e != hipSuccess) return set_err(c, FFTDG_E_DEVICE, std::string("hipEventSynchronize: ") + hipGetErrorString(e));
        c->staging_used = false;
    }
    if (bytes <= c->pinned_n) return FFTDG_OK;
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->pinned_n = 0;
    size_t want = bytes + bytes / 4 + 4096;
    if (hipHostMalloc(&c->pinned, want, hipHostMallocDefault) != hipSuccess) {
        c->pinned = nullptr;
        (void)hipGetLastError();
        return set_err(c, FFTDG_E_NOMEM, "pinned host allocation failed");
    }
    c->pinned_n = want;
    return FFTDG_OK;
}

bool is_fin(double v) { return std::isfinite(v); }

long long isqrt_lt(long long rem) {  // largest s >= 0 with s*s < rem (rem >= 1)
    long long s = (long long)std::sqrt((double)rem);
    while (s > 0 && s * s >= rem) --s;
    while ((s + 1) * (s + 1) < rem) ++s;
    return s;
}
long long floordiv(long long a, long long b) {
    long long q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// Placement (Ligand Sampling; placement and box rule of the FFT-based BPMF
// section): rotate about the unweighted centroid by the normalised
// quaternion, shift the lowest coordinate to 2 spacings, round to the 2^-16
// lattice; box_d = ceil(max u_d) + 2.  Returns false for a zero or
// non-finite quaternion or coordinates beyond the lattice range.
bool place_one(const double *X, int n, const double *quat, double h, int32_t *U, int *box) {
    const double nq = std::sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    if (!(nq > 0.0) || !is_fin(nq)) return false;
    const double w = quat[0] / nq, x = quat[1] / nq, y = quat[2] / nq, z = quat[3] / nq;
    const double R[3][3] = {{1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                            {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
                            {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
    double c[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) c[d] += X[3 * i + d];
    for (int d = 0; d < 3; ++d) c[d] /= n;
    double mn[3] = {INFINITY, INFINITY, INFINITY};
    std::vector<double> Y(3 * (size_t)n);
    for (int i = 0; i < n; ++i) {
        const double v[3] = {X[3 * i] - c[0], X[3 * i + 1] - c[1], X[3 * i + 2] - c[2]};
        for (int d = 0; d < 3; ++d) {
            Y[3 * i + d] = R[d][0] * v[0] + R[d][1] * v[1] + R[d][2] * v[2];
            if (Y[3 * i + d] < mn[d]) mn[d] = Y[3 * i + d];
        }
    }
    long long mx[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            const double v = (Y[3 * i + d] - mn[d]) / h + 2.0;
            if (!(v < 30000.0)) return false;
            const long long L = std::llround(v * kLat);
            U[3 * i + d] = (int32_t)L;
            if (L > mx[d]) mx[d] = L;
        }
    for (int d = 0; d < 3; ++d) box[d] = (int)(-floordiv(-mx[d], 65536LL)) + 2;
    return true;
}

template <typename T>
size_t csize() {
    return 2 * sizeof(T);
}

struct Plan {
    // per configuration (plan order: batch order for a one-configuration
    // plan, else grouped by z-window class; global_cfg is the batch index)
    std::vector<CfgDev> cfg;
    std::vector<int32_t> U;        // lattice coords, [sum atoms][3]
    std::vector<int32_t> cfg_lig;  // ligand of each configuration
    // chunks: contiguous ranges of the plan order
    struct Chunk {
        int c0, c1;               // plan positions [c0, c1)
        size_t off0;              // start of this chunk's fwd_off / inv_off (c1-c0+1 entries each)
        size_t nfwd, ninv;        // forward planes, valid z translations
        size_t z0, nz;            // scanned configurations (local indices)
        int64_t ws_fwd, ws_inv;   // complex elements used
        int pp;                   // plane partial slots used
        int zhalf;                // 1: every scanned configuration's energy planes lie in [0, n_fft/2); 2: and some occupancy window is longer than n_fft/2
        // fused path
        int nitems;               // clash-test items (tz, 64-row group)
        int nitems2;              // phase-2 items (64-row slices of the undecided-row lists)
        int64_t nsurv;            // undecided-row list slots
        int64_t nruns, nfree;     // run slots, free-bit words
        int max_atoms;            // most atoms of a scanned configuration
    };
    std::vector<Chunk> chunks;
    std::vector<int32_t> fwd_off, inv_off, item_off, item2_off;
    std::vector<int32_t> zcfg;
    bool fused = false;         // planned for the fused path
    bool fused_planes = false;  // ... with energy planes written by the forward pass
    int64_t max_fwd = 0, max_inv = 0;
    int64_t max_runs = 0, max_free = 0, max_items = 0, max_chunk_cfgs = 0, max_surv = 0;
    int64_t total_pp = 0;  // plane partial slots of the whole plan (per snapshot)
};

int validate_batch(fftdg_ctx *ctx, const fftdg_batch *b) {
    if (!b) return set_err(ctx, FFTDG_E_INVALID, "batch is NULL");
    if (b->n_lig <= 0) return set_err(ctx, FFTDG_E_INVALID, "n_lig must be > 0");
    if (!b->atom_off || !b->conf_off || !b->cfg_off || !b->q || !b->sigma || !b->eps || !b->conf_xyz ||
        !b->cfg_conf || !b->cfg_quat)
        return set_err(ctx, FFTDG_E_INVALID, "batch has a NULL array");
    if (b->atom_off[0] != 0 || b->conf_off[0] != 0 || b->cfg_off[0] != 0)
        return set_err(ctx, FFTDG_E_INVALID, "offsets must start at 0");
    for (int l = 0; l < b->n_lig; ++l) {
        const int na = b->atom_off[l + 1] - b->atom_off[l];
        const int nc = b->conf_off[l + 1] - b->conf_off[l];
        const int ng = b->cfg_off[l + 1] - b->cfg_off[l];
        if (na <= 0 || na > 256) return set_err(ctx, FFTDG_E_INVALID, "ligand " + std::to_string(l) + ": atom count must be 1..256");
        if (nc <= 0) return set_err(ctx, FFTDG_E_INVALID, "ligand " + std::to_string(l) + ": no conformers");
        if (ng <= 0) return set_err(ctx, FFTDG_E_INVALID, "ligand " + std::to_string(l) + ": no configurations");
    }
    const int na = b->atom_off[b->n_lig];
    for (int i = 0; i < na; ++i) {
        if (!is_fin(b->q[i]) || !is_fin(b->sigma[i]) || !is_fin(b->eps[i]) || b->sigma[i] <= 0 || b->eps[i] < 0)
            return set_err(ctx, FFTDG_E_INVALID, "atom " + std::to_string(i) + ": non-finite or out-of-range parameter");
    }
    size_t rows = 0;
    for (int l = 0; l < b->n_lig; ++l)
        rows += (size_t)(b->conf_off[l + 1] - b->conf_off[l]) * (b->atom_off[l + 1] - b->atom_off[l]);
    for (size_t i = 0; i < 3 * rows; ++i)
        if (!is_fin(b->conf_xyz[i])) return set_err(ctx, FFTDG_E_INVALID, "non-finite conformer coordinate");
    const int ncfg = b->cfg_off[b->n_lig];
    for (int l = 0; l < b->n_lig; ++l) {
        const int nc = b->conf_off[l + 1] - b->conf_off[l];
        for (int c = b->cfg_off[l]; c < b->cfg_off[l + 1]; ++c)
            if (b->cfg_conf[c] < 0 || b->cfg_conf[c] >= nc)
                return set_err(ctx, FFTDG_E_INVALID, "configuration " + std::to_string(c) + ": conformer index out of range");
    }
    for (int i = 0; i < 4 * ncfg; ++i)
        if (!is_fin(b->cfg_quat[i])) return set_err(ctx, FFTDG_E_INVALID, "non-finite quaternion");
    return FFTDG_OK;
}

double occ_threshold(const fftdg_grid_desc &g, double sigma) {
    const double rho = g.occ_f * std::pow(2.0, -1.0 / 6.0) * sigma / g.h;
    return std::ceil(rho * rho * 4294967296.0);
}

// Place every configuration and build the chunked work lists.
int build_plan(fftdg_ctx *ctx, const fftdg_batch *b, bool only_one, int one_cfg, Plan &P) {
    const fftdg_grid_desc &g = ctx->g;
    const int N = g.n_fft, n_rec = g.n_rec;
    const bool occ = g.clash_mode == FFTDG_OCC;
    const int ncfg = b->cfg_off[b->n_lig];
    P.cfg.assign(ncfg, CfgDev{});
    P.cfg_lig.assign(ncfg, 0);
    // atom / conformer-row offsets
    std::vector<size_t> xyz_row(b->n_lig);
    size_t rows = 0;
    for (int l = 0; l < b->n_lig; ++l) {
        xyz_row[l] = rows;
        rows += (size_t)(b->conf_off[l + 1] - b->conf_off[l]) * (b->atom_off[l + 1] - b->atom_off[l]);
    }
    std::vector<size_t> ubase(ncfg + 1, 0);
    for (int l = 0; l < b->n_lig; ++l)
        for (int c = b->cfg_off[l]; c < b->cfg_off[l + 1]; ++c) {
            P.cfg_lig[c] = l;
            ubase[c + 1] = b->atom_off[l + 1] - b->atom_off[l];
        }
    for (int c = 0; c < ncfg; ++c) ubase[c + 1] += ubase[c];
    P.U.assign(3 * ubase[ncfg], 0);
    std::vector<double> thr(b->atom_off[b->n_lig]);
    std::vector<long long> reach(thr.size());
    for (size_t i = 0; i < thr.size(); ++i) {
        thr[i] = occ ? occ_threshold(g, b->sigma[i]) : 0.0;
        reach[i] = occ && thr[i] >= 1.0 ? isqrt_lt((long long)thr[i]) : -1;
    }
    // the fused path's clash table keeps Dil<N>::M rows and points past each
    // end of the domain: the occupancy balls must reach no further past the
    // box (the box starts 2 points after the lowest atom and ends 2 after
    // the highest); wider balls take the plane path
    long long smax = -1;
    for (long long s : reach) smax = std::max(smax, s);
    const long long reach_pts = smax < 0 ? 0 : (smax + 65535) / 65536;
    const bool fz = ctx->fused != 0 && ctx->fs != nullptr && (!occ || reach_pts <= ctx->fs->margin);
    const bool fzp = fz && ctx->fused == 1;
    P.fused = fz;
    P.fused_planes = fzp;
    // fused path: slots for a configuration's occupancy runs.  An atom's ball
    // meets at most r = 2 floor(reach / 2^16) + 2 rows and columns of each
    // axis; runs are written in pieces of at most RUN_MAX points, and the pieces
    // of a row's union never outnumber those of the balls meeting it, so per
    // atom (1 chord + r^2 rows) x ceil(r / RUN_MAX) pieces bound the count
    std::vector<int64_t> run_cap(b->n_lig, 0);
    if (fz && occ)
        for (int l = 0; l < b->n_lig; ++l) {
            int64_t cap = 0;
            for (int i = b->atom_off[l]; i < b->atom_off[l + 1]; ++i)
                if (reach[i] >= 0) {
                    const int64_t r = 2 * (reach[i] >> 16) + 2;
                    cap += (1 + r * r) * ((r + RUN_MAX - 1) / RUN_MAX);
                }
            run_cap[l] = cap;
        }
    std::atomic<int> bad(-1), bad_geom(-1);
    auto work = [&](int c_begin, int c_end) {
        for (int c = c_begin; c < c_end; ++c) {
            const int l = P.cfg_lig[c];
            const int na = b->atom_off[l + 1] - b->atom_off[l];
            const double *X = b->conf_xyz + 3 * (xyz_row[l] + (size_t)b->cfg_conf[c] * na);
            int32_t *U = P.U.data() + 3 * ubase[c];
            int box[3];
            CfgDev &d = P.cfg[c];
            d.u_base = (int32_t)ubase[c];
            d.atom_base = b->atom_off[l];
            d.n_atoms = na;
            d.global_cfg = c;
            if (!place_one(X, na, b->cfg_quat + 4 * c, g.h, U, box)) {
                int exp = -1;
                bad.compare_exchange_strong(exp, c);
                continue;
            }
            long long nv = 1;
            for (int k = 0; k < 3; ++k) {
                d.V[k] = std::max(n_rec - box[k], 0);
                nv *= d.V[k];
            }
            d.n_valid = (int32_t)nv;
            const bool sel = (!only_one && (!b->cfg_select || b->cfg_select[c])) || (only_one && c == one_cfg);
            d.scanned = (sel && nv > 0) ? 1 : 0;
            // energy channel planes and rows (trilinear corners floor(u), floor(u)+1)
            int zlo = 1 << 30, zhi = -(1 << 30), ylo = 1 << 30, yhi = -(1 << 30);
            long long ozlo = 1LL << 40, ozhi = -(1LL << 40), oylo = 1LL << 40, oyhi = -(1LL << 40);
            long long oxlo = 1LL << 40, oxhi = -(1LL << 40);
            for (int i = 0; i < na; ++i) {
                const int az = U[3 * i + 2] >> 16, ay = U[3 * i + 1] >> 16;
                zlo = std::min(zlo, az);
                zhi = std::max(zhi, az + 1);
                ylo = std::min(ylo, ay);
                yhi = std::max(yhi, ay + 1);
                if (occ) {
                    const long long s = reach[b->atom_off[l] + i];
                    if (s < 0) continue;
                    ozlo = std::min(ozlo, -floordiv(-(U[3 * i + 2] - s), 65536LL));
                    ozhi = std::max(ozhi, floordiv(U[3 * i + 2] + s, 65536LL));
                    oylo = std::min(oylo, -floordiv(-(U[3 * i + 1] - s), 65536LL));
                    oyhi = std::max(oyhi, floordiv(U[3 * i + 1] + s, 65536LL));
                    oxlo = std::min(oxlo, -floordiv(-(U[3 * i] - s), 65536LL));
                    oxhi = std::max(oxhi, floordiv(U[3 * i] + s, 65536LL));
                    if (2 * s / 65536 + 2 >= N) {
                        int exp = -1;
                        bad_geom.compare_exchange_strong(exp, c);
                    }
                }
            }
            d.ze0 = zlo;
            d.Le = zhi - zlo + 1;
            d.ye0 = ylo;
            d.Lye = yhi - ylo + 1;
            if (occ && ozhi >= ozlo) {
                d.zo0 = (int32_t)ozlo;
                d.Lo = (int32_t)(ozhi - ozlo + 1);
                d.yo0 = (int32_t)oylo;
                d.Lyo = (int32_t)(oyhi - oylo + 1);
                d.xo0 = (int32_t)oxlo;
                d.Lxo = (int32_t)(oxhi - oxlo + 1);
            } else {
                d.zo0 = 0;
                d.Lo = 0;
                d.yo0 = 0;
                d.Lyo = 0;
                d.xo0 = 0;
                d.Lxo = 0;
            }
            if (d.scanned && (d.Le > N || d.Lye > N || d.Lo > N || d.Lyo > N || d.Lxo > N)) {
                int exp = -1;
                bad_geom.compare_exchange_strong(exp, c);
            }
        }
    };
    const int nthr = std::max(1, std::min<int>((int)std::thread::hardware_concurrency(), ncfg / 64 + 1));
    if (nthr <= 1) {
        work(0, ncfg);
    } else {
        std::vector<std::thread> th;
        const int per = (ncfg + nthr - 1) / nthr;
        for (int t = 0; t < nthr; ++t) {
            const int a = t * per, e = std::min(ncfg, a + per);
            if (a < e) th.emplace_back(work, a, e);
        }
        for (auto &t : th) t.join();
    }
    if (bad.load() >= 0)
        return set_err(ctx, FFTDG_E_INVALID, "configuration " + std::to_string(bad.load()) +
                                                 ": zero or non-finite quaternion, or ligand far larger than the grid");
    if (bad_geom.load() >= 0)
        return set_err(ctx, FFTDG_E_INVALID, "configuration " + std::to_string(bad_geom.load()) +
                                                 ": occupancy extent of the ligand exceeds n_fft");
    // every ligand needs at least one box-valid configuration
    for (int l = 0; l < b->n_lig && !only_one; ++l) {
        bool any = false;
        for (int c = b->cfg_off[l]; c < b->cfg_off[l + 1] && !any; ++c) any = P.cfg[c].n_valid > 0;
        if (!any)
            return set_err(ctx, FFTDG_E_NOVALID, "ligand " + std::to_string(l) +
                                                     " has no box-valid translation in any configuration");
    }
    // Plan order.  A chunk gets the pruned z transforms only if every one of
    // its configurations has its energy planes in [0, n_fft/2), and the
    // cheaper of those two instantiations only if no occupancy window is
    // longer than n_fft/2, so configurations are grouped by these two tests
    // (stable: batch order within a group; unscanned ones last).  Partials
    // are still written at each configuration's batch index (global_cfg).
    if (!only_one) {
        auto group = [&](const CfgDev &d) {
            if (!d.scanned) return 3;
            if (fz) return d.Le <= N / 2 ? 0 : 1;  // the fused z kernel loads the window from plane 0
            if (!(d.ze0 >= 0 && d.ze0 + d.Le <= N / 2)) return 2;
            return (occ && d.Lo > N / 2) ? 1 : 0;
        };
        std::vector<int> ord(ncfg);
        for (int i = 0; i < ncfg; ++i) ord[i] = i;
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return group(P.cfg[x]) < group(P.cfg[y]); });
        std::vector<CfgDev> pc(ncfg);
        for (int i = 0; i < ncfg; ++i) pc[i] = P.cfg[ord[i]];
        P.cfg.swap(pc);
    }
    // chunks
    const int64_t NP = ctx->ks->np;
    const int nout = occ ? 2 : 1;
    const int64_t limit_c = (int64_t)(ctx->ws_limit / (size_t)ctx->ks->cbytes);
    int c = 0;
    int64_t ppt = 0;  // plane partial slots of the chunks before this one
    while (c < ncfg && fz) {
        Plan::Chunk ch{};
        ch.c0 = c;
        ch.off0 = P.fwd_off.size();
        ch.z0 = P.zcfg.size();
        int32_t ni = 0, nit = 0, nit2 = 0, nf = 0;
        int nscan = 0, ma = 0;
        int64_t wi = 0, wf = 0, nr = 0, nfw = 0, nsv = 0;
        int pp = 0;
        bool zhalf = true;
        while (c < ncfg) {
            CfgDev &d = P.cfg[c];
            const int local = c - ch.c0;
            if (d.scanned) {
                const int64_t iv = (int64_t)d.V[2] * NP;
                const int64_t f = fzp ? (int64_t)3 * d.Le * NP : 0;
                if (nscan > 0 && (nscan >= ctx->chunk_cfgs || wi + iv + wf + f > limit_c)) break;
                const int ny = (d.V[1] + 63) / 64, W = (d.V[0] + 31) / 32;
                d.off_fwd = wf;
                d.off_inv = wi;
                d.occ_slot0 = 0;
                d.pp_base = (int32_t)(ppt + pp);
                d.run_off = (int32_t)nr;
                d.run_cap = occ ? (int32_t)run_cap[P.cfg_lig[d.global_cfg]] : 0;
                d.free_off = (int32_t)nfw;
                d.item_base = nit;
                d.surv_off = (int32_t)nsv;
                P.fwd_off.push_back(nf);
                P.inv_off.push_back(ni);
                P.item_off.push_back(nit);
                P.item2_off.push_back(nit2);
                ni += d.V[2];
                if (fzp) {
                    nf += d.Le;  // one forward item per energy plane (all three channels)
                    wf += f;
                }
                if (occ) {
                    nit += d.V[2] * ny;
                    nit2 += (d.V[2] * d.V[1] + 63) / 64;
                    nfw += (int64_t)d.V[2] * d.V[1] * W;
                    nsv += (int64_t)d.V[2] * d.V[1];
                    nr += d.run_cap;
                }
                P.zcfg.push_back(local);
                zhalf = zhalf && d.Le <= N / 2;
                ma = std::max(ma, d.n_atoms);
                wi += iv;
                pp += d.V[2];
                ++nscan;
            } else {
                d.off_fwd = d.off_inv = 0;
                d.pp_base = (int32_t)(ppt + pp);
                d.occ_slot0 = 0;
                d.run_off = d.run_cap = d.free_off = d.surv_off = 0;
                d.item_base = nit;
                P.fwd_off.push_back(nf);
                P.inv_off.push_back(ni);
                P.item_off.push_back(nit);
                P.item2_off.push_back(nit2);
            }
            ++c;
        }
        ch.c1 = c;
        P.fwd_off.push_back(nf);
        P.inv_off.push_back(ni);
        P.item_off.push_back(nit);
        P.item2_off.push_back(nit2);
        ch.nfwd = nf;
        ch.ninv = ni;
        ch.nz = P.zcfg.size() - ch.z0;
        ch.ws_fwd = wf;
        ch.ws_inv = wi;
        ch.pp = pp;
        ch.zhalf = zhalf ? 1 : 0;
        ch.nitems = nit;
        ch.nitems2 = nit2;
        ch.nsurv = nsv;
        ch.nruns = nr;
        ch.nfree = nfw;
        ch.max_atoms = ma;
        if (nr > INT32_MAX || nfw > INT32_MAX || nsv > INT32_MAX)
            return set_err(ctx, FFTDG_E_INVALID, "scan: clash-test tables of one chunk exceed 2^31 entries");
        P.max_inv = std::max(P.max_inv, wi);
        P.max_fwd = std::max(P.max_fwd, wf);
        P.max_runs = std::max(P.max_runs, nr);
        P.max_free = std::max(P.max_free, nfw);
        P.max_items = std::max<int64_t>(P.max_items, nit);
        P.max_surv = std::max(P.max_surv, nsv);
        P.max_chunk_cfgs = std::max<int64_t>(P.max_chunk_cfgs, ch.c1 - ch.c0);
        ppt += pp;
        if (ppt > INT32_MAX) return set_err(ctx, FFTDG_E_INVALID, "scan: more than 2^31 valid z-translations in one batch");
        P.total_pp = ppt;
        P.chunks.push_back(ch);
    }
    while (c < ncfg) {
        Plan::Chunk ch{};
        ch.c0 = c;
        ch.off0 = P.fwd_off.size();
        ch.z0 = P.zcfg.size();
        int32_t nf = 0, ni = 0;
        int nscan = 0;
        int64_t wf = 0, wi = 0;
        int pp = 0;
        bool zhalf = true, olong = false;
        while (c < ncfg) {
            CfgDev &d = P.cfg[c];
            if (d.scanned) {
                const int e_planes = ctx->edirect == 1 ? 0 : 3 * d.Le;
                const int e_items = ctx->edirect == 2 ? d.Le : e_planes;
                d.occ_slot0 = e_planes;
                const int64_t f = (int64_t)(e_planes + (occ ? d.Lo : 0)) * NP;
                const int64_t iv = (int64_t)nout * d.V[2] * NP;
                if (nscan > 0 && (nscan >= ctx->chunk_cfgs || wf + f + wi + iv > limit_c)) break;
                d.off_fwd = wf;
                d.off_inv = wi;
                d.pp_base = (int32_t)(ppt + pp);
                const int local = c - ch.c0;
                P.fwd_off.push_back(nf);
                P.inv_off.push_back(ni);
                P.item_off.push_back(0);
                P.item2_off.push_back(0);
                nf += e_items + (occ ? d.Lo : 0);
                ni += d.V[2];
                P.zcfg.push_back(local);
                zhalf = zhalf && d.ze0 >= 0 && d.ze0 + d.Le <= ctx->g.n_fft / 2;
                olong = olong || (occ && d.Lo > ctx->g.n_fft / 2);
                wf += f;
                wi += iv;
                pp += d.V[2];
                ++nscan;
            } else {
                d.off_fwd = d.off_inv = 0;
                d.pp_base = (int32_t)(ppt + pp);
                d.occ_slot0 = 0;
                P.fwd_off.push_back(nf);
                P.inv_off.push_back(ni);
                P.item_off.push_back(0);
                P.item2_off.push_back(0);
            }
            ++c;
        }
        ch.c1 = c;
        P.fwd_off.push_back(nf);
        P.inv_off.push_back(ni);
        P.item_off.push_back(0);
        P.item2_off.push_back(0);
        ch.nfwd = nf;
        ch.ninv = ni;
        ch.nz = P.zcfg.size() - ch.z0;
        ch.ws_fwd = wf;
        ch.ws_inv = wi;
        ch.pp = pp;
        ch.zhalf = zhalf ? (olong ? 2 : 1) : 0;
        P.max_fwd = std::max(P.max_fwd, wf);
        P.max_inv = std::max(P.max_inv, wi);
        ppt += pp;
        if (ppt > INT32_MAX) return set_err(ctx, FFTDG_E_INVALID, "scan: more than 2^31 valid z-translations in one batch");
        P.total_pp = ppt;
        P.chunks.push_back(ch);
    }
    return FFTDG_OK;
}

template <typename T>
void fill_gamma(const fftdg_batch *b, T *gam) {
    const int na = b->atom_off[b->n_lig];
    for (int i = 0; i < na; ++i) {
        const double s3 = b->sigma[i] * b->sigma[i] * b->sigma[i];
        const double se = std::sqrt(b->eps[i]);
        gam[3 * i + 0] = (T)b->q[i];
        gam[3 * i + 1] = (T)(se * s3 * s3);
        gam[3 * i + 2] = (T)(-2.0 * se * s3);
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Upload the plan and run it; psi/clash export for the energy-grid call.
int run_plan(fftdg_ctx *ctx, const fftdg_batch *b, const Plan &P, double T_K, fftdg_partial *out,
             int snap_only, void *psi_out, uint8_t *clash_out) {
    const fftdg_grid_desc &g = ctx->g;
    const bool occ = g.clash_mode == FFTDG_OCC;
    const int ncfg = b->cfg_off[b->n_lig];
    const int na = b->atom_off[b->n_lig];
    const size_t tsz = g.precision == FFTDG_F32 ? sizeof(float) : sizeof(double);
    // table layout
    const size_t o_cfg = 0;
    const size_t o_u = align256(o_cfg + sizeof(CfgDev) * P.cfg.size());
    const size_t o_fwd = align256(o_u + sizeof(int32_t) * P.U.size());
    const size_t o_inv = align256(o_fwd + sizeof(int32_t) * P.fwd_off.size());
    const size_t o_item = align256(o_inv + sizeof(int32_t) * P.inv_off.size());
    const size_t o_item2 = align256(o_item + sizeof(int32_t) * P.item_off.size());
    const size_t o_z = align256(o_item2 + sizeof(int32_t) * P.item2_off.size());
    const size_t o_gam = align256(o_z + sizeof(int32_t) * P.zcfg.size());
    const size_t o_thr = align256(o_gam + tsz * 3 * na);
    const size_t total = align256(o_thr + sizeof(double) * na);
    int rc;
    if ((rc = reserve_pinned(ctx, total))) return rc;
    if ((rc = reserve(ctx, ctx->tables, total))) return rc;
    char *h = (char *)ctx->pinned;
    std::memcpy(h + o_cfg, P.cfg.data(), sizeof(CfgDev) * P.cfg.size());
    std::memcpy(h + o_u, P.U.data(), sizeof(int32_t) * P.U.size());
    std::memcpy(h + o_fwd, P.fwd_off.data(), sizeof(int32_t) * P.fwd_off.size());
    std::memcpy(h + o_inv, P.inv_off.data(), sizeof(int32_t) * P.inv_off.size());
    std::memcpy(h + o_item, P.item_off.data(), sizeof(int32_t) * P.item_off.size());
    std::memcpy(h + o_item2, P.item2_off.data(), sizeof(int32_t) * P.item2_off.size());
    if (!P.zcfg.empty()) std::memcpy(h + o_z, P.zcfg.data(), sizeof(int32_t) * P.zcfg.size());
    if (g.precision == FFTDG_F32)
        fill_gamma<float>(b, (float *)(h + o_gam));
    else
        fill_gamma<double>(b, (double *)(h + o_gam));
    double *thr = (double *)(h + o_thr);
    for (int i = 0; i < na; ++i) thr[i] = occ ? occ_threshold(g, b->sigma[i]) : 0.0;
    const size_t cb = (size_t)ctx->ks->cbytes;
    if ((!P.fused || P.fused_planes) && (rc = reserve(ctx, ctx->ws_fwd, cb * (size_t)std::max<int64_t>(P.max_fwd, 1))))
        return rc;
    int64_t max_nz_atoms = 1;
    if (P.fused) {
        int64_t nzmax = 1;
        for (const Plan::Chunk &ch : P.chunks) {
            nzmax = std::max<int64_t>(nzmax, (int64_t)ch.nz);
            max_nz_atoms = std::max<int64_t>(max_nz_atoms, (int64_t)ch.nz * std::max(ch.max_atoms, 1));
        }
        if ((rc = reserve(ctx, ctx->zat, ctx->fs->zat_bytes * (size_t)max_nz_atoms))) return rc;
        if ((rc = reserve(ctx, ctx->zbt, sizeof(int32_t) * (size_t)nzmax * (g.n_fft + 2)))) return rc;
    }
    // second stream.  Fused path, OCC: the clash test of the next (chunk,
    // snapshot) item runs on the side stream beside the z pass and inverse of
    // the current one; its results (free bits, live flags, undecided-row
    // lists) alternate between two buffer sets.  Plane path: the inverse xy
    // of one z pass runs on the side stream beside the next z pass; the
    // inverse planes alternate between two workspace sets.
    const bool overlap = (P.fused ? occ : true) && ctx->clash_stream && !ctx->prof && !psi_out && !clash_out;
    const int nsets = overlap ? 2 : 1;
    const size_t e_free = (size_t)std::max<int64_t>(P.max_free, 1), e_items = (size_t)std::max<int64_t>(P.max_items, 1);
    const size_t e_surv = (size_t)std::max<int64_t>(P.max_surv, 1), e_cfgs = (size_t)std::max<int64_t>(P.max_chunk_cfgs, 1);
    if (P.fused && occ) {
        if ((rc = reserve(ctx, ctx->runs, 2 * sizeof(uint32_t) * (size_t)std::max<int64_t>(P.max_runs, 1)))) return rc;
        if ((rc = reserve(ctx, ctx->run_cnt, sizeof(int32_t) * e_cfgs))) return rc;
        if ((rc = reserve(ctx, ctx->fbits, sizeof(uint32_t) * e_free * nsets))) return rc;
        if ((rc = reserve(ctx, ctx->lives, e_items * nsets))) return rc;
        if ((rc = reserve(ctx, ctx->surv, sizeof(uint32_t) * e_surv * nsets))) return rc;
        if ((rc = reserve(ctx, ctx->scnt, sizeof(int32_t) * e_cfgs * nsets))) return rc;
    }
    if (overlap && !ctx->side) {
        // the events first: the stream is set only once all of them exist,
        // so a failed attempt leaves nothing half made for the next call
        for (hipEvent_t *e : {&ctx->ev_fork, &ctx->ev_join, &ctx->ev_side[0], &ctx->ev_side[1], &ctx->ev_main[0],
                              &ctx->ev_main[1]})
            if (!*e) HIPCHK(ctx, hipEventCreateWithFlags(e, hipEventDisableTiming));
        hipStream_t side = nullptr;
        HIPCHK(ctx, hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
        ctx->side = side;
    }
    // snapshots whose inverse planes share the workspace: the z kernel keeps
    // a configuration's forward spectra in registers across the group
    const int s_begin = snap_only >= 0 ? snap_only : 0;
    const int s_end = snap_only >= 0 ? snap_only + 1 : ctx->n_snap;
    const int64_t inv1 = std::max<int64_t>(P.max_inv, 1);
    const int64_t room = (int64_t)(ctx->ws_limit / cb) - P.max_fwd;
    const int grp = P.fused ? 1
                            : (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)(s_end - s_begin), room / inv1,
                                                                           (int64_t)ctx->snap_group}));
    const size_t inv_set = cb * (size_t)inv1 * grp;  // bytes of one workspace set of inverse planes
    if ((rc = reserve(ctx, ctx->ws_inv, inv_set * (overlap && !P.fused ? 2 : 1)))) return rc;
    // plane partials of the whole scan, one region per snapshot, merged into
    // configuration partials once per snapshot after the last chunk
    const size_t pp_snap = (size_t)ctx->ks->ppbytes * (size_t)std::max<int64_t>(P.total_pp, 1);
    if ((rc = reserve(ctx, ctx->pp, pp_snap * (size_t)(s_end - s_begin)))) return rc;
    HIPCHK(ctx, hipMemcpyAsync(ctx->tables.p, h, total, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipEventRecord(ctx->staging_ev, ctx->stream));
    ctx->staging_used = true;
    char *d = (char *)ctx->tables.p;
    const CfgDev *dcfg = (const CfgDev *)(d + o_cfg);
    const int32_t *du = (const int32_t *)(d + o_u);
    const int32_t *dfwd = (const int32_t *)(d + o_fwd);
    const int32_t *dinv = (const int32_t *)(d + o_inv);
    const int32_t *ditem = (const int32_t *)(d + o_item);
    const int32_t *ditem2 = (const int32_t *)(d + o_item2);
    const int32_t *dz = (const int32_t *)(d + o_z);
    const void *dgam = (const void *)(d + o_gam);
    const double *dthr = (const double *)(d + o_thr);
    const double beta = 1.0 / (kR * T_K);
    const size_t spec_per_snap = (size_t)ctx->n_ch * g.n_fft * ctx->ks->np * cb;
    const KernelSet *ks = ctx->ks;
    const double pb = (double)ctx->ks->ppbytes;
    // Every launch of the scan, issued on stream `st`.  The kernels read all
    // per-chunk data from the device tables, so a captured sequence stays
    // valid for any later scan with the same signature (launch shapes,
    // table layout, buffers, temperature).
    const bool exporting = psi_out != nullptr || clash_out != nullptr;
    // Fused path: ligand occupancy runs once per chunk; per snapshot the
    // clash test on bits, the z pass (energy channels, inputs from per-atom
    // factors) and the inverse xy on the planes holding a clash-free
    // translation.
    auto launch_fused = [&](hipStream_t st) -> int {
    const FusedSet *fs = ctx->fs;
    uint32_t *runs = (uint32_t *)ctx->runs.p;
    int32_t *rcnt = (int32_t *)ctx->run_cnt.p;
    const double b_spec3 = 3.0 * (double)g.n_fft * ctx->ks->np * cb;
    // buffer set p of the clash results
    auto fb_of = [&](int p) { return (uint32_t *)ctx->fbits.p + (size_t)p * e_free; };
    auto lv_of = [&](int p) { return (uint8_t *)ctx->lives.p + (size_t)p * e_items; };
    auto surv_of = [&](int p) { return (uint32_t *)ctx->surv.p + (size_t)p * e_surv; };
    auto scnt_of = [&](int p) { return (int32_t *)ctx->scnt.p + (size_t)p * e_cfgs; };
    // stream of the occupancy runs and the clash test; with the overlap it
    // starts after the work already ordered on `st` (the table upload)
    hipStream_t sc = st;
    if (overlap) {
        sc = ctx->side;
        HIPCHK(ctx, hipEventRecord(ctx->ev_fork, st));
        HIPCHK(ctx, hipStreamWaitEvent(sc, ctx->ev_fork, 0));
    }
    int item = 0;
    for (const Plan::Chunk &ch : P.chunks) {
        const CfgDev *ccfg = dcfg + ch.c0;
        const int nloc = ch.c1 - ch.c0;
        // the runs of this chunk follow the previous chunk's clash tests on `sc`
        if (occ)
            HIPCHK(ctx, timed(ctx, FFTDG_K_RUNS, 8.0 * (double)ch.nruns, [&] {
                       return fs->lig_runs(sc, ccfg, dz + ch.z0, (int)ch.nz, du, dthr, runs, rcnt);
                   }));
        if (P.fused_planes)
            HIPCHK(ctx, timed(ctx, FFTDG_K_FWD, (double)ch.ws_fwd * cb, [&] {
                       return ks->fwd(st, true, dfwd + ch.off0, nloc, (int)ch.nfwd, ccfg, du, dgam, dthr, ctx->tw.p,
                                      ctx->ws_fwd.p);
                   }));
        else
            HIPCHK(ctx, timed(ctx, FFTDG_K_RUNS, (double)ch.nz * ch.max_atoms * fs->zat_bytes, [&] {
                       return fs->zprep(st, ccfg, dz + ch.z0, (int)ch.nz, std::max(ch.max_atoms, 1), du, dgam,
                                        ctx->zat.p, (int32_t *)ctx->zbt.p);
                   }));
        for (int s = s_begin; s < s_end; ++s, ++item) {
            const int p = overlap ? (item & 1) : 0;
            uint32_t *fb = fb_of(p);
            uint8_t *lv = lv_of(p);
            if (occ) {
                // set p was last read by the inverse of item - 2
                if (overlap && item >= 2) HIPCHK(ctx, hipStreamWaitEvent(sc, ctx->ev_main[p], 0));
                const uint32_t *dil = (const uint32_t *)ctx->dil.p + (size_t)s * (size_t)fs->dil_words;
                HIPCHK(ctx, timed(ctx, FFTDG_K_CLASH, 4.0 * (double)ch.nfree + (double)ch.nitems, [&] {
                           return fs->clash(sc, ditem + ch.off0, ditem2 + ch.off0, nloc, ch.nitems, ch.nitems2, ccfg,
                                            runs, rcnt, dil, fb, lv, surv_of(p), scnt_of(p));
                       }));
                if (overlap) {
                    HIPCHK(ctx, hipEventRecord(ctx->ev_side[p], sc));
                    HIPCHK(ctx, hipStreamWaitEvent(st, ctx->ev_side[p], 0));
                }
            }
            const char *rs = (const char *)ctx->rspec.p + spec_per_snap * s;
            // planes written are counted on the device (those the inverse reads)
            HIPCHK(ctx, timed(ctx, FFTDG_K_ZPROD, b_spec3 + (P.fused_planes ? (double)ch.ws_fwd * cb : 0.0), [&] {
                       if (P.fused_planes)
                           return fs->zplanes(st, ch.zhalf != 0, occ && !exporting, ccfg, dz + ch.z0, (int)ch.nz,
                                              ctx->ws_fwd.p, rs, ctx->tw.p, ctx->ws_inv.p, lv);
                       return fs->zpass(st, ch.zhalf != 0, occ && !exporting, ccfg, dz + ch.z0, (int)ch.nz,
                                        std::max(ch.max_atoms, 1), ctx->zat.p, (const int32_t *)ctx->zbt.p, rs,
                                        ctx->tw.p, ctx->ws_inv.p, lv);
                   }));
            void *pp_s = (char *)ctx->pp.p + pp_snap * (size_t)(s - s_begin);
            HIPCHK(ctx, timed(ctx, FFTDG_K_INV, pb * ch.pp, [&] {
                       return fs->inv(st, occ, dinv + ch.off0, nloc, (int)ch.ninv, ccfg, ctx->ws_inv.p, beta,
                                      ctx->tw.p, fb, lv, pp_s, psi_out, clash_out,
                                      ctx->prof ? (unsigned int *)ctx->prof_cnt.p : nullptr);
                   }));
            if (overlap) HIPCHK(ctx, hipEventRecord(ctx->ev_main[p], st));
            if (ctx->prof) ctx->prof_fused = true;
        }
    }
    if (overlap) {  // join: later work on `st` sees the side stream's work done
        HIPCHK(ctx, hipEventRecord(ctx->ev_join, sc));
        HIPCHK(ctx, hipStreamWaitEvent(st, ctx->ev_join, 0));
    }
    if (out)
        for (int s = s_begin; s < s_end; ++s) {
            const void *pp_s = (const char *)ctx->pp.p + pp_snap * (size_t)(s - s_begin);
            HIPCHK(ctx, timed(ctx, FFTDG_K_MERGE, pb * (double)P.total_pp + sizeof(fftdg_partial) * (double)ncfg, [&] {
                       return ks->merge(st, dcfg, ncfg, pp_s, out + (size_t)s * ncfg);
                   }));
        }
    return FFTDG_OK;
    };
    auto launch_all = [&](hipStream_t st) -> int {
    if (P.fused) return launch_fused(st);
    hipStream_t si = st;  // stream of the inverse xy
    if (overlap) {
        si = ctx->side;
        HIPCHK(ctx, hipEventRecord(ctx->ev_fork, st));
        HIPCHK(ctx, hipStreamWaitEvent(si, ctx->ev_fork, 0));
    }
    int zpass = 0;
    for (const Plan::Chunk &ch : P.chunks) {
        const CfgDev *ccfg = dcfg + ch.c0;
        // algorithmic bytes: forward planes written once (fwd), read once and
        // inverse planes written once plus one read of the receptor spectra
        // (z product), inverse planes read once (inverse xy), plane partials
        // read and configuration partials written (merge)
        const double b_fwd = (double)ch.ws_fwd * cb;
        const double b_inv = (double)ch.ws_inv * cb;
        HIPCHK(ctx, timed(ctx, FFTDG_K_FWD, b_fwd, [&] {
                   return ks->fwd(st, ctx->edirect == 2, dfwd + ch.off0, ch.c1 - ch.c0, (int)ch.nfwd, ccfg, du, dgam, dthr,
                                  ctx->tw.p, ctx->ws_fwd.p);
               }));
        for (int s0 = s_begin; s0 < s_end; s0 += grp) {
          const int ng = std::min(grp, s_end - s0);
          const char *rs = (const char *)ctx->rspec.p + spec_per_snap * s0;
          const int p = overlap ? (zpass & 1) : 0;
          char *wsi = (char *)ctx->ws_inv.p + (size_t)p * inv_set;
          // set p was last read by the inverse of z pass zpass - 2
          if (overlap && zpass >= 2) HIPCHK(ctx, hipStreamWaitEvent(st, ctx->ev_side[p], 0));
          HIPCHK(ctx, timed(ctx, FFTDG_K_ZPROD, b_fwd + ng * (b_inv + (double)spec_per_snap), [&] {
                     return ks->zprod(st, occ, ctx->edirect == 1, ch.zhalf, ccfg, dz + ch.z0, (int)ch.nz, ctx->ws_fwd.p, rs,
                                      ctx->tw.p, wsi, du, dgam, ng, (int64_t)(spec_per_snap / cb),
                                      (int64_t)ch.ws_inv);
                 }));
          if (overlap) {
              HIPCHK(ctx, hipEventRecord(ctx->ev_main[p], st));
              HIPCHK(ctx, hipStreamWaitEvent(si, ctx->ev_main[p], 0));
          }
          for (int s = s0; s < s0 + ng; ++s) {
            void *wsi_s = wsi + (size_t)(s - s0) * (size_t)ch.ws_inv * cb;
            // inverse xy: occupancy planes always, energy planes only where the
            // plane has a clash-free translation (counted on the device)
            const double b_inv_fixed = (occ ? 0.5 * b_inv : 0.0) + pb * ch.pp;
            void *pp_s = (char *)ctx->pp.p + pp_snap * (size_t)(s - s_begin);
            HIPCHK(ctx, timed(ctx, FFTDG_K_INV, b_inv_fixed, [&] {
                       return ks->inv(si, occ, dinv + ch.off0, ch.c1 - ch.c0, (int)ch.ninv, ccfg, wsi_s, beta,
                                      ctx->tw.p, pp_s, psi_out, clash_out,
                                      ctx->prof ? (unsigned int *)ctx->prof_cnt.p : nullptr);
                   }));
          }
          if (overlap) HIPCHK(ctx, hipEventRecord(ctx->ev_side[p], si));
          ++zpass;
        }
    }
    if (overlap) {  // join: later work on `st` sees the side stream's work done
        HIPCHK(ctx, hipEventRecord(ctx->ev_join, si));
        HIPCHK(ctx, hipStreamWaitEvent(st, ctx->ev_join, 0));
    }
    if (out)
        for (int s = s_begin; s < s_end; ++s) {
            const void *pp_s = (const char *)ctx->pp.p + pp_snap * (size_t)(s - s_begin);
            HIPCHK(ctx, timed(ctx, FFTDG_K_MERGE, pb * (double)P.total_pp + sizeof(fftdg_partial) * (double)ncfg, [&] {
                       return ks->merge(st, dcfg, ncfg, pp_s, out + (size_t)s * ncfg);
                   }));
        }
    return FFTDG_OK;
    };
    const bool graph_ok = ctx->use_graph && !ctx->prof && !psi_out && !clash_out && out;
    if (!graph_ok) return launch_all(ctx->stream);
    std::vector<int64_t> sig = {(int64_t)(intptr_t)ks, occ, ctx->edirect, grp, s_begin, s_end, P.fused, P.fused_planes,
                                overlap, (int64_t)(intptr_t)ctx->side,
                                (int64_t)(intptr_t)ctx->runs.p, (int64_t)(intptr_t)ctx->run_cnt.p,
                                (int64_t)(intptr_t)ctx->fbits.p, (int64_t)(intptr_t)ctx->lives.p,
                                (int64_t)(intptr_t)ctx->dil.p, (int64_t)o_item, (int64_t)(intptr_t)ctx->zat.p,
                                (int64_t)(intptr_t)ctx->zbt.p, (int64_t)(intptr_t)ctx->surv.p,
                                (int64_t)(intptr_t)ctx->scnt.p, (int64_t)o_item2,
                                (int64_t)(intptr_t)out, (int64_t)(intptr_t)ctx->tables.p,
                                (int64_t)(intptr_t)ctx->ws_fwd.p, (int64_t)(intptr_t)ctx->ws_inv.p,
                                (int64_t)(intptr_t)ctx->pp.p, (int64_t)(intptr_t)ctx->rspec.p,
                                (int64_t)o_u, (int64_t)o_fwd, (int64_t)o_inv, (int64_t)o_z, (int64_t)o_gam,
                                (int64_t)o_thr, ncfg};
    int64_t bbits;
    std::memcpy(&bbits, &beta, sizeof(bbits));
    sig.push_back(bbits);
    for (const Plan::Chunk &ch : P.chunks)
        for (int64_t v : {(int64_t)ch.c0, (int64_t)ch.c1, (int64_t)ch.off0, (int64_t)ch.nfwd, (int64_t)ch.ninv,
                          (int64_t)ch.z0, (int64_t)ch.nz, ch.ws_fwd, ch.ws_inv, (int64_t)ch.pp, (int64_t)ch.zhalf,
                          (int64_t)ch.nitems, (int64_t)ch.nitems2, ch.nsurv, ch.nruns, ch.nfree,
                          (int64_t)ch.max_atoms})
            sig.push_back(v);
    if (!(ctx->graph_exec && sig == ctx->graph_sig)) {
        if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
        if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
        ctx->graph_exec = nullptr;
        ctx->graph = nullptr;
        ctx->graph_sig.clear();
        if (!ctx->cap_stream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        HIPCHK(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        const int lrc = launch_all(ctx->cap_stream);
        hipGraph_t gph = nullptr;
        const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &gph);
        if (lrc) {
            if (gph) (void)hipGraphDestroy(gph);
            return lrc;
        }
        if (ec != hipSuccess || !gph)
            return set_err(ctx, FFTDG_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
        hipGraphExec_t ex = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ex, gph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(gph);
            return set_err(ctx, FFTDG_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
        }
        ctx->graph = gph;
        ctx->graph_exec = ex;
        ctx->graph_sig = sig;
    }
    HIPCHK(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
    return FFTDG_OK;
}

// Argument checks shared by the two reduce entry points.
int reduce_check(fftdg_ctx *ctx, const fftdg_batch *b, const fftdg_partial *p, double T_K, const double *B_host,
                 const fftdg_ligand_result *res_host, const char *who) {
    if (!ctx) return FFTDG_E_INVALID;
    if (ctx->n_snap <= 0) return set_err(ctx, FFTDG_E_STATE, std::string(who) + " before set_receptors");
    if (!b || b->n_lig <= 0 || !b->cfg_off) return set_err(ctx, FFTDG_E_INVALID, std::string(who) + ": bad batch");
    if (!p || !B_host || !res_host) return set_err(ctx, FFTDG_E_INVALID, std::string(who) + ": NULL pointer");
    if (!(T_K > 0.0) || !is_fin(T_K))
        return set_err(ctx, FFTDG_E_INVALID, std::string(who) + ": temperature must be > 0");
    return FFTDG_OK;
}

// Eqs. 2, 12 and 13 on the device with the given buffers (cfg_off [n_lig + 1],
// W [n_snap], B [n_lig][n_snap], res [n_lig]); copies B and res to the host
// and synchronizes the stream.  Allocates nothing.
int reduce_into(fftdg_ctx *ctx, const fftdg_batch *b, const fftdg_partial *p, const double *cfg_w, double T_K,
                double *B_host, fftdg_ligand_result *res_host, int32_t *off_d, double *W_d, double *B_d,
                LigRed *res_d, bool profiled) {
    const int nl = b->n_lig, ns = ctx->n_snap;
    HIPCHK(ctx, hipMemcpyAsync(off_d, b->cfg_off, sizeof(int32_t) * (nl + 1), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(W_d, ctx->W.data(), sizeof(double) * ns, hipMemcpyHostToDevice, ctx->stream));
    const double kT = kR * T_K;
    const double h3 = ctx->g.h * ctx->g.h * ctx->g.h;
    auto launch = [&] {
        return launch_reduce(ctx->stream, p, b->cfg_off[nl], ns, nl, off_d, cfg_w, W_d, kT, h3, kC0, B_d, res_d);
    };
    if (profiled)
        HIPCHK(ctx, timed(ctx, FFTDG_K_REDUCE, (double)sizeof(fftdg_partial) * (double)b->cfg_off[nl] * ns, launch));
    else
        HIPCHK(ctx, launch());
    HIPCHK(ctx, hipMemcpyAsync(B_host, B_d, sizeof(double) * (size_t)nl * ns, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(res_host, res_d, sizeof(LigRed) * nl, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return FFTDG_OK;
}

}  // namespace

extern "C" {

int fftdg_version(void) { return FFTDG_VERSION; }

const char *fftdg_status_string(int s) {
    switch (s) {
    case FFTDG_OK: return "ok";
    case FFTDG_E_INVALID: return "invalid argument";
    case FFTDG_E_NOVALID: return "no box-valid translation";
    case FFTDG_E_NOMEM: return "out of memory";
    case FFTDG_E_DEVICE: return "device error";
    case FFTDG_E_STATE: return "call out of order";
    default: return "unknown status";
    }
}

const char *fftdg_last_error(const fftdg_ctx *ctx) { return ctx ? ctx->err.c_str() : "context is NULL"; }

int fftdg_create(fftdg_ctx **out, const fftdg_grid_desc *g, int device, void *hip_stream) {
    if (!out) return FFTDG_E_INVALID;
    *out = nullptr;
    if (!g) return FFTDG_E_INVALID;
    fftdg_ctx tmp;
    auto fail = [&](int code, const std::string &m) {
        std::fprintf(stderr, "fftdg_create: %s\n", m.c_str());
        return code;
    };
    if (g->precision != FFTDG_F32 && g->precision != FFTDG_F64) return fail(FFTDG_E_INVALID, "precision must be FFTDG_F32 or FFTDG_F64");
    if (g->clash_mode != FFTDG_OCC && g->clash_mode != FFTDG_CAP) return fail(FFTDG_E_INVALID, "clash_mode must be FFTDG_OCC or FFTDG_CAP");
    const KernelSet *ks = kernel_set(g->precision, g->n_fft);
    if (!ks) return fail(FFTDG_E_INVALID, "unsupported n_fft for this precision (F32: 32/64/128/256, F64: 32/64)");
    if (g->n_rec < 4 || g->n_rec > g->n_fft) return fail(FFTDG_E_INVALID, "need 4 <= n_rec <= n_fft");
    if (!(g->h > 0.0) || !is_fin(g->h)) return fail(FFTDG_E_INVALID, "h must be finite and > 0");
    for (int d = 0; d < 3; ++d)
        if (!is_fin(g->origin[d])) return fail(FFTDG_E_INVALID, "origin must be finite");
    if (g->clash_mode == FFTDG_CAP && (!(g->ljr_cap > 0.0) || !is_fin(g->ljr_cap)))
        return fail(FFTDG_E_INVALID, "ljr_cap must be finite and > 0 in CAP mode");
    if (g->clash_mode == FFTDG_OCC && (!(g->occ_f > 0.0) || !is_fin(g->occ_f)))
        return fail(FFTDG_E_INVALID, "occ_f must be finite and > 0 in OCC mode");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return fail(FFTDG_E_DEVICE, "no HIP device");
    }
    if (device < 0 || device >= ndev) return fail(FFTDG_E_INVALID, "device index out of range");
    fftdg_ctx *c = new (std::nothrow) fftdg_ctx();
    if (!c) return FFTDG_E_NOMEM;
    c->g = *g;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->ks = ks;
    c->fs = fused_set(g->precision, g->n_fft);
    c->fused = c->fs != nullptr ? 1 : 0;
    c->n_ch = g->clash_mode == FFTDG_OCC ? 4 : 3;
    if (hipSetDevice(device) != hipSuccess || hipEventCreateWithFlags(&c->staging_ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return fail(FFTDG_E_DEVICE, "hipSetDevice/hipEventCreate failed");
    }
    {
        std::string why;
        c->scratch = static_scratch_ptr(device, &why);
        if (!c->scratch) {
            fftdg_destroy(c);
            return fail(FFTDG_E_DEVICE, why);
        }
    }
    // twiddles w_N^k = exp(-2 pi i k / N), FP64 then rounded once
    const int N = g->n_fft;
    std::vector<char> tw((size_t)N * ks->cbytes);
    for (int k = 0; k < N; ++k) {
        const double a = 2.0 * M_PI * (double)k / (double)N;
        const double re = std::cos(a), im = -std::sin(a);
        if (g->precision == FFTDG_F32) {
            float *f = (float *)tw.data();
            f[2 * k] = (float)re;
            f[2 * k + 1] = (float)im;
        } else {
            double *f = (double *)tw.data();
            f[2 * k] = re;
            f[2 * k + 1] = im;
        }
    }
    int rc = reserve(c, c->tw, tw.size());
    if (rc) {
        fftdg_destroy(c);
        return rc;
    }
    if (hipMemcpy(c->tw.p, tw.data(), tw.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        fftdg_destroy(c);
        return fail(FFTDG_E_DEVICE, "twiddle upload failed");
    }
    *out = c;
    return FFTDG_OK;
}

void fftdg_destroy(fftdg_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    DevBuf *bufs[] = {&c->tw, &c->rspec, &c->rxy, &c->ws_fwd, &c->ws_inv, &c->pp, &c->tables,
                      &c->red_B, &c->red_res, &c->red_off, &c->red_W, &c->prof_cnt, &c->tune_out,
                      &c->sir_psi, &c->sir_clash, &c->sir_u, &c->sir_lin, &c->sir_psi_out,
                      &c->dil, &c->runs, &c->run_cnt, &c->fbits, &c->lives, &c->zat, &c->zbt, &c->surv,
                      &c->scnt};
    for (DevBuf *b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->staging_ev) (void)hipEventDestroy(c->staging_ev);
    for (auto &r : c->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (hipEvent_t e : {c->ev_fork, c->ev_join, c->ev_side[0], c->ev_side[1], c->ev_main[0], c->ev_main[1]})
        if (e) (void)hipEventDestroy(e);
    if (c->side) (void)hipStreamDestroy(c->side);
    delete c;
}

int fftdg_set_stream(fftdg_ctx *ctx, void *s) {
    if (!ctx) return FFTDG_E_INVALID;
    ctx->stream = (hipStream_t)s;
    return FFTDG_OK;
}

int fftdg_receptor_grids(fftdg_ctx *ctx, int32_t n_atoms, const double *xyz, const double *q, const double *sg,
                         const double *ep, void *grids, uint8_t *occ) {
    if (!ctx) return FFTDG_E_INVALID;
    if (n_atoms <= 0 || !xyz || !q || !sg || !ep || !grids)
        return set_err(ctx, FFTDG_E_INVALID, "receptor_grids: bad atom count or NULL pointer");
    if (ctx->g.clash_mode == FFTDG_OCC && !occ) return set_err(ctx, FFTDG_E_INVALID, "receptor_grids: occ_dev required in OCC mode");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, launch_receptor_grids(ctx->stream, ctx->g.precision, n_atoms, xyz, q, sg, ep, ctx->g.n_rec, ctx->g.h,
                                      ctx->g.origin, ctx->g.clash_mode == FFTDG_CAP ? 1 : 0, ctx->g.ljr_cap,
                                      ctx->g.occ_f, grids, ctx->g.clash_mode == FFTDG_OCC ? occ : nullptr));
    return FFTDG_OK;
}

int fftdg_set_receptors(fftdg_ctx *ctx, int32_t n_snap, const void *grids, const uint8_t *occ, const double *w) {
    if (!ctx) return FFTDG_E_INVALID;
    if (n_snap <= 0 || !grids) return set_err(ctx, FFTDG_E_INVALID, "set_receptors: n_snap must be > 0 and grids non-NULL");
    const bool is_occ = ctx->g.clash_mode == FFTDG_OCC;
    if (is_occ && !occ) return set_err(ctx, FFTDG_E_INVALID, "set_receptors: occupancy grids required in OCC mode");
    std::vector<double> W(n_snap, 1.0);
    if (w) {
        double s = 0.0;
        for (int i = 0; i < n_snap; ++i) {
            if (!is_fin(w[i]) || w[i] < 0.0) return set_err(ctx, FFTDG_E_INVALID, "set_receptors: weights must be finite and >= 0");
            s += w[i];
        }
        if (!(s > 0.0)) return set_err(ctx, FFTDG_E_INVALID, "set_receptors: weights sum to 0");
        for (int i = 0; i < n_snap; ++i) W[i] = w[i] / s;
    } else {
        for (int i = 0; i < n_snap; ++i) W[i] = 1.0 / n_snap;
    }
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const fftdg_grid_desc &g = ctx->g;
    const size_t cb = ctx->ks->cbytes;
    const size_t per_snap = (size_t)ctx->n_ch * g.n_fft * ctx->ks->np * cb;
    int rc;
    if ((rc = reserve(ctx, ctx->rspec, per_snap * n_snap))) return rc;
    if ((rc = reserve(ctx, ctx->rxy, (size_t)ctx->n_ch * g.n_rec * ctx->ks->np * cb))) return rc;
    const size_t n3 = (size_t)g.n_rec * g.n_rec * g.n_rec;
    const size_t tsz = g.precision == FFTDG_F32 ? 4 : 8;
    // bytes: grids read, xy planes written and read back, spectra written
    const double b_spec = (double)(3 * n3 * tsz + (is_occ ? n3 : 0)) +
                          2.0 * ctx->n_ch * g.n_rec * (double)ctx->ks->np * cb + (double)per_snap;
    for (int s = 0; s < n_snap; ++s) {
        HIPCHK(ctx, timed(ctx, FFTDG_K_SPECTRA, b_spec, [&] {
                   return ctx->ks->rec_spectra(ctx->stream, (const char *)grids + s * 3 * n3 * tsz,
                                               is_occ ? occ + s * n3 : nullptr, g.n_rec, ctx->n_ch, ctx->tw.p,
                                               ctx->rxy.p, (char *)ctx->rspec.p + s * per_snap);
               }));
    }
    if (is_occ && ctx->fs) {
        // bit rows of the clash test (fused path), one table per snapshot
        const size_t dw = (size_t)ctx->fs->dil_words;
        if ((rc = reserve(ctx, ctx->dil, sizeof(uint32_t) * dw * n_snap))) return rc;
        for (int s = 0; s < n_snap; ++s)
            HIPCHK(ctx, timed(ctx, FFTDG_K_SPECTRA, (double)n3 + 4.0 * (double)dw, [&] {
                       return ctx->fs->rec_dilate(ctx->stream, occ + s * n3, g.n_rec, (uint32_t *)ctx->dil.p + s * dw);
                   }));
    }
    ctx->n_snap = n_snap;
    ctx->W = W;
    return FFTDG_OK;
}

int fftdg_scan(fftdg_ctx *ctx, const fftdg_batch *b, double T_K, fftdg_partial *out) {
    if (!ctx) return FFTDG_E_INVALID;
    if (ctx->n_snap <= 0) return set_err(ctx, FFTDG_E_STATE, "scan before set_receptors");
    if (!out) return set_err(ctx, FFTDG_E_INVALID, "scan: out_dev is NULL");
    if (!(T_K > 0.0) || !is_fin(T_K)) return set_err(ctx, FFTDG_E_INVALID, "scan: temperature must be finite and > 0");
    int rc = validate_batch(ctx, b);
    if (rc) return rc;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    Plan P;
    if ((rc = build_plan(ctx, b, false, -1, P))) return rc;
    return run_plan(ctx, b, P, T_K, out, -1, nullptr, nullptr);
}

int fftdg_energy_grid(fftdg_ctx *ctx, int32_t snap, const fftdg_batch *b, int32_t cfg, double T_K, void *psi,
                      uint8_t *clash, int32_t *shape) {
    if (!ctx) return FFTDG_E_INVALID;
    int rc = validate_batch(ctx, b);
    if (rc) return rc;
    const int ncfg = b->cfg_off[b->n_lig];
    if (cfg < 0 || cfg >= ncfg) return set_err(ctx, FFTDG_E_INVALID, "energy_grid: configuration index out of range");
    if (!shape) return set_err(ctx, FFTDG_E_INVALID, "energy_grid: shape_host is NULL");
    if (!(T_K > 0.0) || !is_fin(T_K)) return set_err(ctx, FFTDG_E_INVALID, "energy_grid: temperature must be > 0");
    // placement of this configuration only
    const int l = (int)(std::upper_bound(b->cfg_off, b->cfg_off + b->n_lig + 1, cfg) - b->cfg_off) - 1;
    fftdg_batch one = *b;
    (void)l;
    Plan P;
    if ((rc = build_plan(ctx, &one, true, cfg, P))) return rc;
    const CfgDev &d = P.cfg[cfg];
    shape[0] = d.V[2];
    shape[1] = d.V[1];
    shape[2] = d.V[0];
    if (!psi) return FFTDG_OK;
    if (ctx->n_snap <= 0) return set_err(ctx, FFTDG_E_STATE, "energy_grid before set_receptors");
    if (snap < 0 || snap >= ctx->n_snap) return set_err(ctx, FFTDG_E_INVALID, "energy_grid: snapshot out of range");
    if (d.n_valid <= 0) return FFTDG_OK;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if ((rc = run_plan(ctx, b, P, T_K, nullptr, snap, psi, clash))) return rc;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return FFTDG_OK;
}

int fftdg_place(fftdg_ctx *ctx, const fftdg_batch *b, int32_t cfg, int32_t *U, int32_t *box) {
    if (!ctx) return FFTDG_E_INVALID;
    int rc = validate_batch(ctx, b);
    if (rc) return rc;
    const int ncfg = b->cfg_off[b->n_lig];
    if (cfg < 0 || cfg >= ncfg || !U || !box) return set_err(ctx, FFTDG_E_INVALID, "place: bad index or NULL output");
    const int l = (int)(std::upper_bound(b->cfg_off, b->cfg_off + b->n_lig + 1, cfg) - b->cfg_off) - 1;
    const int na = b->atom_off[l + 1] - b->atom_off[l];
    size_t row = 0;
    for (int k = 0; k < l; ++k) row += (size_t)(b->conf_off[k + 1] - b->conf_off[k]) * (b->atom_off[k + 1] - b->atom_off[k]);
    const double *X = b->conf_xyz + 3 * (row + (size_t)b->cfg_conf[cfg] * na);
    int bx[3];
    if (!place_one(X, na, b->cfg_quat + 4 * cfg, ctx->g.h, U, bx))
        return set_err(ctx, FFTDG_E_INVALID, "place: zero or non-finite quaternion");
    for (int d = 0; d < 3; ++d) box[d] = bx[d];
    return FFTDG_OK;
}

int fftdg_reduce(fftdg_ctx *ctx, const fftdg_batch *b, const fftdg_partial *p, const double *cfg_w, double T_K,
                 double *B_host, fftdg_ligand_result *res_host) {
    int rc = reduce_check(ctx, b, p, T_K, B_host, res_host, "reduce");
    if (rc) return rc;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int nl = b->n_lig, ns = ctx->n_snap;
    if ((rc = reserve(ctx, ctx->red_off, sizeof(int32_t) * (nl + 1)))) return rc;
    if ((rc = reserve(ctx, ctx->red_W, sizeof(double) * ns))) return rc;
    if ((rc = reserve(ctx, ctx->red_B, sizeof(double) * (size_t)nl * ns))) return rc;
    if ((rc = reserve(ctx, ctx->red_res, sizeof(LigRed) * nl))) return rc;
    return reduce_into(ctx, b, p, cfg_w, T_K, B_host, res_host, (int32_t *)ctx->red_off.p, (double *)ctx->red_W.p,
                       (double *)ctx->red_B.p, (LigRed *)ctx->red_res.p, true);
}

int fftdg_reduce_static(fftdg_ctx *ctx, const fftdg_batch *b, const fftdg_partial *p, const double *cfg_w,
                        double T_K, double *B_host, fftdg_ligand_result *res_host) {
    int rc = reduce_check(ctx, b, p, T_K, B_host, res_host, "reduce_static");
    if (rc) return rc;
    const size_t nl = (size_t)b->n_lig, ns = (size_t)ctx->n_snap;
    // scratch layout: cfg_off [nl + 1] | W [ns] | B [nl][ns] | LigRed [nl], each 256-byte aligned
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t o_W = up(sizeof(int32_t) * (nl + 1));
    const size_t o_B = o_W + up(sizeof(double) * ns);
    const size_t o_res = o_B + up(sizeof(double) * nl * ns);
    const size_t need = o_res + sizeof(LigRed) * nl;
    if (need > (size_t)FFTDG_REDUCE_STATIC_BYTES)
        return set_err(ctx, FFTDG_E_INVALID,
                       "reduce_static: " + std::to_string(nl) + " ligands x " + std::to_string(ns) +
                           " snapshots need " + std::to_string(need) + " bytes of static scratch; the limit is " +
                           std::to_string((size_t)FFTDG_REDUCE_STATIC_BYTES) + " (fftdg_reduce has no limit)");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    char *base = (char *)ctx->scratch;
    return reduce_into(ctx, b, p, cfg_w, T_K, B_host, res_host, (int32_t *)base, (double *)(base + o_W),
                       (double *)(base + o_B), (LigRed *)(base + o_res), false);
}

int fftdg_profile(fftdg_ctx *ctx, int enable) {
    if (!ctx) return FFTDG_E_INVALID;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (auto &r : ctx->recs) {
        ctx->ev_pool.push_back(r.a);
        ctx->ev_pool.push_back(r.b);
    }
    ctx->recs.clear();
    ctx->prof_fused = false;
    for (int k = 0; k < FFTDG_N_KERNELS; ++k) {
        ctx->prof_ms[k] = 0.0;
        ctx->prof_n[k] = 0;
        ctx->prof_bytes[k] = 0.0;
    }
    if (enable) {
        int rc = reserve(ctx, ctx->prof_cnt, sizeof(unsigned int));
        if (rc) return rc;
        const unsigned int zero = 0;
        HIPCHK(ctx, hipMemcpy(ctx->prof_cnt.p, &zero, sizeof(zero), hipMemcpyHostToDevice));
    }
    ctx->prof = enable != 0;
    return FFTDG_OK;
}

int fftdg_profile_read(fftdg_ctx *ctx, int32_t k, double *ms, int64_t *n, double *bytes) {
    if (!ctx) return FFTDG_E_INVALID;
    if (k < 0 || k >= FFTDG_N_KERNELS || !ms || !n || !bytes)
        return set_err(ctx, FFTDG_E_INVALID, "profile_read: bad kernel id or NULL output");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (auto &r : ctx->recs) {
        float t = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&t, r.a, r.b));
        ctx->prof_ms[r.k] += t;
        ctx->prof_n[r.k] += 1;
        ctx->prof_bytes[r.k] += r.bytes;
        ctx->ev_pool.push_back(r.a);
        ctx->ev_pool.push_back(r.b);
    }
    ctx->recs.clear();
    if (ctx->prof_cnt.p) {
        unsigned int cnt = 0;
        HIPCHK(ctx, hipMemcpy(&cnt, ctx->prof_cnt.p, sizeof(cnt), hipMemcpyDeviceToHost));
        const unsigned int zero = 0;
        HIPCHK(ctx, hipMemcpy(ctx->prof_cnt.p, &zero, sizeof(zero), hipMemcpyHostToDevice));
        ctx->prof_bytes[FFTDG_K_INV] += (double)cnt * ctx->ks->np * ctx->ks->cbytes;
        if (ctx->prof_fused) ctx->prof_bytes[FFTDG_K_ZPROD] += (double)cnt * ctx->ks->np * ctx->ks->cbytes;
        ctx->prof_fused = false;
    }
    *ms = ctx->prof_ms[k];
    *n = ctx->prof_n[k];
    *bytes = ctx->prof_bytes[k];
    return FFTDG_OK;
}

int fftdg_get_tuning(const fftdg_ctx *ctx, fftdg_tuning *t) {
    if (!ctx || !t) return FFTDG_E_INVALID;
    t->configs_per_chunk = ctx->chunk_cfgs;
    t->energy_xy_direct = ctx->edirect;
    t->snapshots_per_pass = ctx->snap_group;
    t->use_graph = ctx->use_graph ? 1 : 0;
    t->fused = ctx->fused;
    t->clash_stream = ctx->clash_stream ? 1 : 0;
    return FFTDG_OK;
}

int fftdg_set_tuning(fftdg_ctx *ctx, const fftdg_tuning *t) {
    if (!ctx) return FFTDG_E_INVALID;
    if (!t) return set_err(ctx, FFTDG_E_INVALID, "set_tuning: NULL");
    if (t->configs_per_chunk < 1) return set_err(ctx, FFTDG_E_INVALID, "set_tuning: configs_per_chunk must be >= 1");
    if (t->energy_xy_direct < 0 || t->energy_xy_direct > 2)
        return set_err(ctx, FFTDG_E_INVALID, "set_tuning: energy_xy_direct must be 0, 1 or 2");
    if (t->energy_xy_direct == 1 && ctx->g.n_fft > 128)
        return set_err(ctx, FFTDG_E_INVALID, "set_tuning: energy_xy_direct = 1 needs n_fft <= 128");
    if (t->snapshots_per_pass < 1) return set_err(ctx, FFTDG_E_INVALID, "set_tuning: snapshots_per_pass must be >= 1");
    if (t->use_graph != 0 && t->use_graph != 1) return set_err(ctx, FFTDG_E_INVALID, "set_tuning: use_graph must be 0 or 1");
    if (t->fused < 0 || t->fused > 2) return set_err(ctx, FFTDG_E_INVALID, "set_tuning: fused must be 0, 1 or 2");
    if (t->fused && !ctx->fs) return set_err(ctx, FFTDG_E_INVALID, "set_tuning: the fused path needs n_fft <= 128");
    if (t->clash_stream != 0 && t->clash_stream != 1)
        return set_err(ctx, FFTDG_E_INVALID, "set_tuning: clash_stream must be 0 or 1");
    ctx->chunk_cfgs = t->configs_per_chunk;
    ctx->edirect = t->energy_xy_direct;
    ctx->snap_group = t->snapshots_per_pass;
    ctx->use_graph = t->use_graph != 0;
    ctx->fused = t->fused;
    ctx->clash_stream = t->clash_stream != 0;
    return FFTDG_OK;
}

int fftdg_config_features(fftdg_ctx *ctx, const fftdg_batch *b, float *feat) {
    if (!ctx) return FFTDG_E_INVALID;
    int rc = validate_batch(ctx, b);
    if (rc) return rc;
    if (!feat) return set_err(ctx, FFTDG_E_INVALID, "config_features: NULL output");
    size_t row = 0;
    for (int l = 0; l < b->n_lig; ++l) {
        const int na = b->atom_off[l + 1] - b->atom_off[l];
        const int nc = b->conf_off[l + 1] - b->conf_off[l];
        std::vector<double> rg(nc);
        for (int k = 0; k < nc; ++k) {
            const double *X = b->conf_xyz + 3 * (row + (size_t)k * na);
            double cm[3] = {0, 0, 0}, s2 = 0.0;
            for (int i = 0; i < na; ++i)
                for (int d = 0; d < 3; ++d) cm[d] += X[3 * i + d] / na;
            for (int i = 0; i < na; ++i)
                for (int d = 0; d < 3; ++d) s2 += (X[3 * i + d] - cm[d]) * (X[3 * i + d] - cm[d]);
            rg[k] = std::sqrt(s2 / na);
        }
        std::vector<int32_t> U(3 * (size_t)na);
        for (int c = b->cfg_off[l]; c < b->cfg_off[l + 1]; ++c) {
            float *f = feat + (size_t)c * FFTDG_N_FEATURES;
            const double *q = b->cfg_quat + 4 * c;
            const double nq = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
            if (!(nq > 0.0)) return set_err(ctx, FFTDG_E_INVALID, "config_features: zero quaternion");
            const double sg = q[0] < 0.0 ? -1.0 : 1.0;
            for (int d = 0; d < 4; ++d) f[d] = (float)(sg * q[d] / nq);
            for (int d = 0; d < 8; ++d) f[4 + d] = (b->cfg_conf[c] % 8) == d ? 1.f : 0.f;
            f[12] = (float)(na / 40.0);
            f[13] = (float)(std::log((double)na) / std::log(40.0));
            const int k = b->cfg_conf[c];
            int box[3];
            if (!place_one(b->conf_xyz + 3 * (row + (size_t)k * na), na, q, ctx->g.h, U.data(), box))
                return set_err(ctx, FFTDG_E_INVALID, "config_features: placement failed");
            for (int d = 0; d < 3; ++d) {
                int32_t mx = U[d];
                for (int i = 1; i < na; ++i) mx = std::max(mx, U[3 * i + d]);
                f[14 + d] = (float)((mx / 65536.0 - 2.0) * ctx->g.h / 10.0);
            }
            f[17] = (float)(rg[k] / 5.0);
        }
        row += (size_t)nc * na;
    }
    return FFTDG_OK;
}

int fftdg_autotune(fftdg_ctx *ctx, const fftdg_batch *b, double T_K, int32_t max_cfgs, fftdg_tuning *out,
                   double *ms_host) {
    if (!ctx) return FFTDG_E_INVALID;
    if (ctx->n_snap <= 0) return set_err(ctx, FFTDG_E_STATE, "autotune before set_receptors");
    if (max_cfgs < 1) return set_err(ctx, FFTDG_E_INVALID, "autotune: max_cfgs must be >= 1");
    if (!(T_K > 0.0) || !is_fin(T_K)) return set_err(ctx, FFTDG_E_INVALID, "autotune: temperature must be > 0");
    int rc = validate_batch(ctx, b);
    if (rc) return rc;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int ncfg = b->cfg_off[b->n_lig];
    // evenly strided sample, within the caller's selection
    std::vector<uint8_t> sel(ncfg, 0);
    const int stride = std::max(1, (ncfg + max_cfgs - 1) / max_cfgs);
    int nsel = 0;
    for (int c = 0; c < ncfg; c += stride)
        if (!b->cfg_select || b->cfg_select[c]) {
            sel[c] = 1;
            ++nsel;
        }
    if (nsel == 0) return set_err(ctx, FFTDG_E_INVALID, "autotune: empty sample");
    fftdg_batch bs = *b;
    bs.cfg_select = sel.data();
    if ((rc = reserve(ctx, ctx->tune_out, sizeof(fftdg_partial) * (size_t)ncfg * ctx->n_snap))) return rc;
    const fftdg_tuning keep = {ctx->chunk_cfgs, ctx->edirect, ctx->snap_group, ctx->use_graph ? 1 : 0,
                               ctx->fused, ctx->clash_stream ? 1 : 0};
    auto apply = [&](const fftdg_tuning &t) {
        ctx->chunk_cfgs = t.configs_per_chunk;
        ctx->edirect = t.energy_xy_direct;
        ctx->snap_group = t.snapshots_per_pass;
        ctx->use_graph = t.use_graph != 0;
        ctx->fused = t.fused;
        ctx->clash_stream = t.clash_stream != 0;
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return set_err(ctx, FFTDG_E_DEVICE, "autotune: hipEventCreate failed");
    }
    const bool prof = ctx->prof;
    ctx->prof = false;
    std::vector<fftdg_tuning> cand;
    std::vector<int> passes = {1};
    if (ctx->n_snap > 1) passes.push_back(ctx->n_snap);
    for (int chunk : {64, 128, 256, 512}) {
        if (ctx->fs)
            for (int fu : {1, 2})
                for (int gr : {0, 1})
                    for (int cs : {0, 1})
                        if (cs == 0 || ctx->g.clash_mode == FFTDG_OCC)
                            cand.push_back(fftdg_tuning{chunk, ctx->edirect, 1, gr, fu, cs});
        for (int ed : {0, 1, 2})
            for (int sp : passes)
                for (int gr : {0, 1})
                    for (int cs : {0, 1})
                        if (ed != 1 || ctx->g.n_fft <= 128) cand.push_back(fftdg_tuning{chunk, ed, sp, gr, 0, cs});
    }
    double best = INFINITY;
    fftdg_tuning bt = keep;
    int err = FFTDG_OK;
    for (const fftdg_tuning &t : cand) {
        apply(t);
        float tmin = INFINITY;
        for (int rep = 0; rep < 5 && !err; ++rep) {  // a warm-up run, then the fastest of four
            Plan P;
            if ((err = build_plan(ctx, &bs, false, -1, P))) break;
            if (hipEventRecord(e0, ctx->stream) != hipSuccess) err = FFTDG_E_DEVICE;
            if (!err) err = run_plan(ctx, &bs, P, T_K, (fftdg_partial *)ctx->tune_out.p, -1, nullptr, nullptr);
            if (!err && hipEventRecord(e1, ctx->stream) != hipSuccess) err = FFTDG_E_DEVICE;
            if (!err && hipEventSynchronize(e1) != hipSuccess) err = FFTDG_E_DEVICE;
            float ms = 0.f;
            if (!err && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) err = FFTDG_E_DEVICE;
            if (!err && rep > 0) tmin = std::min(tmin, ms);  // first run warms the plan's buffers
        }
        if (err) break;
        if (tmin < best) {
            best = tmin;
            bt = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->prof = prof;
    if (err) {
        apply(keep);
        if (err == FFTDG_E_DEVICE && ctx->err.empty()) ctx->err = "autotune: HIP event error";
        return err;
    }
    apply(bt);
    if (out) *out = bt;
    if (ms_host) *ms_host = best / ((double)nsel * ctx->n_snap);
    return FFTDG_OK;
}

int fftdg_scan_features(fftdg_ctx *ctx, const fftdg_batch *b, const fftdg_partial *p, float *feat, int32_t ld,
                        int32_t col0) {
    if (!ctx) return FFTDG_E_INVALID;
    if (ctx->n_snap <= 0) return set_err(ctx, FFTDG_E_STATE, "scan_features before set_receptors");
    if (!b || b->n_lig <= 0 || !b->cfg_off) return set_err(ctx, FFTDG_E_INVALID, "scan_features: bad batch");
    if (!p || !feat) return set_err(ctx, FFTDG_E_INVALID, "scan_features: NULL pointer");
    if (col0 < 0 || ld < col0 + FFTDG_N_SCAN_FEATURES)
        return set_err(ctx, FFTDG_E_INVALID, "scan_features: columns col0..col0+2 must lie within ld");
    for (int l = 0; l < b->n_lig; ++l)
        if (b->cfg_off[l + 1] < b->cfg_off[l]) return set_err(ctx, FFTDG_E_INVALID, "scan_features: bad cfg_off");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int nl = b->n_lig, ns = ctx->n_snap;
    int rc;
    if ((rc = reserve(ctx, ctx->red_off, sizeof(int32_t) * (nl + 1)))) return rc;
    if ((rc = reserve(ctx, ctx->red_W, sizeof(double) * ns))) return rc;
    HIPCHK(ctx, hipMemcpyAsync(ctx->red_off.p, b->cfg_off, sizeof(int32_t) * (nl + 1), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(ctx->red_W.p, ctx->W.data(), sizeof(double) * ns, hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(ctx, launch_scan_features(ctx->stream, p, b->cfg_off[nl], ns, nl, (const int32_t *)ctx->red_off.p,
                                     (const double *)ctx->red_W.p, feat, ld, col0));
    return FFTDG_OK;
}

int fftdg_is_plan(fftdg_ctx *ctx, const fftdg_batch *b, const float *yhat, double top_frac, double draw_frac,
                  double alpha, double tau, const double *u, int64_t n_u, uint8_t *sel, double *wt,
                  int64_t *n_scan) {
    // host only; ctx (may be NULL) just keeps the error message
    if (!b || b->n_lig <= 0 || !b->cfg_off) return set_err(ctx, FFTDG_E_INVALID, "is_plan: bad batch");
    if (!yhat || !sel || !wt || (!u && n_u > 0)) return set_err(ctx, FFTDG_E_INVALID, "is_plan: NULL pointer");
    if (!(top_frac >= 0.0 && top_frac <= 1.0) || !(draw_frac >= 0.0 && draw_frac <= 1.0))
        return set_err(ctx, FFTDG_E_INVALID, "is_plan: fractions must lie in [0, 1]");
    if (!(alpha >= 0.0 && alpha <= 1.0)) return set_err(ctx, FFTDG_E_INVALID, "is_plan: alpha must lie in [0, 1]");
    if (!(tau > 0.0) || !is_fin(tau)) return set_err(ctx, FFTDG_E_INVALID, "is_plan: tau must be > 0");
    const int nl = b->n_lig;
    // uniforms needed, checked before anything is written
    int64_t need = 0;
    for (int l = 0; l < nl; ++l) {
        const int P = b->cfg_off[l + 1] - b->cfg_off[l];
        if (P < 0) return set_err(ctx, FFTDG_E_INVALID, "is_plan: bad cfg_off");
        const int nt = std::min<int64_t>(P, (int64_t)std::ceil(top_frac * P));
        if (P - nt > 0) need += (int64_t)std::ceil(draw_frac * P);
    }
    if (need > n_u) return set_err(ctx, FFTDG_E_INVALID, "is_plan: fewer uniforms than draws");
    for (int64_t c = 0; c < (int64_t)b->cfg_off[nl]; ++c)
        if (!is_fin((double)yhat[c])) return set_err(ctx, FFTDG_E_INVALID, "is_plan: non-finite prediction");
    for (int64_t k = 0; k < need; ++k)
        if (!(u[k] >= 0.0 && u[k] < 1.0)) return set_err(ctx, FFTDG_E_INVALID, "is_plan: uniforms must lie in [0, 1)");
    int64_t used = 0, n_sel = 0;
    std::vector<int> order, rest;
    std::vector<double> cdf;
    for (int l = 0; l < nl; ++l) {
        const int c0 = b->cfg_off[l], P = b->cfg_off[l + 1] - c0;
        for (int j = 0; j < P; ++j) {
            sel[c0 + j] = 0;
            wt[c0 + j] = 0.0;
        }
        if (P == 0) continue;
        const int nt = (int)std::min<int64_t>(P, (int64_t)std::ceil(top_frac * P));
        order.resize(P);
        for (int j = 0; j < P; ++j) order[j] = j;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int c) { return yhat[c0 + a] > yhat[c0 + c]; });
        std::vector<uint8_t> top(P, 0);
        for (int j = 0; j < nt; ++j) {
            top[order[j]] = 1;
            sel[c0 + order[j]] = 1;
            wt[c0 + order[j]] = 1.0;
        }
        const int R = P - nt;
        if (R == 0) continue;
        const int K = (int)std::ceil(draw_frac * P);
        if (K == 0) continue;
        rest.clear();
        for (int j = 0; j < P; ++j)
            if (!top[j]) rest.push_back(j);
        double ymax = -INFINITY;
        for (int j : rest) ymax = std::max(ymax, (double)yhat[c0 + j] / tau);
        double se = 0.0;
        for (int j : rest) se += std::exp((double)yhat[c0 + j] / tau - ymax);
        cdf.resize(R);
        std::vector<double> q(R);
        double run = 0.0;
        for (int i = 0; i < R; ++i) {
            q[i] = (1.0 - alpha) * std::exp((double)yhat[c0 + rest[i]] / tau - ymax) / se + alpha / R;
            run += q[i];
            cdf[i] = run;
        }
        std::vector<int> mult(R, 0);
        for (int k = 0; k < K; ++k) {
            const double x = u[used + k] * cdf[R - 1];
            int i = (int)(std::upper_bound(cdf.begin(), cdf.end(), x) - cdf.begin());
            if (i > R - 1) i = R - 1;
            ++mult[i];
        }
        used += K;
        for (int i = 0; i < R; ++i)
            if (mult[i] > 0) {
                sel[c0 + rest[i]] = 2;
                wt[c0 + rest[i]] = (double)mult[i] / ((double)K * q[i]);
            }
    }
    for (int64_t c = 0; c < (int64_t)b->cfg_off[nl]; ++c) n_sel += sel[c] != 0;
    if (n_scan) *n_scan = n_sel;
    return FFTDG_OK;
}

int fftdg_sample_poses(fftdg_ctx *ctx, const fftdg_batch *b, const fftdg_partial *p, int32_t lig, int32_t snap,
                       double T_K, int32_t K, const double *u, int32_t *cfg_out, int32_t *t_out, double *psi_out) {
    if (!ctx) return FFTDG_E_INVALID;
    if (ctx->n_snap <= 0) return set_err(ctx, FFTDG_E_STATE, "sample_poses before set_receptors");
    int rc = validate_batch(ctx, b);
    if (rc) return rc;
    if (lig < 0 || lig >= b->n_lig) return set_err(ctx, FFTDG_E_INVALID, "sample_poses: ligand out of range");
    if (snap < 0 || snap >= ctx->n_snap) return set_err(ctx, FFTDG_E_INVALID, "sample_poses: snapshot out of range");
    if (!(T_K > 0.0) || !is_fin(T_K)) return set_err(ctx, FFTDG_E_INVALID, "sample_poses: temperature must be > 0");
    if (K < 0) return set_err(ctx, FFTDG_E_INVALID, "sample_poses: K must be >= 0");
    if (K == 0) return FFTDG_OK;
    if (!p || !u || !cfg_out || !t_out || !psi_out) return set_err(ctx, FFTDG_E_INVALID, "sample_poses: NULL pointer");
    for (int k = 0; k < 2 * K; ++k)
        if (!(u[k] >= 0.0 && u[k] < 1.0)) return set_err(ctx, FFTDG_E_INVALID, "sample_poses: uniforms must lie in [0, 1)");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int ncfg = b->cfg_off[b->n_lig];
    const int c0 = b->cfg_off[lig], P = b->cfg_off[lig + 1] - c0;
    std::vector<fftdg_partial> hp(P);
    HIPCHK(ctx, hipMemcpyAsync(hp.data(), p + (int64_t)snap * ncfg + c0, sizeof(fftdg_partial) * P,
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    // configuration level: Z_c = exp(m_c - M) s_c in index order
    double M = -INFINITY;
    for (int j = 0; j < P; ++j)
        if (hp[j].n_finite > 0) M = std::max(M, hp[j].m);
    if (!(M > -INFINITY)) return set_err(ctx, FFTDG_E_NOVALID, "sample_poses: no clash-free translation to draw");
    std::vector<double> cdf(P);
    double run = 0.0;
    for (int j = 0; j < P; ++j) {
        if (hp[j].n_finite > 0) run += std::exp(hp[j].m - M) * hp[j].s;
        cdf[j] = run;
    }
    std::vector<int> pick(K);
    for (int k = 0; k < K; ++k) {
        const double x = u[2 * k] * cdf[P - 1];
        int j = (int)(std::upper_bound(cdf.begin(), cdf.end(), x) - cdf.begin());
        if (j > P - 1) j = P - 1;
        while (j > 0 && hp[j].n_finite == 0) --j;  // only at x == total (rounding)
        pick[k] = j;
    }
    // translation level, one drawn configuration at a time
    const double beta = 1.0 / (kR * T_K);
    const size_t tsz = ctx->g.precision == FFTDG_F32 ? sizeof(float) : sizeof(double);
    std::vector<int> order(K);
    for (int k = 0; k < K; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return pick[a] < pick[c]; });
    std::vector<double> uu;
    std::vector<int32_t> lin;
    std::vector<double> ps;
    for (size_t q = 0; q < order.size();) {
        const int j = pick[order[q]];
        size_t r = q;
        uu.clear();
        while (r < order.size() && pick[order[r]] == j) uu.push_back(u[2 * order[r++] + 1]);
        const int cfg = c0 + j;
        Plan PL;
        if ((rc = build_plan(ctx, b, true, cfg, PL))) return rc;
        const CfgDev &d = PL.cfg[cfg];
        const int n = d.n_valid;
        if (n <= 0) return set_err(ctx, FFTDG_E_INVALID, "sample_poses: drawn configuration has no valid translation");
        if ((rc = reserve(ctx, ctx->sir_psi, tsz * (size_t)n))) return rc;
        if ((rc = reserve(ctx, ctx->sir_clash, (size_t)n))) return rc;
        if ((rc = reserve(ctx, ctx->sir_u, sizeof(double) * uu.size()))) return rc;
        if ((rc = reserve(ctx, ctx->sir_lin, sizeof(int32_t) * uu.size()))) return rc;
        if ((rc = reserve(ctx, ctx->sir_psi_out, sizeof(double) * uu.size()))) return rc;
        if ((rc = run_plan(ctx, b, PL, T_K, nullptr, snap, ctx->sir_psi.p, (uint8_t *)ctx->sir_clash.p))) return rc;
        HIPCHK(ctx, hipMemcpyAsync(ctx->sir_u.p, uu.data(), sizeof(double) * uu.size(), hipMemcpyHostToDevice,
                                   ctx->stream));
        HIPCHK(ctx, launch_sample_translations(ctx->stream, ctx->g.precision, ctx->sir_psi.p,
                                               (const uint8_t *)ctx->sir_clash.p, n, beta,
                                               (const double *)ctx->sir_u.p, (int)uu.size(),
                                               (int32_t *)ctx->sir_lin.p, (double *)ctx->sir_psi_out.p));
        lin.resize(uu.size());
        ps.resize(uu.size());
        HIPCHK(ctx, hipMemcpyAsync(lin.data(), ctx->sir_lin.p, sizeof(int32_t) * uu.size(), hipMemcpyDeviceToHost,
                                   ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(ps.data(), ctx->sir_psi_out.p, sizeof(double) * uu.size(), hipMemcpyDeviceToHost,
                                   ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        const int Vx = d.V[0], Vy = d.V[1];
        for (size_t i = 0; i < uu.size(); ++i) {
            const int k = order[q + i];
            const int l = lin[i];
            cfg_out[k] = cfg;
            t_out[3 * k + 0] = l % Vx;
            t_out[3 * k + 1] = (l / Vx) % Vy;
            t_out[3 * k + 2] = l / (Vx * Vy);
            psi_out[k] = ps[i];
        }
        q = r;
    }
    return FFTDG_OK;
}

static int grid_desc_ok(const fftdg_grid_desc *g) {
    return g && g->n_rec >= 2 && g->n_rec <= 1024 && g->h > 0.0 && is_fin(g->h) && is_fin(g->origin[0]) &&
           is_fin(g->origin[1]) && is_fin(g->origin[2]) && (g->precision == FFTDG_F32 || g->precision == FFTDG_F64) &&
           (g->clash_mode == FFTDG_OCC || g->clash_mode == FFTDG_CAP) && g->occ_f > 0.0 && is_fin(g->ljr_cap);
}

int fftdg_grids_build(int device, void *stream, const fftdg_grid_desc *g, int32_t n_atoms, const double *xyz,
                      const double *q, const double *sg, const double *ep, void *grids, uint8_t *occ) {
    if (!grid_desc_ok(g) || n_atoms <= 0 || !xyz || !q || !sg || !ep || !grids) return FFTDG_E_INVALID;
    if (g->clash_mode == FFTDG_OCC && !occ) return FFTDG_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) return FFTDG_E_DEVICE;
    if (launch_receptor_grids((hipStream_t)stream, g->precision, n_atoms, xyz, q, sg, ep, g->n_rec, g->h, g->origin,
                              g->clash_mode == FFTDG_CAP ? 1 : 0, g->ljr_cap, g->occ_f, grids,
                              g->clash_mode == FFTDG_OCC ? occ : nullptr) != hipSuccess)
        return FFTDG_E_DEVICE;
    return FFTDG_OK;
}

int fftdg_grid_energies(int device, void *stream, const fftdg_grid_desc *g, const void *grids, int32_t n_poses,
                        int32_t n_atoms, const double *q, const double *sg, const double *ep, const double *pose_xyz,
                        double *out) {
    if (!grid_desc_ok(g) || n_poses < 0 || n_atoms <= 0 || n_atoms > 256 || !grids || !q || !sg || !ep ||
        (n_poses > 0 && (!pose_xyz || !out)))
        return FFTDG_E_INVALID;
    if (n_poses == 0) return FFTDG_OK;
    if (hipSetDevice(device) != hipSuccess) return FFTDG_E_DEVICE;
    if (launch_grid_energies((hipStream_t)stream, g->precision, grids, g->n_rec, g->h, g->origin, n_atoms, q, sg, ep,
                             n_poses, pose_xyz, out) != hipSuccess)
        return FFTDG_E_DEVICE;
    return FFTDG_OK;
}

int fftdg_pair_energies(int device, void *stream, int32_t n_rec_atoms, const double *rxyz, const double *rq,
                        const double *rs, const double *re, int32_t n_poses, int32_t n_atoms, const double *q,
                        const double *sg, const double *ep, const double *pose_xyz, int32_t exclusion, double *out) {
    if (n_rec_atoms <= 0 || !rxyz || !rq || !rs || !re || n_poses < 0 || n_atoms <= 0 || n_atoms > 256 || !q ||
        !sg || !ep || (n_poses > 0 && (!pose_xyz || !out)) || (exclusion != 0 && exclusion != 1))
        return FFTDG_E_INVALID;
    if (n_poses == 0) return FFTDG_OK;
    if (hipSetDevice(device) != hipSuccess) return FFTDG_E_DEVICE;
    if (launch_pair_energies((hipStream_t)stream, n_rec_atoms, rxyz, rq, rs, re, n_atoms, q, sg, ep, n_poses,
                             pose_xyz, exclusion, out) != hipSuccess)
        return FFTDG_E_DEVICE;
    return FFTDG_OK;
}

}  // extern "C"

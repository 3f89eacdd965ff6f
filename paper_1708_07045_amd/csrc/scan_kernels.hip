// gfx950 kernels of the FFT translational scan.
//
// Data path for one ligand configuration (Eqs. 8-9, FFT-based BPMF section):
//   k_lig_fwd_xy  per (channel, ligand z-plane): spread the atoms' weights
//                 (trilinear, Eqs. 4-6) or occupancy balls (Eq. 10) of that
//                 plane straight into registers, R2C FFT along x, C2C FFT
//                 along y, write the half-plane (HBM).  Only planes that hold
//                 ligand data are transformed (z-pruned input).
//   k_zprod       per (tile of z-pencils, configuration): forward FFT along
//                 z, multiply with the receptor spectra and sum the energy
//                 channels (Eq. 9), inverse FFT along z, keep only the valid
//                 z-translations (z-pruned output).
//   k_inv_xy_lse  per (configuration, valid z-translation): inverse FFT along
//                 y then C2R along x; clash mask from the occupancy channel;
//                 max-shifted log-sum-exp, minimum and counts of Eq. 2 over
//                 the plane's box-valid translations.
//   k_merge       per configuration: merge its plane partials.
//   k_reduce      per ligand, FP64: exponential averages over configurations
//                 (Eq. 2) and snapshots (Eq. 13).
// Receptor spectra (Eq. 9, FT(G_R)) are built once per snapshot by
// k_rec_xy + k_rec_z with the same transforms.  k_receptor_grids evaluates
// Eq. 7 and Eq. 10 from receptor atoms in FP64.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/fftdg.h"
#include "fft_device.hpp"
#include "kernels.hpp"
#include "scan_types.hpp"
#include "scan_common.hpp"

namespace fftdg {


// ------------------------------------------------------------------ fills
// A fill produces, for lane n1 of the unit that owns storage rows (r, r+1),
// the real values at x = n1 + R1*n2 of row r (into re) and row r+1 (into im).

template <typename T>
struct EAtom {
    int ax, ay;
    T fx, fy, w;  // w = gamma_ch * (z weight)
};
struct OAtom {
    long long Ux, Uy, remz;  // remz = thr - (2^16 z - Uz)^2 > 0
};

template <typename T, int N>
struct LigEnergyFill {
    const EAtom<T> *list;
    int n, y0;
    // does any atom reach storage rows r or r+1?
    __device__ bool any(int r) const {
        const int ya = y0 + r;
        for (int a = 0; a < n; ++a) {
            const int ay = list[a].ay;
            if (ay + 1 >= ya && ay <= ya + 1) return true;
        }
        return false;
    }
    __device__ void rows(int r, int n1, T *re, T *im, bool live, bool has_b) const {
        constexpr int R1 = Shape<N>::R1, R2 = Shape<N>::R2;
#pragma unroll
        for (int i = 0; i < R2; ++i) re[i] = im[i] = (T)0;
        if (!live) return;
        const int ya = y0 + r, yb = ya + 1;
        for (int a = 0; a < n; ++a) {
            const EAtom<T> e = list[a];
            const T wa = (e.ay == ya) ? (T)1 - e.fy : ((e.ay + 1 == ya) ? e.fy : (T)0);
            T wb = (e.ay == yb) ? (T)1 - e.fy : ((e.ay + 1 == yb) ? e.fy : (T)0);
            if (!has_b) wb = (T)0;
            if (wa == (T)0 && wb == (T)0) continue;
            const T w0 = e.w * ((T)1 - e.fx), w1 = e.w * e.fx;
#pragma unroll
            for (int i = 0; i < R2; ++i) {
                const int x = n1 + R1 * i;
                const T cx = (x == e.ax) ? w0 : ((x == e.ax + 1) ? w1 : (T)0);
                re[i] += wa * cx;
                im[i] += wb * cx;
            }
        }
    }
};

template <typename T, int N>
struct LigOccFill {
    const OAtom *list;
    int n, y0;
    __device__ bool any(int) const { return n > 0; }
    __device__ void rows(int r, int n1, T *re, T *im, bool live, bool has_b) const {
        constexpr int R1 = Shape<N>::R1, R2 = Shape<N>::R2;
#pragma unroll
        for (int i = 0; i < R2; ++i) re[i] = im[i] = (T)0;
        if (!live) return;
        for (int a = 0; a < n; ++a) {
            const OAtom e = list[a];
#pragma unroll
            for (int row = 0; row < 2; ++row) {
                if (row == 1 && !has_b) continue;
                const long long yt = (long long)(y0 + r + row);
                const long long dy = yt * 65536LL - e.Uy;
                const long long rem = e.remz - dy * dy;
                if (rem <= 0) continue;
                const long long s = isqrt_lt(rem);
                const long long xlo = -floordiv(-(e.Ux - s), 65536LL);  // ceil
                const long long xhi = floordiv(e.Ux + s, 65536LL);
                const int span = (int)(xhi - xlo);
                if (span < 0) continue;
                const int xl = (int)xlo & (N - 1);
#pragma unroll
                for (int i = 0; i < R2; ++i) {
                    const int x = n1 + R1 * i;
                    const int d = (x - xl) & (N - 1);
                    if (d <= span) {
                        if (row == 0) re[i] = (T)1; else im[i] = (T)1;
                    }
                }
            }
        }
    }
};

template <typename T, int N, typename Src>
struct DenseFill {
    const Src *plane;  // [n_rec][n_rec] plane of the receptor grid
    int n_rec;
    __device__ bool any(int) const { return true; }
    __device__ void rows(int r, int n1, T *re, T *im, bool live, bool has_b) const {
        constexpr int R1 = Shape<N>::R1, R2 = Shape<N>::R2;
#pragma unroll
        for (int i = 0; i < R2; ++i) {
            const int x = n1 + R1 * i;
            const bool okx = live && x < n_rec;
            re[i] = (okx && r < n_rec) ? (T)plane[r * n_rec + x] : (T)0;
            im[i] = (okx && has_b && r + 1 < n_rec) ? (T)plane[(r + 1) * n_rec + x] : (T)0;
        }
    }
};

// ------------------------------------------------------- xy forward of a plane
// Rows r = 0..Ly-1 of the plane hold data (true y = y0 + r); every other
// row is zero.  Writes the 2-D half spectrum [N][H] (ky, kx) to `out`.
template <typename T, int N, class Fill>
__device__ void xy_forward(const Fill &fill, int y0, int Ly, typename Cx<T>::t *Pl,
                           const typename Cx<T>::t *tw, typename Cx<T>::t *out) {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    constexpr int R1 = G::R1, R2 = G::R2, M = G::M, S = G::S, H = G::H, U = G::U;
    static_assert(N + (R1 - 1) * G::RPAD <= 2 * S && H <= S, "plane layout");
    const int unit = threadIdx.x / R1, n1 = threadIdx.x % R1;
    T re[R2], im[R2];

    // Phase A: x transform of row pairs packed as one complex sequence.
    const int npairs = (Ly + 1) / 2;
    const int rounds_a = (npairs + U - 1) / U;
    for (int rd = 0; rd < rounds_a; ++rd) {
        const int r = 2 * (unit + U * rd);
        const bool inside = r < Ly;
        // a pair of all-zero rows transforms to zeros: skip its FFT
        const bool live = inside && fill.any(r);
        C2 *row = Pl + (inside ? r * S : 0);
        if (inside && !live) {
            for (int k = n1; k <= N / 2; k += R1) {
                row[k] = C2{(T)0, (T)0};
                row[S + k] = C2{(T)0, (T)0};
            }
        }
        if (live) {  // a wavefront whose units all hold zero pairs skips the transform
            fill.rows(r, n1, re, im, live, r + 1 < Ly);
            fft_unit<T, N, false>(re, im, n1, row, 1, tw, live, G::RPAD);
        }
        wave_sync();  // rows r, r+1 are private to this unit during phase A
        if (live) {
#pragma unroll
            for (int i = 0; i < M; ++i)
#pragma unroll
                for (int k1 = 0; k1 < R1; ++k1) row[spec_index<N>(n1, i, k1)] = C2{re[i * R1 + k1], im[i * R1 + k1]};
        }
        wave_sync();
        // unpack Z = A + iB (A, B the spectra of rows r and r+1), k = 0..N/2
        constexpr int Q = (N / 2) / R1 + 1;
        C2 A[Q], B[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int k = n1 + R1 * q;
            if (live && k <= N / 2) {
                const C2 zk = row[k], zn = row[(N - k) & (N - 1)];
                A[q] = C2{(T)0.5 * (zk.x + zn.x), (T)0.5 * (zk.y - zn.y)};
                B[q] = C2{(T)0.5 * (zk.y + zn.y), (T)-0.5 * (zk.x - zn.x)};
            }
        }
        wave_sync();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int k = n1 + R1 * q;
            if (live && k <= N / 2) {
                row[k] = A[q];
                row[S + k] = B[q];
            }
        }
    }
    __syncthreads();

    // Phase B: y transform of columns; kx = 0 and kx = N/2 (both real
    // columns) travel together as column 0.
    constexpr int rounds_b = (N / 2 + U - 1) / U;
    for (int rd = 0; rd < rounds_b; ++rd) {
        const int c = unit + U * rd;
        const bool live = c < N / 2;
#pragma unroll
        for (int i = 0; i < R2; ++i) {
            const int rr = (n1 + R1 * i - y0) & (N - 1);
            re[i] = im[i] = (T)0;
            if (live && rr < Ly) {
                if (c == 0) {
                    re[i] = Pl[rr * S].x;
                    im[i] = Pl[rr * S + N / 2].x;
                } else {
                    const C2 v = Pl[rr * S + c];
                    re[i] = v.x;
                    im[i] = v.y;
                }
            }
        }
        C2 *col = Pl + (live ? c : 0);
        fft_unit<T, N, false, false, true>(re, im, n1, col, S, tw, live);
        wave_sync();  // column c (and column N/2 for c = 0) is private to this unit
        if (live) {
#pragma unroll
            for (int i = 0; i < M; ++i)
#pragma unroll
                for (int k1 = 0; k1 < R1; ++k1) col[spec_index<N>(n1, i, k1) * S] = C2{re[i * R1 + k1], im[i * R1 + k1]};
        }
        wave_sync();
        constexpr int QY = N / R1;
        C2 F0[QY], F1[QY];
        const bool unpack = live && c == 0;
#pragma unroll
        for (int q = 0; q < QY; ++q) {
            if (unpack) {
                const int ky = n1 + R1 * q;
                const C2 x1 = Pl[ky * S], x2 = Pl[((N - ky) & (N - 1)) * S];
                F0[q] = C2{(T)0.5 * (x1.x + x2.x), (T)0.5 * (x1.y - x2.y)};
                F1[q] = C2{(T)0.5 * (x1.y + x2.y), (T)-0.5 * (x1.x - x2.x)};
            }
        }
        wave_sync();
#pragma unroll
        for (int q = 0; q < QY; ++q) {
            if (unpack) {
                const int ky = n1 + R1 * q;
                Pl[ky * S] = F0[q];
                Pl[ky * S + N / 2] = F1[q];
            }
        }
    }
    __syncthreads();

    // Phase C: store [ky][kx] contiguously.
    plane_copy<T, N, false>(Pl, out);
}

// ------------------------------------------------------------------ kernels
// Energy planes by direct evaluation (forward mode 2): one block per
// (configuration, energy plane z) writes the half spectra of all three
// channels.  A trilinearly spread atom has 2 x 2 corners in the plane, so
// its 2-D DFT factorises:
//   F(ky, kx) = w^(kx ax) ((1-fx) + fx w^kx) * w^(ky ay) ((1-fy) + fy w^ky)
// (w = exp(-2 pi i / N)), scaled by gamma_ch times its z weight; the plane's
// spectrum is the sum over the few atoms that touch it.  Per-atom factors
// are tabulated in LDS (de_atoms<N>() atoms per pass, as many as fit in the
// plane buffer the FFT path uses); with more atoms the passes accumulate in
// the output.  This is the xy FFT of the spread plane with its zero inputs
// pruned, exact in exact arithmetic.
template <int N>
__host__ __device__ constexpr int de_atoms() {
    // X [a][N/2+1] and Y [a][N] tables must fit in the N x S plane buffer
    return (N * Geo<float, N>::S) / (N / 2 + 1 + N) < 32 ? (N * Geo<float, N>::S) / (N / 2 + 1 + N) : 32;
}

// tab holds DE_A * (N/2 + 1 + N) complex values.
template <typename T, int N, int DE_A>
__device__ void energy_plane_direct(const CfgDev &c, int p, const int32_t *__restrict__ ulat,
                                    const T *__restrict__ gam, const typename Cx<T>::t *tw,
                                    typename Cx<T>::t *tab, typename Cx<T>::t *__restrict__ ws) {
    using C2 = typename Cx<T>::t;
    constexpr int H = N / 2 + 1, NP = N * H;
    static_assert(DE_A >= 1, "at least one atom per pass");
    __shared__ T wgt[DE_A][3];
    __shared__ int2 axy[DE_A];
    __shared__ T fxy[DE_A][2];
    __shared__ int nsel;
    __shared__ int list[MAXA];
    const int zt = c.ze0 + p;
    // atoms touching plane zt, in atom order
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int base = 0;
        for (int a0 = 0; a0 < c.n_atoms; a0 += 64) {
            const int a = a0 + lane;
            bool take = false;
            if (a < c.n_atoms) {
                const int az = ulat[3 * (c.u_base + a) + 2] >> 16;
                take = (az == zt) || (az + 1 == zt);
            }
            const unsigned long long m = __ballot(take);
            if (take) list[base + __popcll(m & ((1ULL << lane) - 1ULL))] = a;
            base += __popcll(m);
        }
        if (lane == 0) nsel = base;
    }
    __syncthreads();
    const int na = nsel;
    C2 *X = tab, *Y = tab + DE_A * H;
    C2 *out0 = ws + c.off_fwd + (int64_t)p * NP;
    const int64_t chs = (int64_t)c.Le * NP;  // channel stride of the forward planes
    for (int a0 = 0; a0 < na || a0 == 0; a0 += DE_A) {
        const int nb = min(DE_A, na - a0);
        if (threadIdx.x < nb) {
            const int a = list[a0 + threadIdx.x];
            const int32_t *U = ulat + 3 * (c.u_base + a);
            const int az = U[2] >> 16;
            const T fz = (T)(U[2] & 0xffff) * (T)(1.0 / 65536.0);
            const T wz = (az == zt) ? (T)1 - fz : fz;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) wgt[threadIdx.x][ch] = gam[3 * (c.atom_base + a) + ch] * wz;
            axy[threadIdx.x] = int2{U[0] >> 16, U[1] >> 16};
            fxy[threadIdx.x][0] = (T)(U[0] & 0xffff) * (T)(1.0 / 65536.0);
            fxy[threadIdx.x][1] = (T)(U[1] & 0xffff) * (T)(1.0 / 65536.0);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nb * (H + N); e += NT) {
            const int a = e / (H + N), k = e - a * (H + N);
            const bool isx = k < H;
            const int kk = isx ? k : k - H;
            const int ax = isx ? axy[a].x : axy[a].y;
            const T f = isx ? fxy[a][0] : fxy[a][1];
            const C2 e1 = tw[(kk * ax) & (N - 1)], wk = tw[kk & (N - 1)];
            const T sr = (T)1 - f + f * wk.x, si = f * wk.y;
            const C2 v = C2{e1.x * sr - e1.y * si, e1.x * si + e1.y * sr};
            if (isx) X[a * H + kk] = v; else Y[a * N + kk] = v;
        }
        __syncthreads();
        for (int o = threadIdx.x; o < NP; o += NT) {
            const int ky = o / H, kx = o - ky * H;
            T ar[3] = {(T)0, (T)0, (T)0}, ai[3] = {(T)0, (T)0, (T)0};
            for (int a = 0; a < nb; ++a) {
                const C2 x = X[a * H + kx], y = Y[a * N + ky];
                const T vr = x.x * y.x - x.y * y.y, vi = x.x * y.y + x.y * y.x;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) {
                    ar[ch] += wgt[a][ch] * vr;
                    ai[ch] += wgt[a][ch] * vi;
                }
            }
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                C2 *dst = out0 + ch * chs + o;
                if (a0 > 0) {
                    const C2 prev = *dst;
                    ar[ch] += prev.x;
                    ai[ch] += prev.y;
                }
                *dst = C2{ar[ch], ai[ch]};
            }
        }
        __syncthreads();
        if (na == 0) break;
    }
}

// Atoms of one configuration that touch plane zt of a channel, compacted in
// atom order by the first wavefront: energy channel ch -> (ax, ay, fx, fy,
// gamma_ch * z weight); occupancy -> lattice x, y and the squared radius left
// after the z offset.  nl receives the count.
template <typename T>
__device__ void gather_plane_atoms(const CfgDev &c, bool occ, int zt, int ch, const int32_t *__restrict__ ulat,
                                   const T *__restrict__ gam, const double *__restrict__ thr, EAtom<T> *Le,
                                   OAtom *Lo, int &nl) {
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        int base = 0;
        for (int a0 = 0; a0 < c.n_atoms; a0 += 64) {
            const int a = a0 + lane;
            bool take = false;
            EAtom<T> ea{};
            OAtom oa{};
            if (a < c.n_atoms) {
                const int32_t *U = ulat + 3 * (c.u_base + a);
                if (!occ) {
                    const int az = U[2] >> 16;
                    const T fz = (T)(U[2] & 0xffff) * (T)(1.0 / 65536.0);
                    take = (az == zt) || (az + 1 == zt);
                    const T wz = (az == zt) ? (T)1 - fz : fz;
                    ea.ax = U[0] >> 16;
                    ea.ay = U[1] >> 16;
                    ea.fx = (T)(U[0] & 0xffff) * (T)(1.0 / 65536.0);
                    ea.fy = (T)(U[1] & 0xffff) * (T)(1.0 / 65536.0);
                    ea.w = gam[3 * (c.atom_base + a) + ch] * wz;
                } else {
                    const long long dz = (long long)zt * 65536LL - U[2];
                    const long long remz = (long long)thr[c.atom_base + a] - dz * dz;
                    take = remz > 0;
                    oa.Ux = U[0];
                    oa.Uy = U[1];
                    oa.remz = remz;
                }
            }
            const unsigned long long m = __ballot(take);
            const int pos = base + __popcll(m & ((1ULL << lane) - 1ULL));
            if (take) {
                if (!occ) Le[pos] = ea; else Lo[pos] = oa;
            }
            base += __popcll(m);
        }
        if (lane == 0) nl = base;
    }
}

template <typename T, int N, bool EDF>
__global__ __launch_bounds__(NT) void k_lig_fwd_xy(const int32_t *__restrict__ fwd_off, int n_cfg,
                                                    const CfgDev *__restrict__ cfgs,
                                                    const int32_t *__restrict__ ulat,
                                                    const T *__restrict__ gam,
                                                    const double *__restrict__ thr,
                                                    const typename Cx<T>::t *__restrict__ twg,
                                                    typename Cx<T>::t *__restrict__ ws) {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    __shared__ C2 Pl[N * G::S];
    __shared__ C2 tw[N];
    __shared__ union {
        EAtom<T> e[MAXA];
        OAtom o[MAXA];
    } L;
    __shared__ int nl;
    const int ic = find_cfg(fwd_off, n_cfg, (int)blockIdx.x);
    const CfgDev c = cfgs[ic];
    const int item = (int)blockIdx.x - fwd_off[ic];
    load_tw<T, N>(tw, twg);
    if constexpr (EDF) {
        if (item < c.Le) {  // block-uniform: the whole block takes this path
            __syncthreads();
            constexpr int DEA = de_atoms<N>();
            static_assert(DEA * (N / 2 + 1 + N) <= N * G::S, "per-atom tables must fit the plane buffer");
            energy_plane_direct<T, N, DEA>(c, item, ulat, gam, tw, Pl, ws);
            return;
        }
    }
    // forward-plane slot in the workspace (energy planes ch * Le + p, then
    // the occupancy planes from occ_slot0)
    const int slot = EDF ? c.occ_slot0 + (item - c.Le) : item;
    const bool occ = slot >= c.occ_slot0;
    struct {
        int ch, p;
    } it = {occ ? 3 : slot / c.Le, occ ? slot - c.occ_slot0 : slot % c.Le};
    const int zt = (occ ? c.zo0 : c.ze0) + it.p;
    const int y0 = occ ? c.yo0 : c.ye0;
    const int Ly = occ ? c.Lyo : c.Lye;
    gather_plane_atoms<T>(c, occ, zt, it.ch, ulat, gam, thr, L.e, L.o, nl);
    __syncthreads();
    C2 *out = ws + c.off_fwd + (int64_t)slot * G::NP;
    if (occ) {
        LigOccFill<T, N> f{L.o, nl, y0};
        xy_forward<T, N>(f, y0, Ly, Pl, tw, out);
    } else {
        LigEnergyFill<T, N> f{L.e, nl, y0};
        xy_forward<T, N>(f, y0, Ly, Pl, tw, out);
    }
}

// Receptor xy pass: block b -> (channel, z) over n_ch * n_rec planes.
template <typename T, int N>
__global__ __launch_bounds__(NT) void k_rec_xy(const T *__restrict__ grids, const uint8_t *__restrict__ occ,
                                                int n_rec, const typename Cx<T>::t *__restrict__ twg,
                                                typename Cx<T>::t *__restrict__ rxy) {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    __shared__ C2 Pl[N * G::S];
    __shared__ C2 tw[N];
    load_tw<T, N>(tw, twg);
    __syncthreads();
    const int ch = blockIdx.x / n_rec, z = blockIdx.x % n_rec;
    const int64_t n2 = (int64_t)n_rec * n_rec;
    C2 *out = rxy + ((int64_t)ch * n_rec + z) * G::NP;
    if (ch < 3) {
        DenseFill<T, N, T> f{grids + (int64_t)ch * n2 * n_rec + z * n2, n_rec};
        xy_forward<T, N>(f, 0, n_rec, Pl, tw, out);
    } else {
        DenseFill<T, N, uint8_t> f{occ + z * n2, n_rec};
        xy_forward<T, N>(f, 0, n_rec, Pl, tw, out);
    }
}

// Receptor z pass: block b -> (channel, tile of pencils); all N outputs kept.
template <typename T, int N>
__global__ __launch_bounds__(NT) void k_rec_z(const typename Cx<T>::t *__restrict__ rxy, int n_rec, int n_tiles,
                                               const typename Cx<T>::t *__restrict__ twg,
                                               typename Cx<T>::t *__restrict__ rspec) {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    constexpr int R1 = G::R1, R2 = G::R2, M = G::M, P = G::U;
    __shared__ C2 buf[4 * G::WREG];
    __shared__ C2 tw[N];
    load_tw<T, N>(tw, twg);
    __syncthreads();
    const int ch = blockIdx.x / n_tiles, tile = blockIdx.x % n_tiles;
    const ZLane<N> zl;
    const int n1 = zl.n1;
    C2 *ex = buf + zl.w * G::WREG + zl.pl;
    const int pen = tile * P + zl.p;
    const bool ok = pen < G::NP;
    T re[R2], im[R2];
#pragma unroll
    for (int i = 0; i < R2; ++i) {
        const int z = n1 + R1 * i;
        re[i] = im[i] = (T)0;
        if (ok && z < n_rec) {
            const C2 v = rxy[((int64_t)ch * n_rec + z) * G::NP + pen];
            re[i] = v.x;
            im[i] = v.y;
        }
    }
    fft_unit<T, N, false>(re, im, n1, ex, G::PW, tw, true, G::PAD);
    if (ok) {
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) {
                const int k = spec_index<N>(n1, i, k1);
                rspec[(int64_t)ch * N * G::NP + G::rs_index(k, pen)] = C2{re[i * R1 + k1], im[i * R1 + k1]};
            }
    }
}

// ------------------------------------------------ split-plane xy transforms
// For an FFT size whose half plane does not fit in LDS (N = 256: a 256 x 129
// complex plane is 264 KB), the xy transforms run as separate passes over
// planes in global memory.  Each FFT unit (R1 lanes) owns a private LDS
// exchange region.  The column passes work in place: a unit reads its whole
// column into registers before it writes the column back.
template <typename T, int N>
struct Split {
    static constexpr int R1 = Shape<N>::R1, R2 = Shape<N>::R2, M = R2 / R1;
    static constexpr int H = N / 2 + 1, NP = N * H, U = NT / R1;
    static constexpr int XPAD = 1;                // pad per block of R2 in a region
    static constexpr int XREG = N + R1 * XPAD;    // complex per unit region
    __device__ static int rg(int k) { return k + (k / R2) * XPAD; }
};

// Row pass of a forward plane: x transform (R2C) of the rows r in [0, Ly)
// that a fill produces, as packed row pairs; the half spectrum of spatial row
// y0 + r is written to row (y0 + r) mod N of `plane` ([N][H]).  Other rows
// are not written (the column pass reads them as zero).
template <typename T, int N, class Fill>
__device__ void rows_fwd(const Fill &fill, int y0, int Ly, typename Cx<T>::t *reg_all,
                         const typename Cx<T>::t *tw, typename Cx<T>::t *__restrict__ plane) {
    using C2 = typename Cx<T>::t;
    using SG = Split<T, N>;
    constexpr int R1 = SG::R1, R2 = SG::R2, M = SG::M, U = SG::U, H = SG::H;
    const int unit = threadIdx.x / R1, n1 = threadIdx.x % R1;
    C2 *reg = reg_all + unit * SG::XREG;
    const int npairs = (Ly + 1) / 2;
    for (int rd = 0; rd < (npairs + U - 1) / U; ++rd) {
        const int r = 2 * (unit + U * rd);
        const bool inside = r < Ly;
        const bool has_b = r + 1 < Ly;
        const bool live = inside && fill.any(r);
        T re[R2], im[R2];
        if (live) {
            fill.rows(r, n1, re, im, true, has_b);
            fft_unit<T, N, false>(re, im, n1, reg, 1, tw, true, SG::XPAD);
        }
        wave_sync();
        if (live) {
#pragma unroll
            for (int i = 0; i < M; ++i)
#pragma unroll
                for (int k1 = 0; k1 < R1; ++k1)
                    reg[SG::rg(spec_index<N>(n1, i, k1))] = C2{re[i * R1 + k1], im[i * R1 + k1]};
        }
        wave_sync();
        if (inside) {
            C2 *ra = plane + (int64_t)((y0 + r) & (N - 1)) * H;
            C2 *rb = plane + (int64_t)((y0 + r + 1) & (N - 1)) * H;
            for (int k = n1; k <= N / 2; k += R1) {
                C2 A = C2{(T)0, (T)0}, B = C2{(T)0, (T)0};
                if (live) {
                    const C2 zk = reg[SG::rg(k)], zn = reg[SG::rg((N - k) & (N - 1))];
                    A = C2{(T)0.5 * (zk.x + zn.x), (T)0.5 * (zk.y - zn.y)};
                    B = C2{(T)0.5 * (zk.y + zn.y), (T)-0.5 * (zk.x - zn.x)};
                }
                ra[k] = A;
                if (has_b) rb[k] = B;
            }
        }
        wave_sync();  // the region is reused by the next round
    }
}

// Column pass over a tile of CT = U consecutive columns of a plane ([N][H]
// in global memory), one column per FFT unit: the tile is staged through LDS
// with coalesced row reads and writes, and each unit transforms its column
// in place in the tile (the column doubles as its exchange area).  Forward:
// rows outside the window y0 .. y0+Ly-1 (mod N) read as zero and all N rows
// are written; inverse: every row is read and rows y < rows_out written.
template <typename T, int N>
struct Tile {
    static constexpr int CT = NT / Shape<N>::R1;  // columns per tile (one per unit)
    static constexpr int TS = CT + 1;             // LDS row stride (complex)
    static constexpr int NTILE = (N / 2 + 1 + CT - 1) / CT;
};

template <typename T, int N, bool INV>
__device__ void cols_tile(typename Cx<T>::t *__restrict__ plane, int tile, int y0, int Ly, int rows_out,
                          typename Cx<T>::t *tb, const typename Cx<T>::t *tw) {
    using C2 = typename Cx<T>::t;
    constexpr int R1 = Shape<N>::R1, R2 = Shape<N>::R2, M = R2 / R1, H = N / 2 + 1;
    constexpr int CT = Tile<T, N>::CT, TS = Tile<T, N>::TS;
    const int c0 = tile * CT;
    for (int e = threadIdx.x; e < N * CT; e += NT) {
        const int row = e / CT, cc = e - row * CT, col = c0 + cc;
        C2 v = C2{(T)0, (T)0};
        if (col < H && (INV || ((row - y0) & (N - 1)) < Ly)) v = plane[(int64_t)row * H + col];
        tb[row * TS + cc] = v;
    }
    __syncthreads();
    const int unit = threadIdx.x / R1, n1 = threadIdx.x % R1;
    const bool live = c0 + unit < H;
    C2 *colp = tb + unit;
    T re[R2], im[R2];
#pragma unroll
    for (int i = 0; i < R2; ++i) {
        const C2 v = colp[(n1 + R1 * i) * TS];
        re[i] = v.x;
        im[i] = v.y;
    }
    fft_unit<T, N, INV, false, true>(re, im, n1, colp, TS, tw, live);
    wave_sync();  // the column is private to this unit
    if (live) {
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) colp[spec_index<N>(n1, i, k1) * TS] = C2{re[i * R1 + k1], im[i * R1 + k1]};
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows_out * CT; e += NT) {
        const int row = e / CT, cc = e - row * CT, col = c0 + cc;
        if (col < H) plane[(int64_t)row * H + col] = tb[row * TS + cc];
    }
}

// Ligand forward planes, row pass (one block per forward item, as
// k_lig_fwd_xy).  With EDF the energy items are evaluated directly here
// (final planes; the column pass skips them).
template <typename T, int N, bool EDF>
__global__ __launch_bounds__(NT) void k_fwd_rows(const int32_t *__restrict__ fwd_off, int n_cfg,
                                                  const CfgDev *__restrict__ cfgs, const int32_t *__restrict__ ulat,
                                                  const T *__restrict__ gam, const double *__restrict__ thr,
                                                  const typename Cx<T>::t *__restrict__ twg,
                                                  typename Cx<T>::t *__restrict__ ws) {
    using C2 = typename Cx<T>::t;
    using SG = Split<T, N>;
    __shared__ C2 reg[SG::U * SG::XREG];
    __shared__ C2 tw[N];
    __shared__ union {
        EAtom<T> e[MAXA];
        OAtom o[MAXA];
    } L;
    __shared__ int nl;
    const int ic = find_cfg(fwd_off, n_cfg, (int)blockIdx.x);
    const CfgDev c = cfgs[ic];
    const int item = (int)blockIdx.x - fwd_off[ic];
    load_tw<T, N>(tw, twg);
    if constexpr (EDF) {
        if (item < c.Le) {
            __syncthreads();
            constexpr int DEA = (SG::U * SG::XREG) / (SG::H + N);
            energy_plane_direct<T, N, DEA>(c, item, ulat, gam, tw, reg, ws);
            return;
        }
    }
    const int slot = EDF ? c.occ_slot0 + (item - c.Le) : item;
    const bool occ = slot >= c.occ_slot0;
    const int ch = occ ? 3 : slot / c.Le, p = occ ? slot - c.occ_slot0 : slot % c.Le;
    const int zt = (occ ? c.zo0 : c.ze0) + p;
    const int y0 = occ ? c.yo0 : c.ye0;
    const int Ly = occ ? c.Lyo : c.Lye;
    gather_plane_atoms<T>(c, occ, zt, ch, ulat, gam, thr, L.e, L.o, nl);
    __syncthreads();
    C2 *out = ws + c.off_fwd + (int64_t)slot * SG::NP;
    if (occ) {
        LigOccFill<T, N> f{L.o, nl, y0};
        rows_fwd<T, N>(f, y0, Ly, reg, tw, out);
    } else {
        LigEnergyFill<T, N> f{L.e, nl, y0};
        rows_fwd<T, N>(f, y0, Ly, reg, tw, out);
    }
}

template <typename T, int N, bool EDF>
__global__ __launch_bounds__(NT) void k_fwd_cols(const int32_t *__restrict__ fwd_off, int n_cfg,
                                                  const CfgDev *__restrict__ cfgs,
                                                  const typename Cx<T>::t *__restrict__ twg,
                                                  typename Cx<T>::t *__restrict__ ws) {
    using C2 = typename Cx<T>::t;
    using TL = Tile<T, N>;
    __shared__ C2 tb[N * TL::TS];
    __shared__ C2 tw[N];
    const int lb = xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int bi = lb / TL::NTILE, tile = lb % TL::NTILE;
    const int ic = find_cfg(fwd_off, n_cfg, bi);
    const CfgDev c = cfgs[ic];
    const int item = bi - fwd_off[ic];
    if (EDF && item < c.Le) return;  // written whole by the row pass
    load_tw<T, N>(tw, twg);
    const int slot = EDF ? c.occ_slot0 + (item - c.Le) : item;
    const bool occ = slot >= c.occ_slot0;
    cols_tile<T, N, false>(ws + c.off_fwd + (int64_t)slot * Geo<T, N>::NP, tile, occ ? c.yo0 : c.ye0,
                           occ ? c.Lyo : c.Lye, N, tb, tw);
}

// Receptor planes: row pass and in-place column pass; block -> (channel, z).
template <typename T, int N>
__global__ __launch_bounds__(NT) void k_rec_rows(const T *__restrict__ grids, const uint8_t *__restrict__ occ,
                                                  int n_rec, const typename Cx<T>::t *__restrict__ twg,
                                                  typename Cx<T>::t *__restrict__ rxy) {
    using C2 = typename Cx<T>::t;
    using SG = Split<T, N>;
    __shared__ C2 reg[SG::U * SG::XREG];
    __shared__ C2 tw[N];
    load_tw<T, N>(tw, twg);
    __syncthreads();
    const int ch = blockIdx.x / n_rec, z = blockIdx.x % n_rec;
    const int64_t n2 = (int64_t)n_rec * n_rec;
    C2 *out = rxy + ((int64_t)ch * n_rec + z) * SG::NP;
    if (ch < 3) {
        DenseFill<T, N, T> f{grids + (int64_t)ch * n2 * n_rec + z * n2, n_rec};
        rows_fwd<T, N>(f, 0, n_rec, reg, tw, out);
    } else {
        DenseFill<T, N, uint8_t> f{occ + z * n2, n_rec};
        rows_fwd<T, N>(f, 0, n_rec, reg, tw, out);
    }
}

template <typename T, int N>
__global__ __launch_bounds__(NT) void k_rec_cols(int n_rec, const typename Cx<T>::t *__restrict__ twg,
                                                  typename Cx<T>::t *__restrict__ rxy) {
    using C2 = typename Cx<T>::t;
    using TL = Tile<T, N>;
    __shared__ C2 tb[N * TL::TS];
    __shared__ C2 tw[N];
    load_tw<T, N>(tw, twg);
    const int plane = (int)blockIdx.x / TL::NTILE, tile = (int)blockIdx.x % TL::NTILE;
    cols_tile<T, N, false>(rxy + (int64_t)plane * Geo<T, N>::NP, tile, 0, n_rec, N, tb, tw);
}


// Placed ligand atom as the fused energy transform uses it.
template <typename T>
struct DAtom {
    int ax, ay, az;
    T fx, fy, fz;
    T g[3];
};

// z pass of the scan.  Block -> (tile of z-pencils, configuration) with an
// XCD-aware order: blocks land on the 8 XCDs round-robin, so block b is
// given the logical index (b % 8) * (nb / 8) + b / 8 and each XCD sweeps a
// contiguous range of tiles, all configurations of a tile back to back,
// keeping its share of the receptor spectra in its own L2.
//
// Energy channels: with EDIRECT the x and y transforms of each ligand plane
// are evaluated here, per atom, as the DFT of its trilinear corners:
//   sum_{dx,dy} w_dx w_dy w^(kx (ax+dx) + ky (ay+dy))
//     = w^(kx ax) ((1-fx) + fx w^kx) * w^(ky ay) ((1-fy) + fy w^ky)
// (w = exp(-2 pi i / N)), i.e. the xy FFT of the spread plane with its zero
// inputs pruned; only the two planes floor(uz), floor(uz)+1 receive the
// atom, with weights 1-fz and fz.  Without EDIRECT the xy-transformed planes
// come from k_lig_fwd_xy through HBM.  The occupancy channel always comes
// from k_lig_fwd_xy.  Then: forward FFT along z, product with the receptor
// spectra summed over the energy channels (Eq. 9, R * conj(L)), inverse FFT
// along z, store the valid z-translations only.  The ligand's forward
// spectra stay in registers while the product and inverse run for each of
// n_snap receptor snapshots (spectra spec_stride apart, outputs inv_stride
// apart).  The 128-point FP32 long-window instantiation (ZH == 2) is held to
// 3 waves per SIMD (168 VGPRs, no spills), the occupancy of the common one;
// the allocator would otherwise take 172 and leave it at 2.
template <typename T, int N, bool OCC, bool EDIRECT, bool MULTI, int ZH>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu((ZH == 2 && N == 128 && sizeof(T) == 4 && !EDIRECT && !MULTI) ? 3 : 1)))
void k_zprod(const CfgDev *__restrict__ cfgs, const int32_t *__restrict__ zcfg,
                                               int nz, int n_tiles, const typename Cx<T>::t *__restrict__ ws,
                                               const typename Cx<T>::t *__restrict__ rspec,
                                               const typename Cx<T>::t *__restrict__ twg,
                                               typename Cx<T>::t *__restrict__ wsi,
                                               const int32_t *__restrict__ ulat, const T *__restrict__ gam,
                                               int n_snap, int64_t spec_stride, int64_t inv_stride) {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    constexpr int R1 = G::R1, R2 = G::R2, P = G::U, NP = G::NP, H = G::H;
    constexpr int AC = 64;  // atoms per XY table chunk
    constexpr int PW = G::PW, PAD = G::PAD;
    __shared__ C2 buf[4 * G::WREG];
    __shared__ C2 tw[N];
    __shared__ DAtom<T> at[EDIRECT ? MAXA : 1];
    __shared__ C2 xy[EDIRECT ? AC * P : 1];
    const int nb = gridDim.x, b = blockIdx.x;
    const int L = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    if (L >= n_tiles * nz) return;
    const int tile = L / nz, zi = L % nz;
    const CfgDev c = cfgs[zcfg[zi]];
    load_tw<T, N>(tw, twg);
    if (EDIRECT) {
        for (int a = threadIdx.x; a < c.n_atoms; a += NT) {
            const int32_t *U = ulat + 3 * (c.u_base + a);
            DAtom<T> d;
            d.ax = U[0] >> 16;
            d.ay = U[1] >> 16;
            d.az = U[2] >> 16;
            d.fx = (T)(U[0] & 0xffff) * (T)(1.0 / 65536.0);
            d.fy = (T)(U[1] & 0xffff) * (T)(1.0 / 65536.0);
            d.fz = (T)(U[2] & 0xffff) * (T)(1.0 / 65536.0);
            d.g[0] = gam[3 * (c.atom_base + a)];
            d.g[1] = gam[3 * (c.atom_base + a) + 1];
            d.g[2] = gam[3 * (c.atom_base + a) + 2];
            at[a] = d;
        }
    }
    __syncthreads();
    const ZLane<N> zl;
    const int n1 = zl.n1, p = zl.p;
    C2 *wbuf = buf + zl.w * G::WREG;  // this wave's exchange region
    C2 *ex = wbuf + zl.pl;
    const int pen = tile * P + p;
    const bool ok = pen < NP;
    const int rlane = rs_lane<T, N>(n1, ok ? pen : 0);  // receptor offsets, lane part
    const int nchunk = EDIRECT ? (c.n_atoms + AC - 1) / AC : 0;
    // ZH (launch-wide) > 0: every configuration's energy planes lie in
    // [0, N/2), so the upper half of the z inputs is zero: not loaded, first
    // FFT stage pruned.  ZH == 2: some occupancy window is longer than N/2
    // planes (a separate instantiation keeps the common one's registers low).
    constexpr bool half = ZH > 0 && !EDIRECT;
    constexpr bool olong = ZH == 2;
    // element e of this lane's pencil in the wave region
    auto eaddr = [&](int e) { return e * PW + (e / R2) * PAD; };
    if constexpr (!MULTI && half) {
    // Every energy window lies in the lower half of the pencil.  The planes
    // of the next channel (energy channels, then occupancy) are loaded while
    // the current one is transformed.  Energy planes sit at z = ze0 + s.  The
    // occupancy window is loaded from z = 0 instead of z = zo0: the circular
    // correlation of the shifted ligand grid is the wanted one shifted by
    // zo0, C(t) = C'(t + zo0 mod N), so the store takes element z to
    // translation t = z - zo0 mod N.
    //
    // N = 256 (4 pencils per wavefront): a lane's own elements lie in 16
    // planes at 4 pencils each, 32-byte pieces per load.  There the block
    // loads and stores its 16 pencils plane row by plane row instead (thread
    // (r, q): pencil q, planes r + 16 i; each plane row 128 contiguous bytes)
    // and transposes through LDS (the wavefronts' exchange regions, between
    // block barriers).
    constexpr int HZ = R2 / 2;
    constexpr bool STG = N == 256;
    constexpr int SQ = P + 1;  // LDS row stride of the staging transpose (complex)
    static_assert(!STG || (P == 16 && NT == 256 && N * SQ <= 4 * G::WREG), "staging layout");
    const int po = ok ? pen : NP * N;
    const int sr = threadIdx.x / P, sq = threadIdx.x % P;            // staging: plane row, pencil
    const int spo = (tile * P + sq < NP) ? tile * P + sq : NP * N;  // out of every descriptor's range
    C2 pf[HZ];
    auto fetch = [&](int ch) {
        const int lz = STG ? sr : n1, lp = STG ? spo : po;
        if (ch < 3) {
            const auto rs = make_rsrc(ws + c.off_fwd + (int64_t)ch * c.Le * NP, c.Le * NP * (int)sizeof(C2));
#pragma unroll
            for (int i = 0; i < HZ; ++i) {
                const int s = (lz + R1 * i - c.ze0) & (N - 1);
                pf[i] = buf_load(rs, (s * NP + lp) * (int)sizeof(C2), (C2 *)nullptr);
            }
        } else {
            const auto rs = make_rsrc(ws + c.off_fwd + (int64_t)c.occ_slot0 * NP, c.Lo * NP * (int)sizeof(C2));
#pragma unroll
            for (int i = 0; i < HZ; ++i)
                pf[i] = buf_load(rs, ((lz + R1 * i) * NP + lp) * (int)sizeof(C2), (C2 *)nullptr);
        }
    };
    // the prefetched planes into this lane's registers (lower half), upper half zero
    auto take = [&](T *re, T *im) {
        if constexpr (STG) {
            __syncthreads();  // every wavefront is done with its exchange region
#pragma unroll
            for (int i = 0; i < HZ; ++i) buf[(sr + R1 * i) * SQ + sq] = pf[i];
            __syncthreads();
#pragma unroll
            for (int i = 0; i < HZ; ++i) {
                const C2 v = buf[(n1 + R1 * i) * SQ + p];
                re[i] = v.x;
                im[i] = v.y;
            }
            __syncthreads();  // read before the exchange regions are reused
        } else {
#pragma unroll
            for (int i = 0; i < HZ; ++i) {
                re[i] = pf[i].x;
                im[i] = pf[i].y;
            }
        }
#pragma unroll
        for (int i = HZ; i < R2; ++i) re[i] = im[i] = (T)0;
    };
    // store this lane's transform outputs (element z = n1 + R1 i) at
    // translation (z - z0) mod N of an inverse region of Vz planes
    auto put = [&](const T *re, const T *im, C2 *dst, int Vzz, int z0) {
        const auto rd = make_rsrc(dst, Vzz * NP * (int)sizeof(C2));
        if constexpr (STG) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < R2; ++i) buf[(n1 + R1 * i) * SQ + p] = C2{re[i], im[i]};
            __syncthreads();
#pragma unroll
            for (int i = 0; i < R2; ++i) {
                const int z = sr + R1 * i, t = (z - z0) & (N - 1);
                buf_store(rd, (t * NP + spo) * (int)sizeof(C2), buf[z * SQ + sq]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < R2; ++i) {
                const int t = (n1 + R1 * i - z0) & (N - 1);
                buf_store(rd, (t * NP + po) * (int)sizeof(C2), C2{re[i], im[i]});
            }
        }
    };
    T er[R2], ei[R2];
#pragma unroll
    for (int i = 0; i < R2; ++i) er[i] = ei[i] = (T)0;
    fetch(0);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        T re[R2], im[R2];
        take(re, im);
        if (ch < 2 || OCC) fetch(ch + 1);
        fft_unit<T, N, false, true>(re, im, n1, ex, PW, tw, true, PAD);
        rprod<T, N, true>(make_rsrc(rspec + (int64_t)ch * N * NP, N * NP * (int)sizeof(C2)), rlane, re, im, er, ei);
    }
    const int Vz = c.V[2];
    fft_unit_rev<T, N, true>(er, ei, n1, ex, PW, tw, true, PAD);
    // valid z-translations only: tz >= Vz lies beyond the descriptor
    put(er, ei, wsi + c.off_inv, Vz, 0);
    // the energy stores are issued before any occupancy work is scheduled
    __builtin_amdgcn_sched_barrier(0);
    if (OCC) {
        T re[R2], im[R2];
        take(re, im);
        if (!olong || c.Lo <= N / 2) {
            fft_unit<T, N, false, true>(re, im, n1, ex, PW, tw, true, PAD);
        } else {
            // a window longer than half the pencil: its upper planes now
            const auto rs = make_rsrc(ws + c.off_fwd + (int64_t)c.occ_slot0 * NP, c.Lo * NP * (int)sizeof(C2));
#pragma unroll
            for (int i = HZ; i < R2; ++i) {
                const C2 v = buf_load(rs, ((n1 + R1 * i) * NP + po) * (int)sizeof(C2), (C2 *)nullptr);
                re[i] = v.x;
                im[i] = v.y;
            }
            fft_unit<T, N, false>(re, im, n1, ex, PW, tw, true, PAD);
        }
        rprod<T, N, false>(make_rsrc(rspec + (int64_t)3 * N * NP, N * NP * (int)sizeof(C2)), rlane, re, im, nullptr,
                           nullptr);
        fft_unit_rev<T, N, true>(re, im, n1, ex, PW, tw, true, PAD);
        put(re, im, wsi + c.off_inv + (int64_t)Vz * NP, Vz, c.zo0);
    }
    } else if constexpr (!MULTI) {
    T er[R2], ei[R2];
#pragma unroll
    for (int i = 0; i < R2; ++i) er[i] = ei[i] = (T)0;
#pragma unroll 1
    for (int ch = 0; ch < 3; ++ch) {
        T re[R2], im[R2];
#pragma unroll
        for (int i = 0; i < R2; ++i) re[i] = im[i] = (T)0;
        if (EDIRECT) {
            // Lane (n1, p) owns the z-planes n1 + R1*i of pencil p in its wave region.
            wave_sync();  // previous exchange reads of the region are done
#pragma unroll
            for (int i = 0; i < R2; ++i) ex[eaddr(n1 + R1 * i)] = C2{(T)0, (T)0};
            for (int ck = 0; ck < nchunk; ++ck) {
                const int a0 = ck * AC, na = min(AC, c.n_atoms - a0);
                if (ch == 0 || nchunk > 1) {
                    if (nchunk > 1) __syncthreads();
                    // XY[a][p] = w^(kx ax)((1-fx) + fx w^kx) * w^(ky ay)((1-fy) + fy w^ky)
                    for (int e = threadIdx.x; e < na * P; e += NT) {
                        const int a = e / P, q = e - a * P;
                        const int pq = tile * P + q;
                        const int kyq = pq / H, kxq = pq - kyq * H;
                        const DAtom<T> d = at[a0 + a];
                        const C2 wx = tw[kxq & (N - 1)], wy = tw[kyq & (N - 1)];
                        const C2 ex = tw[(kxq * d.ax) & (N - 1)], ey = tw[(kyq * d.ay) & (N - 1)];
                        const T sxr = (T)1 - d.fx + d.fx * wx.x, sxi = d.fx * wx.y;
                        const T syr = (T)1 - d.fy + d.fy * wy.x, syi = d.fy * wy.y;
                        const T xr = ex.x * sxr - ex.y * sxi, xi = ex.x * sxi + ex.y * sxr;
                        const T yr = ey.x * syr - ey.y * syi, yi = ey.x * syi + ey.y * syr;
                        xy[a * P + q] = C2{xr * yr - xi * yi, xr * yi + xi * yr};
                    }
                    __syncthreads();
                }
                for (int a = 0; a < na; ++a) {
                    const DAtom<T> d = at[a0 + a];
                    const int za = d.az, zb = d.az + 1;
                    const bool ha = (za & (R1 - 1)) == n1, hb = (zb & (R1 - 1)) == n1;
                    if (!ha && !hb) continue;
                    const C2 v = xy[a * P + p];
                    const T g = d.g[ch];
                    if (ha) {
                        C2 &t = ex[eaddr(za & (N - 1))];
                        const T w = g * ((T)1 - d.fz);
                        t.x += w * v.x;
                        t.y += w * v.y;
                    }
                    if (hb) {
                        C2 &t = ex[eaddr(zb & (N - 1))];
                        const T w = g * d.fz;
                        t.x += w * v.x;
                        t.y += w * v.y;
                    }
                }
            }
            if (ok) {
#pragma unroll
                for (int i = 0; i < R2; ++i) {
                    const C2 v = ex[eaddr(n1 + R1 * i)];
                    re[i] = v.x;
                    im[i] = v.y;
                }
            }
        } else {
            // planes outside the channel's window lie beyond the descriptor
            // and read as zero
            const auto rs = make_rsrc(ws + c.off_fwd + (int64_t)ch * c.Le * NP, c.Le * NP * (int)sizeof(C2));
            const int po = ok ? pen : NP * N;
#pragma unroll
            for (int i = 0; i < (half ? R2 / 2 : R2); ++i) {
                const int s = (n1 + R1 * i - c.ze0) & (N - 1);
                const C2 v = buf_load(rs, (s * NP + po) * (int)sizeof(C2), (C2 *)nullptr);
                re[i] = v.x;
                im[i] = v.y;
            }
        }
        fft_unit<T, N, false, half>(re, im, n1, ex, PW, tw, true, PAD);
        rprod<T, N, true>(make_rsrc(rspec + (int64_t)ch * N * NP, N * NP * (int)sizeof(C2)), rlane, re, im, er, ei);
    }
    const int Vz = c.V[2];
    const int po = ok ? pen : NP * N;  // out of every descriptor's range
    fft_unit_rev<T, N, true>(er, ei, n1, ex, PW, tw, true, PAD);
    {
        // valid z-translations only: tz >= Vz lies beyond the descriptor
        const auto rd = make_rsrc(wsi + c.off_inv, Vz * NP * (int)sizeof(C2));
#pragma unroll
        for (int i = 0; i < R2; ++i)
            buf_store(rd, ((n1 + R1 * i) * NP + po) * (int)sizeof(C2), C2{er[i], ei[i]});
    }
    if (OCC) {
        T re[R2], im[R2];
        const auto rs = make_rsrc(ws + c.off_fwd + (int64_t)c.occ_slot0 * NP, c.Lo * NP * (int)sizeof(C2));
#pragma unroll
        for (int i = 0; i < R2; ++i) {
            const int s = ((n1 + R1 * i - c.zo0) & (N - 1));
            const C2 v = buf_load(rs, (s * NP + po) * (int)sizeof(C2), (C2 *)nullptr);
            re[i] = v.x;
            im[i] = v.y;
        }
        fft_unit<T, N, false>(re, im, n1, ex, PW, tw, true, PAD);
        rprod<T, N, false>(make_rsrc(rspec + (int64_t)3 * N * NP, N * NP * (int)sizeof(C2)), rlane, re, im, nullptr,
                           nullptr);
        fft_unit_rev<T, N, true>(re, im, n1, ex, PW, tw, true, PAD);
        const auto rd = make_rsrc(wsi + c.off_inv + (int64_t)Vz * NP, Vz * NP * (int)sizeof(C2));
#pragma unroll
        for (int i = 0; i < R2; ++i)
            buf_store(rd, ((n1 + R1 * i) * NP + po) * (int)sizeof(C2), C2{re[i], im[i]});
    }
    } else {
    // forward z transforms of the three energy channels, kept in registers
    // for every snapshot of the group
    T lr[3][R2], li[3][R2];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        T *re = lr[ch], *im = li[ch];
#pragma unroll
        for (int i = 0; i < R2; ++i) re[i] = im[i] = (T)0;
        if (EDIRECT) {
            // Lane (n1, p) owns the z-planes n1 + R1*i of pencil p in its wave region.
            wave_sync();  // previous exchange reads of the region are done
#pragma unroll
            for (int i = 0; i < R2; ++i) ex[eaddr(n1 + R1 * i)] = C2{(T)0, (T)0};
            for (int ck = 0; ck < nchunk; ++ck) {
                const int a0 = ck * AC, na = min(AC, c.n_atoms - a0);
                if (ch == 0 || nchunk > 1) {
                    if (nchunk > 1) __syncthreads();
                    // XY[a][p] = w^(kx ax)((1-fx) + fx w^kx) * w^(ky ay)((1-fy) + fy w^ky)
                    for (int e = threadIdx.x; e < na * P; e += NT) {
                        const int a = e / P, q = e - a * P;
                        const int pq = tile * P + q;
                        const int kyq = pq / H, kxq = pq - kyq * H;
                        const DAtom<T> d = at[a0 + a];
                        const C2 wx = tw[kxq & (N - 1)], wy = tw[kyq & (N - 1)];
                        const C2 ex_ = tw[(kxq * d.ax) & (N - 1)], ey = tw[(kyq * d.ay) & (N - 1)];
                        const T sxr = (T)1 - d.fx + d.fx * wx.x, sxi = d.fx * wx.y;
                        const T syr = (T)1 - d.fy + d.fy * wy.x, syi = d.fy * wy.y;
                        const T xr = ex_.x * sxr - ex_.y * sxi, xi = ex_.x * sxi + ex_.y * sxr;
                        const T yr = ey.x * syr - ey.y * syi, yi = ey.x * syi + ey.y * syr;
                        xy[a * P + q] = C2{xr * yr - xi * yi, xr * yi + xi * yr};
                    }
                    __syncthreads();
                }
                for (int a = 0; a < na; ++a) {
                    const DAtom<T> d = at[a0 + a];
                    const int za = d.az, zb = d.az + 1;
                    const bool ha = (za & (R1 - 1)) == n1, hb = (zb & (R1 - 1)) == n1;
                    if (!ha && !hb) continue;
                    const C2 v = xy[a * P + p];
                    const T g = d.g[ch];
                    if (ha) {
                        C2 &t = ex[eaddr(za & (N - 1))];
                        const T w = g * ((T)1 - d.fz);
                        t.x += w * v.x;
                        t.y += w * v.y;
                    }
                    if (hb) {
                        C2 &t = ex[eaddr(zb & (N - 1))];
                        const T w = g * d.fz;
                        t.x += w * v.x;
                        t.y += w * v.y;
                    }
                }
            }
            if (ok) {
#pragma unroll
                for (int i = 0; i < R2; ++i) {
                    const C2 v = ex[eaddr(n1 + R1 * i)];
                    re[i] = v.x;
                    im[i] = v.y;
                }
            }
        } else {
            // planes outside the channel's window lie beyond the descriptor
            // and read as zero
            const auto rs = make_rsrc(ws + c.off_fwd + (int64_t)ch * c.Le * NP, c.Le * NP * (int)sizeof(C2));
            const int po = ok ? pen : NP * N;
#pragma unroll
            for (int i = 0; i < (half ? R2 / 2 : R2); ++i) {
                const int s = (n1 + R1 * i - c.ze0) & (N - 1);
                const C2 v = buf_load(rs, (s * NP + po) * (int)sizeof(C2), (C2 *)nullptr);
                re[i] = v.x;
                im[i] = v.y;
            }
        }
        fft_unit<T, N, false, half>(re, im, n1, ex, PW, tw, true, PAD);
    }
    const int Vz = c.V[2];
    const int po = ok ? pen : NP * N;  // out of every descriptor's range
#pragma unroll 1
    for (int sn = 0; sn < n_snap; ++sn) {
        T er[R2], ei[R2];
#pragma unroll
        for (int i = 0; i < R2; ++i) er[i] = ei[i] = (T)0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            rprod<T, N, true>(make_rsrc(rspec + sn * spec_stride + (int64_t)ch * N * NP, N * NP * (int)sizeof(C2)),
                              rlane, lr[ch], li[ch], er, ei);
        }
        fft_unit_rev<T, N, true>(er, ei, n1, ex, PW, tw, true, PAD);
        // valid z-translations only: tz >= Vz lies beyond the descriptor
        const auto rd = make_rsrc(wsi + sn * inv_stride + c.off_inv, Vz * NP * (int)sizeof(C2));
#pragma unroll
        for (int i = 0; i < R2; ++i)
            buf_store(rd, ((n1 + R1 * i) * NP + po) * (int)sizeof(C2), C2{er[i], ei[i]});
    }
    if (OCC) {
        T orr[R2], oi[R2];
        const auto rs = make_rsrc(ws + c.off_fwd + (int64_t)c.occ_slot0 * NP, c.Lo * NP * (int)sizeof(C2));
#pragma unroll
        for (int i = 0; i < R2; ++i) {
            const int s = ((n1 + R1 * i - c.zo0) & (N - 1));
            const C2 v = buf_load(rs, (s * NP + po) * (int)sizeof(C2), (C2 *)nullptr);
            orr[i] = v.x;
            oi[i] = v.y;
        }
        fft_unit<T, N, false>(orr, oi, n1, ex, PW, tw, true, PAD);
#pragma unroll 1
        for (int sn = 0; sn < n_snap; ++sn) {
            T re[R2], im[R2];
#pragma unroll
            for (int i = 0; i < R2; ++i) {
                re[i] = orr[i];
                im[i] = oi[i];
            }
            rprod<T, N, false>(make_rsrc(rspec + sn * spec_stride + (int64_t)3 * N * NP, N * NP * (int)sizeof(C2)),
                               rlane, re, im, nullptr, nullptr);
            fft_unit_rev<T, N, true>(re, im, n1, ex, PW, tw, true, PAD);
            const auto rd =
                make_rsrc(wsi + sn * inv_stride + c.off_inv + (int64_t)Vz * NP, Vz * NP * (int)sizeof(C2));
#pragma unroll
            for (int i = 0; i < R2; ++i)
                buf_store(rd, ((n1 + R1 * i) * NP + po) * (int)sizeof(C2), C2{re[i], im[i]});
        }
    }
    }
}


// Inverse xy + clash mask + Eq. 2 partials for one valid z-translation.
// In a scan (no energy export) the energy channel of a plane whose every
// translation clashes is not transformed: those energies are infinite by the
// method and never enter Eq. 2.  e_count counts energy planes transformed.
template <typename T, int N, bool OCC>
__global__ __launch_bounds__(NT) void k_inv_xy_lse(const int32_t *__restrict__ inv_off, int n_cfg,
                                                    const CfgDev *__restrict__ cfgs,
                                                    const typename Cx<T>::t *__restrict__ wsi, T beta, T inv_n3,
                                                    const typename Cx<T>::t *__restrict__ twg,
                                                    PlanePartial<T> *__restrict__ pp, T *__restrict__ psi_out,
                                                    uint8_t *__restrict__ clash_out, unsigned int *__restrict__ e_count) {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    constexpr int R1 = G::R1, R2 = G::R2, M = G::M, S = G::S, U = G::U, NP = G::NP;
    constexpr int MAXR = (N / 2 + U - 1) / U;  // rounds of row pairs
    static_assert(N + (R1 - 1) * G::RPAD <= 2 * S, "row-pair exchange must fit in two rows");
    __shared__ C2 Pl[N * S];
    __shared__ C2 tw[N];
    __shared__ uint32_t cflags[MAXR * NT];  // per thread and round: its outputs not folded in
    __shared__ LseAcc<T> red[NT / 64];
    const int ic = find_cfg(inv_off, n_cfg, (int)blockIdx.x);
    const CfgDev c = cfgs[ic];
    const int Vx = c.V[0], Vy = c.V[1], Vz = c.V[2], tz = (int)blockIdx.x - inv_off[ic];
    load_tw<T, N>(tw, twg);
    const int unit = threadIdx.x / R1, n1 = threadIdx.x % R1;
    LseAcc<T> acc;
    acc.init();
    int any_free = 0;
    constexpr int NCH = OCC ? 2 : 1;
    for (int pass = 0; pass < NCH; ++pass) {
        const int och = OCC ? 1 - pass : 0;  // occupancy first
        const C2 *src = wsi + c.off_inv + ((int64_t)och * Vz + tz) * NP;
        if (OCC && och == 0 && !psi_out) {
            // any clash-free translation on this plane?
            if (!__syncthreads_or(any_free)) break;
        }
        if (och == 0 && threadIdx.x == 0 && e_count) atomicAdd(e_count, 1u);
        __syncthreads();
        plane_copy<T, N, true>(Pl, const_cast<C2 *>(src));
        __syncthreads();
        T re[R2], im[R2];
        // inverse y on columns (kx = 0 and N/2 packed into column 0), keep y < Vy
        constexpr int rounds_b = (N / 2 + U - 1) / U;
        for (int rd = 0; rd < rounds_b; ++rd) {
            const int col = unit + U * rd;
            const bool live = col < N / 2;
            const bool c0 = col == 0;
#pragma unroll
            for (int i = 0; i < R2; ++i) {
                const int ky = n1 + R1 * i;
                re[i] = im[i] = (T)0;
                if (live) {
                    const C2 v = Pl[ky * S + col];
                    const C2 bq = c0 ? Pl[ky * S + N / 2] : C2{(T)0, (T)0};
                    re[i] = v.x - bq.y;
                    im[i] = v.y + bq.x;
                }
            }
            C2 *cp = Pl + (live ? col : 0);
            fft_unit<T, N, true, false, true>(re, im, n1, cp, S, tw, live);
            wave_sync();  // column col (and N/2 for col = 0) is private to this unit
            if (live) {
#pragma unroll
                for (int i = 0; i < M; ++i)
#pragma unroll
                    for (int k1 = 0; k1 < R1; ++k1) {
                        const int y = spec_index<N>(n1, i, k1);
                        if (y < Vy) {
                            if (c0) {
                                Pl[y * S] = C2{re[i * R1 + k1], (T)0};
                                Pl[y * S + N / 2] = C2{im[i * R1 + k1], (T)0};
                            } else {
                                Pl[y * S + col] = C2{re[i * R1 + k1], im[i * R1 + k1]};
                            }
                        }
                    }
            }
        }
        __syncthreads();
        // inverse x (C2R) of row pairs (y, y+1), y < Vy
        const int npairs = (Vy + 1) / 2;
        const int rounds_a = (npairs + U - 1) / U;
        for (int rd = 0; rd < rounds_a; ++rd) {
            const int y = 2 * (unit + U * rd);
            const bool live = y < Vy;
            // energy pass of a scan: a wavefront whose row pairs hold no
            // clash-free valid translation has nothing to add
            if (OCC && och == 0 && !psi_out && !clash_out &&
                !__any(live && cflags[rd * NT + threadIdx.x] != ~0u))
                continue;
            C2 *row = Pl + (live ? y * S : 0);
#pragma unroll
            for (int i = 0; i < R2; ++i) {
                const int k = n1 + R1 * i;
                re[i] = im[i] = (T)0;
                if (live) {
                    // row values at k (k <= N/2) or conj at N - k; kx = 0, N/2 are real
                    const int kk = k <= N / 2 ? k : N - k;
                    C2 a = row[kk], bq = row[S + kk];
                    const T sg = (k == 0 || k == N / 2) ? (T)0 : (k < N / 2 ? (T)1 : (T)-1);
                    a.y *= sg;
                    bq.y *= sg;
                    re[i] = a.x - bq.y;
                    im[i] = a.y + bq.x;
                }
            }
            fft_unit<T, N, true>(re, im, n1, row, 1, tw, live, G::RPAD);
            if (live) {
                // per thread and round: the outputs NOT to fold in (invalid or
                // clashing); written and read by this thread only
                uint32_t &cw = cflags[rd * NT + threadIdx.x];
                uint32_t vb;
                const uint32_t f = row_pair_epilogue<T, N, OCC>(re, im, n1, y, Vx, Vy, tz, OCC && och == 1,
                                                                (OCC && och == 0) ? cw : 0u, inv_n3, beta, psi_out,
                                                                clash_out, acc, vb);
                if (OCC && och == 1) {
                    cw = ~(vb & ~f);
                    any_free |= (vb & ~f) != 0u;
                }
            }
        }
    }
    block_partial_store(acc, red, pp + c.pp_base + tz);
}

// Per configuration: merge its plane partials (fixed order, working precision).
template <typename T>
__global__ void k_merge(const CfgDev *__restrict__ cfgs, int n_cfg, const PlanePartial<T> *__restrict__ pp,
                        fftdg_partial *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_cfg) return;
    const CfgDev c = cfgs[i];
    LseAcc<T> a;
    a.init();
    if (c.scanned) {
        for (int tz = 0; tz < c.V[2]; ++tz) {
            const PlanePartial<T> p = pp[c.pp_base + tz];
            LseAcc<T> b;
            b.m = p.m;
            b.s = p.s;
            b.pmin = p.psi_min;
            b.n = p.n_finite;
            b.amin = p.argmin;
            a.merge(b);
        }
    }
    fftdg_partial o;
    o.m = (double)a.m;
    o.s = (double)a.s;
    o.psi_min = (double)a.pmin;
    o.n_valid = c.n_valid;
    o.n_finite = a.n;
    o.argmin = a.amin;
    o.scanned = c.scanned;
    out[c.global_cfg] = o;
}

// FP64 exponential averages per ligand (one workgroup per ligand).
__global__ __launch_bounds__(NT) void k_reduce(const fftdg_partial *__restrict__ p, int64_t n_cfg_total,
                                                int n_snap, const int32_t *__restrict__ cfg_off,
                                                const double *__restrict__ cfg_w, const double *__restrict__ W,
                                                double kT, double h3, double c0, double *__restrict__ B,
                                                LigRed *__restrict__ res) {
    __shared__ double sd[NT];
    __shared__ long long sl[NT];
    __shared__ long long sf[NT];
    const int lig = blockIdx.x;
    const int c0i = cfg_off[lig], c1i = cfg_off[lig + 1];
    const int t = threadIdx.x;
    double pmin_all = INFINITY;
    long long nfin_all = 0, nsamp = 0;
    double gmax = -INFINITY;
    for (int s = 0; s < n_snap; ++s) {
        const fftdg_partial *ps = p + (int64_t)s * n_cfg_total;
        double mx = -INFINITY;
        long long nv = 0, nf = 0;
        for (int c = c0i + t; c < c1i; c += NT) {
            const fftdg_partial q = ps[c];
            nv += q.n_valid;
            nf += q.n_finite;
            if (q.psi_min < pmin_all) pmin_all = q.psi_min;
            const double w = cfg_w ? cfg_w[c] : 1.0;
            if (q.n_finite > 0 && w > 0.0) {
                const double x = log(w) + q.m + log(q.s);
                if (x > mx) mx = x;
            }
        }
        sd[t] = mx;
        sl[t] = nv;
        sf[t] = nf;
        __syncthreads();
        for (int w = NT / 2; w > 0; w >>= 1) {
            if (t < w) {
                sd[t] = sd[t] > sd[t + w] ? sd[t] : sd[t + w];
                sl[t] += sl[t + w];
                sf[t] += sf[t + w];
            }
            __syncthreads();
        }
        const double M = sd[0];
        const long long NV = sl[0], NF = sf[0];
        __syncthreads();
        double sum = 0.0;
        if (M > -INFINITY) {
            for (int c = c0i + t; c < c1i; c += NT) {
                const fftdg_partial q = ps[c];
                const double w = cfg_w ? cfg_w[c] : 1.0;
                if (q.n_finite > 0 && w > 0.0) sum += exp(log(w) + q.m + log(q.s) - M);
            }
        }
        sd[t] = sum;
        __syncthreads();
        for (int w = NT / 2; w > 0; w >>= 1) {
            if (t < w) sd[t] += sd[t + w];
            __syncthreads();
        }
        if (t == 0) {
            double Bs = INFINITY;
            if (M > -INFINITY && NV > 0) Bs = -kT * (M + log(sd[0]) - log((double)NV));
            B[(int64_t)lig * n_snap + s] = Bs;
            nfin_all += NF;
            nsamp = NV;
        }
        __syncthreads();
    }
    // psi_min over threads
    sd[t] = pmin_all;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w) sd[t] = sd[t] < sd[t + w] ? sd[t] : sd[t + w];
        __syncthreads();
    }
    if (t == 0) {
        const double pm = sd[0];
        // Eq. 13 over snapshots (sequential, n_snap is small)
        for (int s = 0; s < n_snap; ++s) {
            const double Bs = B[(int64_t)lig * n_snap + s];
            if (W[s] > 0.0 && Bs < INFINITY) {
                const double x = log(W[s]) - Bs / kT;
                if (x > gmax) gmax = x;
            }
        }
        double sum = 0.0;
        if (gmax > -INFINITY)
            for (int s = 0; s < n_snap; ++s) {
                const double Bs = B[(int64_t)lig * n_snap + s];
                if (W[s] > 0.0 && Bs < INFINITY) sum += exp(log(W[s]) - Bs / kT - gmax);
            }
        const int ncfg = c1i - c0i;
        const double vs = ncfg > 0 ? h3 * (double)nsamp / (double)ncfg : 0.0;
        LigRed r;
        r.v_site = vs;
        r.dG = (gmax > -INFINITY && vs > 0.0) ? -kT * (gmax + log(sum)) - kT * log(vs * c0) : INFINITY;
        r.psi_min = pm;
        r.n_finite = nfin_all;
        r.n_samples = nsamp;
        res[lig] = r;
    }
}

// A copy of v the compiler cannot see through: index arithmetic derived from
// it is recomputed where it is used instead of being hoisted out of loops and
// held in registers across the whole kernel.
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Whole-plane inverse xy for the split-plane grid: one workgroup of WT = 1024
// threads (64 FFT units of R1 = 16 lanes) per (configuration, valid z), so
// each plane is read from device memory once and nothing is written back.
// Inverse y: columns kx = 1 .. N/2-1 of the half spectrum, and columns 0 and
// N/2 packed as one complex column (both transform to real rows: Re and Im
// of the packed result), N/2 columns in all, staged through LDS in batches of
// 64 by coalesced row reads; each unit reads one column into registers,
// transforms it in a private region of the tile and keeps its outputs, rows
// y = R1 k1 + n1, in registers.  Inverse x (C2R): rows y < Vy are transposed
// through LDS 128 at a time and each unit transforms one row pair (y, y + 1)
// packed as one complex row, its two tile rows doubling as its exchange
// area; then the clash bits, energies and partial as k_inv_xy_lse.
template <bool B>
struct BoolTag {
    static constexpr bool value = B;
};

template <typename T, int N>
struct Whole {
    static constexpr int WT = 1024;
    static constexpr int R1 = Shape<N>::R1, R2 = Shape<N>::R2;
    static constexpr int U = WT / R1;            // units
    static constexpr int H = N / 2 + 1, NP = N * H;
    static constexpr int NHALF = (N / 2) / U;    // column batches of U packed columns
    static constexpr int NRND = N / (2 * U);     // row batches of 2U rows
    static constexpr int KR = R2 / NRND;         // output slots per row batch
    static constexpr int XP = 1;                 // exchange pad per block of R2
    static constexpr int XR = N + R1 * XP;       // exchange region (complex)
    // LDS row strides (complex), odd: the column reads (stride TSA) and the
    // transposing writes (stride TSB) of a unit's 16 lanes fall on distinct
    // banks (an even TSA = U + 4 made them 4-way conflicts: 54.0 -> 50.1 ms
    // per 1000 whole-surface configurations)
    static constexpr int TSA = U + 5, TSB = N / 2 + 9;
    static constexpr int TA = N * TSA > U * XR ? N * TSA : U * XR;
    static constexpr int TILE = TA > 2 * U * TSB ? TA : 2 * U * TSB;
    static_assert(Shape<N>::R2 == Shape<N>::R1, "one output slot per k1");
    static_assert(NHALF * U == N / 2 && NRND * 2 * U == N && KR * NRND == R2, "tiling");
    static_assert(2 * TSB >= XR, "a row pair holds its exchange area");
};

template <typename T, int N, bool OCC>
__global__ __launch_bounds__(1024) void k_inv_plane(const int32_t *__restrict__ inv_off, int n_cfg,
                                                    const CfgDev *__restrict__ cfgs,
                                                    const typename Cx<T>::t *__restrict__ wsi, T beta, T inv_n3,
                                                    const typename Cx<T>::t *__restrict__ twg,
                                                    PlanePartial<T> *__restrict__ pp, T *__restrict__ psi_out,
                                                    uint8_t *__restrict__ clash_out,
                                                    unsigned int *__restrict__ e_count) {
    using C2 = typename Cx<T>::t;
    using W = Whole<T, N>;
    constexpr int R1 = W::R1, R2 = W::R2, U = W::U, H = W::H, WT = W::WT;
    constexpr int NHALF = W::NHALF, NRND = W::NRND, KR = W::KR, TSA = W::TSA, TSB = W::TSB;
    static_assert(WT == 1024, "launch bounds");
    __shared__ C2 tile[W::TILE];
    __shared__ C2 tw2[LaneTw<N>::SIZE];
    __shared__ LseAcc<T> red[WT / 64];
    const int ic = find_cfg(inv_off, n_cfg, (int)blockIdx.x);
    const CfgDev c = cfgs[ic];
    const int Vx = c.V[0], Vy = c.V[1], Vz = c.V[2], tz = (int)blockIdx.x - inv_off[ic];
    if (threadIdx.x < R1 * R2) {  // tw2[n1 S + k2] = w_N^(n1 k2)
        const int a = (int)threadIdx.x / R2, k2 = (int)threadIdx.x % R2;
        tw2[a * LaneTw<N>::S + k2] = twg[a * k2];
    }
    const int unit = threadIdx.x / R1, n1 = threadIdx.x % R1;
    LseAcc<T> acc;
    acc.init();
    int any_free = 0;
    uint32_t cw[NRND];
#pragma unroll
    for (int r = 0; r < NRND; ++r) cw[r] = 0u;
    // one channel of the plane: the occupancy pass (clash bits) or the energies
    auto channel = [&](auto occ_tag) {
        constexpr bool OCC_PASS = decltype(occ_tag)::value;
        const int och = OCC_PASS ? 1 : 0;
        const C2 *src = wsi + c.off_inv + ((int64_t)och * Vz + tz) * W::NP;
        if (!OCC_PASS && threadIdx.x == 0 && e_count) atomicAdd(e_count, 1u);
        // inverse y: column batch hb holds packed columns hb U .. hb U + U - 1
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(src, W::NP * (int)sizeof(C2));
        T cr[NHALF][R2], ci[NHALF][R2];
#pragma unroll
        for (int hb = 0; hb < NHALF; ++hb) {
            // wavefront w stages rows w + (WT/U) j, one row segment of U columns per load
            constexpr int RS = WT / U, NJ = N / RS;
            const int r0 = (int)threadIdx.x / U, cc = (int)threadIdx.x % U;
            const int voff = (r0 * H + hb * U + cc) * (int)sizeof(C2);
            C2 v[NJ];
#pragma unroll
            for (int j = 0; j < NJ; ++j) v[j] = buf_load(rs, voff, j * RS * H * (int)sizeof(C2), (C2 *)nullptr);
            // column N/2, packed into column 0 as its imaginary part: row t by thread t
            C2 q = C2{(T)0, (T)0};
            if (hb == 0 && threadIdx.x < N) q = buf_load(rs, ((int)threadIdx.x * H + N / 2) * (int)sizeof(C2), (C2 *)nullptr);
            __syncthreads();  // the tile's previous readers are done
#pragma unroll
            for (int j = 0; j < NJ; ++j) tile[(r0 + RS * j) * TSA + cc] = v[j];
            __syncthreads();
            if (hb == 0 && threadIdx.x < N) {
                C2 &t0 = tile[threadIdx.x * TSA];
                t0 = C2{t0.x - q.y, t0.y + q.x};
            }
            if (hb == 0) __syncthreads();
            const int m1 = opaque(n1) & (R1 - 1);
            T re[R2], im[R2];
            {
                const C2 *colp = tile + unit + m1 * TSA;
#pragma unroll
                for (int i = 0; i < R2; ++i) {
                    const C2 x = colp[R1 * TSA * i];
                    re[i] = x.x;
                    im[i] = x.y;
                }
            }
            __syncthreads();  // every column is in registers: the tile becomes the units' exchange regions
            fft_unit_lt<T, N, true>(re, im, m1, tile + unit * W::XR, 1, tw2, true, W::XP);
#pragma unroll
            for (int k1 = 0; k1 < R2; ++k1) {  // row y = R1 k1 + n1 of column hb U + unit
                cr[hb][k1] = re[k1];
                ci[hb][k1] = im[k1];
            }
        }
        // inverse x: row batch rd holds rows rd 2U .. rd 2U + 2U - 1.  The
        // next batch is written to the tile as soon as this batch's
        // transforms are done with it, before the epilogue, so its registers
        // are free while the epilogue runs.
        auto put = [&](int rd) {  // the outputs of row batch rd into the tile
            C2 *wp = tile + (opaque(n1) & (R1 - 1)) * TSB + unit;
#pragma unroll
            for (int hb = 0; hb < NHALF; ++hb)
#pragma unroll
                for (int kk = 0; kk < KR; ++kk)
                    wp[R1 * TSB * kk + hb * U] = C2{cr[hb][rd * KR + kk], ci[hb][rd * KR + kk]};
        };
        __syncthreads();  // the tile's previous readers are done
        put(0);
        __syncthreads();
#pragma unroll
        for (int rd = 0; rd < NRND; ++rd) {
            const int y0 = rd * 2 * U;
            if (y0 >= Vy) break;  // block-uniform
            const int y = y0 + 2 * unit;
            const bool live = y < Vy, has_b = y + 1 < Vy;
            C2 *ra = tile + (2 * unit) * TSB, *rb = ra + TSB;
            const int m1 = opaque(n1) & (R1 - 1);
            T re[R2], im[R2];
#pragma unroll
            for (int i = 0; i < R2; ++i) {
                const int k = m1 + R1 * i;
                // rows past Vy hold stale tile data: transformed, never used
                C2 a, bq;
                if (k == 0 || k == N / 2) {  // the packed column: Re at x-frequency 0, Im at N/2
                    const C2 p = ra[0], q = rb[0];
                    a = C2{k == 0 ? p.x : p.y, (T)0};
                    bq = C2{k == 0 ? q.x : q.y, (T)0};
                } else if (k < N / 2) {
                    a = ra[k];
                    bq = rb[k];
                } else {
                    a = ra[N - k];
                    bq = rb[N - k];
                    a.y = -a.y;
                    bq.y = -bq.y;
                }
                if (!has_b) bq = C2{(T)0, (T)0};
                re[i] = a.x - bq.y;
                im[i] = a.y + bq.x;
            }
            fft_unit_lt<T, N, true>(re, im, m1, ra, 1, tw2, true, W::XP);
            if (rd + 1 < NRND && y0 + 2 * U < Vy) {  // block-uniform
                __syncthreads();  // every unit is done with this batch's rows
                put(rd + 1);
                __syncthreads();
            }
            if (live) {
                uint32_t vb;
                const uint32_t f = row_pair_epilogue<T, N, OCC>(re, im, m1, y, Vx, Vy, tz, OCC_PASS,
                                                                (OCC && !OCC_PASS) ? cw[rd] : 0u, inv_n3, beta,
                                                                psi_out, clash_out, acc, vb);
                if (OCC_PASS) {
                    cw[rd] = f;
                    any_free |= (vb & ~f) != 0u;
                }
            }
        }
    };
    if constexpr (OCC) {
        channel(BoolTag<true>{});
        // the energies only where some translation is clash-free (always when exporting)
        if (psi_out || __syncthreads_or(any_free)) channel(BoolTag<false>{});
    } else {
        channel(BoolTag<false>{});
    }
    block_partial_store<T, WT>(acc, red, pp + c.pp_base + tz);
}

// Per-configuration descriptors of a finished scan (inputs of the learned
// proposal), one block per ligand, FP64:
//   x_c   = ln sum_s W_s Z_{c,s}            (Eq. 2 numerator of one configuration)
//   psi_c = min_s psi_min_{c,s}
//   f_c   = sum_s n_finite / sum_s n_valid
// written as floats  (max(x_c - max_c' x_c', -25) / 5,
//                     min(psi_c - min_c' psi_c', 50) / 10,  f_c)
// into columns col0..col0+2 of the row-major matrix feat[n_cfg][ld].
// Configurations with nothing finite get (-5, 5, 0).
__device__ __forceinline__ void cfg_stats(const fftdg_partial *__restrict__ p, int64_t n_cfg_total, int n_snap,
                                          const double *__restrict__ W, int c, double &x, double &psi,
                                          double &frac) {
    double mx = -INFINITY;
    psi = INFINITY;
    long long nv = 0, nf = 0;
    for (int s = 0; s < n_snap; ++s) {
        const fftdg_partial q = p[(int64_t)s * n_cfg_total + c];
        nv += q.n_valid;
        nf += q.n_finite;
        if (q.psi_min < psi) psi = q.psi_min;
        if (q.n_finite > 0 && W[s] > 0.0) {
            const double v = log(W[s]) + q.m + log(q.s);
            if (v > mx) mx = v;
        }
    }
    double sum = 0.0;
    if (mx > -INFINITY)
        for (int s = 0; s < n_snap; ++s) {
            const fftdg_partial q = p[(int64_t)s * n_cfg_total + c];
            if (q.n_finite > 0 && W[s] > 0.0) sum += exp(log(W[s]) + q.m + log(q.s) - mx);
        }
    x = mx > -INFINITY ? mx + log(sum) : -INFINITY;
    frac = nv > 0 ? (double)nf / (double)nv : 0.0;
}

__global__ __launch_bounds__(NT) void k_scan_features(const fftdg_partial *__restrict__ p, int64_t n_cfg_total,
                                                       int n_snap, const int32_t *__restrict__ cfg_off,
                                                       const double *__restrict__ W, float *__restrict__ feat,
                                                       int ld, int col0) {
    __shared__ double sx[NT], sp[NT];
    const int lig = blockIdx.x, t = threadIdx.x;
    const int c0i = cfg_off[lig], c1i = cfg_off[lig + 1];
    double xm = -INFINITY, pm = INFINITY;
    for (int c = c0i + t; c < c1i; c += NT) {
        double x, psi, f;
        cfg_stats(p, n_cfg_total, n_snap, W, c, x, psi, f);
        if (x > xm) xm = x;
        if (psi < pm) pm = psi;
    }
    sx[t] = xm;
    sp[t] = pm;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w) {
            sx[t] = sx[t] > sx[t + w] ? sx[t] : sx[t + w];
            sp[t] = sp[t] < sp[t + w] ? sp[t] : sp[t + w];
        }
        __syncthreads();
    }
    const double X = sx[0], PM = sp[0];
    for (int c = c0i + t; c < c1i; c += NT) {
        double x, psi, f;
        cfg_stats(p, n_cfg_total, n_snap, W, c, x, psi, f);
        const double a = x > -INFINITY ? fmax(x - X, -25.0) / 5.0 : -5.0;
        const double b = psi < INFINITY ? fmin(psi - PM, 50.0) / 10.0 : 5.0;
        float *row = feat + (int64_t)c * ld + col0;
        row[0] = (float)a;
        row[1] = (float)b;
        row[2] = (float)f;
    }
}

// Translation draws of sampling importance resampling for one
// configuration (one block): weights w_i = exp(-beta (Psi_i - Psi_min)) over
// the clash-free translations i of the exported grid (linear order
// (tz, ty, tx)), FP64; draw j takes the first i whose running sum of w
// exceeds u_j times the total.  Each thread owns a contiguous segment; a
// draw finds its segment from the segments' running sums, then scans it.
template <typename T>
__global__ __launch_bounds__(NT) void k_sample_translations(const T *__restrict__ psi,
                                                            const uint8_t *__restrict__ clash, int n, double beta,
                                                            const double *__restrict__ u, int nu,
                                                            int32_t *__restrict__ out_lin, double *__restrict__ out_psi) {
    __shared__ double seg[NT + 1];
    __shared__ double red[NT];
    const int t = threadIdx.x;
    const int L = (n + NT - 1) / NT;
    const int a = min(n, t * L), e = min(n, a + L);
    double pm = INFINITY;
    for (int i = a; i < e; ++i)
        if (!clash[i] && (double)psi[i] < pm) pm = (double)psi[i];
    red[t] = pm;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w) red[t] = red[t] < red[t + w] ? red[t] : red[t + w];
        __syncthreads();
    }
    const double P0 = red[0];
    double sum = 0.0;
    for (int i = a; i < e; ++i)
        if (!clash[i]) sum += exp(-beta * ((double)psi[i] - P0));
    seg[t + 1] = sum;
    __syncthreads();
    if (t == 0) {
        seg[0] = 0.0;
        for (int k = 1; k <= NT; ++k) seg[k] += seg[k - 1];
    }
    __syncthreads();
    const double total = seg[NT];
    for (int j = t; j < nu; j += NT) {
        const double x = u[j] * total;
        // segment k: seg[k] <= x < seg[k + 1]
        int lo = 0, hi = NT;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (seg[mid] <= x) lo = mid; else hi = mid;
        }
        const int sa = min(n, lo * L), se = min(n, sa + L);
        double run = seg[lo];
        int pick = -1;
        for (int i = sa; i < se; ++i) {
            if (clash[i]) continue;
            run += exp(-beta * ((double)psi[i] - P0));
            pick = i;
            if (run > x) break;
        }
        if (pick < 0) {  // x at the very top: the last clash-free translation
            for (int i = n - 1; i >= 0; --i)
                if (!clash[i]) { pick = i; break; }
        }
        out_lin[j] = pick;
        out_psi[j] = (double)psi[pick];
    }
}

// Interaction energy of ligand poses from the receptor grids by trilinear
// interpolation at each atom's position (what the FFT correlation gives at
// one translation, Eq. 8), FP64 accumulation; one block per pose.  Corners
// outside [0, n_rec) read as zero (the zero padding the FFT sees).
template <typename T>
__global__ __launch_bounds__(NT) void k_grid_energies(const T *__restrict__ grids, int n_rec, double h, double ox,
                                                      double oy, double oz, int n_atoms,
                                                      const double *__restrict__ lq, const double *__restrict__ ls,
                                                      const double *__restrict__ le,
                                                      const double *__restrict__ pose, double *__restrict__ out) {
    __shared__ double red[3][NT];
    const int p = blockIdx.x, t = threadIdx.x;
    const long long n2 = (long long)n_rec * n_rec, n3 = n2 * n_rec;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = t; i < n_atoms; i += NT) {
        const double *x = pose + 3 * ((long long)p * n_atoms + i);
        const double u[3] = {(x[0] - ox) / h, (x[1] - oy) / h, (x[2] - oz) / h};
        int i0[3];
        double f[3];
        for (int d = 0; d < 3; ++d) {
            const double fl = floor(u[d]);
            i0[d] = (int)fl;
            f[d] = u[d] - fl;
        }
        const double s3 = ls[i] * ls[i] * ls[i];
        const double se = sqrt(le[i]);
        const double gam[3] = {lq[i], se * s3 * s3, -2.0 * se * s3};
        double v[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < 8; ++c) {
            const int cx = i0[0] + (c & 1), cy = i0[1] + ((c >> 1) & 1), cz = i0[2] + (c >> 2);
            if (cx < 0 || cy < 0 || cz < 0 || cx >= n_rec || cy >= n_rec || cz >= n_rec) continue;
            const double w = ((c & 1) ? f[0] : 1.0 - f[0]) * (((c >> 1) & 1) ? f[1] : 1.0 - f[1]) *
                             ((c >> 2) ? f[2] : 1.0 - f[2]);
            const long long g = (long long)cz * n2 + (long long)cy * n_rec + cx;
            for (int ch = 0; ch < 3; ++ch) v[ch] += w * (double)grids[ch * n3 + g];
        }
        for (int ch = 0; ch < 3; ++ch) acc[ch] += gam[ch] * v[ch];
    }
    for (int ch = 0; ch < 3; ++ch) red[ch][t] = acc[ch];
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int ch = 0; ch < 3; ++ch) red[ch][t] += red[ch][t + w];
        __syncthreads();
    }
    if (t < 3) out[3 * p + t] = red[t][0];
}

// Direct atom-pair interaction energies of ligand poses (Eqs. 4-6), FP64,
// no grid: ELE 332.05 q_i q_j / r, LJr sqrt(eps_i eps_j) (sigma_i sigma_j)^6 / r^12,
// LJa -2 sqrt(eps_i eps_j) (sigma_i sigma_j)^3 / r^6; with `excl` every term
// of a pair closer than 2^(-1/6) sigma_j (the receptor atom's) is zero, as
// in the occupancy-mode grids.  One block per pose.
__global__ __launch_bounds__(NT) void k_pair_energies(int n_rec_atoms, const double *__restrict__ rxyz,
                                                      const double *__restrict__ rq, const double *__restrict__ rs,
                                                      const double *__restrict__ re, int n_atoms,
                                                      const double *__restrict__ lq, const double *__restrict__ ls,
                                                      const double *__restrict__ le,
                                                      const double *__restrict__ pose, int excl,
                                                      double *__restrict__ out) {
    __shared__ double lx[MAXA], ly[MAXA], lz[MAXA], lg[3][MAXA];
    __shared__ double red[3][NT];
    const int p = blockIdx.x, t = threadIdx.x;
    for (int i = t; i < n_atoms; i += NT) {
        const double *x = pose + 3 * ((long long)p * n_atoms + i);
        lx[i] = x[0];
        ly[i] = x[1];
        lz[i] = x[2];
        const double s3 = ls[i] * ls[i] * ls[i];
        const double se = sqrt(le[i]);
        lg[0][i] = lq[i];
        lg[1][i] = se * s3 * s3;
        lg[2][i] = -2.0 * se * s3;
    }
    __syncthreads();
    const double k6 = pow(2.0, -1.0 / 6.0);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int j = t; j < n_rec_atoms; j += NT) {
        const double X = rxyz[3 * j], Y = rxyz[3 * j + 1], Z = rxyz[3 * j + 2];
        const double s3 = rs[j] * rs[j] * rs[j];
        const double se = sqrt(re[j]);
        const double rex = k6 * rs[j];
        for (int i = 0; i < n_atoms; ++i) {
            const double dx = lx[i] - X, dy = ly[i] - Y, dz = lz[i] - Z;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (excl && r < rex) continue;
            const double r6 = r * r * r * r * r * r;
            acc[0] += lg[0][i] * 332.05 * rq[j] / r;
            acc[1] += lg[1][i] * se * s3 * s3 / (r6 * r6);
            acc[2] += lg[2][i] * se * s3 / r6;
        }
    }
    for (int ch = 0; ch < 3; ++ch) red[ch][t] = acc[ch];
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int ch = 0; ch < 3; ++ch) red[ch][t] += red[ch][t + w];
        __syncthreads();
    }
    if (t < 3) out[3 * p + t] = red[t][0];
}

// Eq. 7 receptor grids and Eq. 10 occupancy from atoms, FP64, one thread per
// grid point, atoms staged through LDS in order.
#pragma clang fp contract(off)
template <typename T>
__global__ __launch_bounds__(NT) void k_receptor_grids(int n_atoms, const double *__restrict__ xyz,
                                                        const double *__restrict__ q, const double *__restrict__ sg,
                                                        const double *__restrict__ ep, int n_rec, double h, double ox,
                                                        double oy, double oz, int mode, double cap, double occ_f,
                                                        T *__restrict__ grids, uint8_t *__restrict__ occ) {
    __shared__ double ax[NT], ay[NT], az[NT], aq[NT], as[NT], ae[NT];
    const long long n3 = (long long)n_rec * n_rec * n_rec;
    const long long idx = (long long)blockIdx.x * NT + threadIdx.x;
    const bool ok = idx < n3;
    const int x = ok ? (int)(idx % n_rec) : 0;
    const int y = ok ? (int)((idx / n_rec) % n_rec) : 0;
    const int z = ok ? (int)(idx / ((long long)n_rec * n_rec)) : 0;
    const double px = ox + h * x, py = oy + h * y, pz = oz + h * z;
    const double k6 = pow(2.0, -1.0 / 6.0);
    double ele = 0.0, ljr = 0.0, lja = 0.0;
    int hit = 0;
    for (int a0 = 0; a0 < n_atoms; a0 += NT) {
        __syncthreads();
        const int a = a0 + threadIdx.x;
        if (a < n_atoms) {
            ax[threadIdx.x] = xyz[3 * a];
            ay[threadIdx.x] = xyz[3 * a + 1];
            az[threadIdx.x] = xyz[3 * a + 2];
            aq[threadIdx.x] = q[a];
            as[threadIdx.x] = sg[a];
            ae[threadIdx.x] = ep[a];
        }
        __syncthreads();
        const int na = min(NT, n_atoms - a0);
        for (int j = 0; j < na; ++j) {
            const double dx = ax[j] - px, dy = ay[j] - py, dz = az[j] - pz;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double rex = k6 * as[j];
            if (r < occ_f * rex) hit = 1;
            const double s3 = as[j] * as[j] * as[j];
            const double se = sqrt(ae[j]);
            const double r6 = r * r * r * r * r * r;
            if (r >= rex) {
                ele += 332.05 * aq[j] / r;
                lja += se * s3 / r6;
                ljr += se * s3 * s3 / (r6 * r6);
            } else if (mode == 1) {
                ljr += se * s3 * s3 / (r6 * r6);
            }
        }
    }
    if (!ok) return;
    if (mode == 1 && ljr > cap) ljr = cap;
    grids[idx] = (T)ele;
    grids[n3 + idx] = (T)ljr;
    grids[2 * n3 + idx] = (T)lja;
    if (occ) occ[idx] = (uint8_t)hit;
}
#pragma clang fp contract(on)

// ------------------------------------------------------------------ launchers
template <typename T, int N>
struct Launch {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    static hipError_t rec_spectra(hipStream_t st, const void *grids, const uint8_t *occ, int n_rec, int n_ch,
                                  const void *tw, void *rxy, void *rspec) {
        hipLaunchKernelGGL((k_rec_xy<T, N>), dim3(n_ch * n_rec), dim3(NT), 0, st, (const T *)grids, occ, n_rec,
                           (const C2 *)tw, (C2 *)rxy);
        const int n_tiles = (G::NP + G::U - 1) / G::U;
        hipLaunchKernelGGL((k_rec_z<T, N>), dim3(n_ch * n_tiles), dim3(NT), 0, st, (const C2 *)rxy, n_rec, n_tiles,
                           (const C2 *)tw, (C2 *)rspec);
        return hipGetLastError();
    }
    static hipError_t fwd(hipStream_t st, bool edf, const int32_t *fwd_off, int n_cfg, int n_items,
                          const CfgDev *cfgs, const int32_t *ulat, const void *gam, const double *thr,
                          const void *tw, void *ws) {
        if (n_items <= 0) return hipSuccess;
        if (edf)
            hipLaunchKernelGGL((k_lig_fwd_xy<T, N, true>), dim3(n_items), dim3(NT), 0, st, fwd_off, n_cfg, cfgs,
                               ulat, (const T *)gam, thr, (const C2 *)tw, (C2 *)ws);
        else
            hipLaunchKernelGGL((k_lig_fwd_xy<T, N, false>), dim3(n_items), dim3(NT), 0, st, fwd_off, n_cfg, cfgs,
                               ulat, (const T *)gam, thr, (const C2 *)tw, (C2 *)ws);
        return hipGetLastError();
    }
    static hipError_t zprod(hipStream_t st, bool occ, bool edirect, int zhalf, const CfgDev *cfgs, const int32_t *zcfg,
                            int nz, const void *ws, const void *rspec, const void *tw, void *wsi,
                            const int32_t *ulat, const void *gam, int n_snap, int64_t spec_stride,
                            int64_t inv_stride) {
        if (nz <= 0) return hipSuccess;
        const int n_tiles = (G::NP + G::U - 1) / G::U;
        long long nb = (long long)n_tiles * nz;
        nb = (nb + 7) / 8 * 8;
#define FFTDG_ZPROD(O, E, Z)                                                                              \
    if (n_snap > 1)                                                                                       \
        hipLaunchKernelGGL((k_zprod<T, N, O, E, true, Z>), dim3((unsigned)nb), dim3(NT), 0, st, cfgs, zcfg,  \
                           nz, n_tiles, (const C2 *)ws, (const C2 *)rspec, (const C2 *)tw, (C2 *)wsi, ulat,    \
                           (const T *)gam, n_snap, spec_stride, inv_stride);                                   \
    else                                                                                                  \
        hipLaunchKernelGGL((k_zprod<T, N, O, E, false, Z>), dim3((unsigned)nb), dim3(NT), 0, st, cfgs, zcfg, \
                           nz, n_tiles, (const C2 *)ws, (const C2 *)rspec, (const C2 *)tw, (C2 *)wsi, ulat,    \
                           (const T *)gam, n_snap, spec_stride, inv_stride)
        if (occ && edirect) FFTDG_ZPROD(true, true, 0);
        else if (occ && zhalf == 2) FFTDG_ZPROD(true, false, 2);
        else if (occ && zhalf) FFTDG_ZPROD(true, false, 1);
        else if (occ) FFTDG_ZPROD(true, false, 0);
        else if (edirect) FFTDG_ZPROD(false, true, 0);
        else if (zhalf) FFTDG_ZPROD(false, false, 1);
        else FFTDG_ZPROD(false, false, 0);
#undef FFTDG_ZPROD
        return hipGetLastError();
    }
    static hipError_t inv(hipStream_t st, bool occ, const int32_t *inv_off, int n_cfg, int n_items,
                          const CfgDev *cfgs, const void *wsi, double beta, const void *tw, void *pp, void *psi_out,
                          uint8_t *clash_out, unsigned int *e_count) {
        if (n_items <= 0) return hipSuccess;
        const T b = (T)beta, s = (T)(1.0 / ((double)N * N * N));
        if (occ)
            hipLaunchKernelGGL((k_inv_xy_lse<T, N, true>), dim3(n_items), dim3(NT), 0, st, inv_off, n_cfg, cfgs,
                               (const C2 *)wsi, b, s, (const C2 *)tw, (PlanePartial<T> *)pp, (T *)psi_out, clash_out,
                               e_count);
        else
            hipLaunchKernelGGL((k_inv_xy_lse<T, N, false>), dim3(n_items), dim3(NT), 0, st, inv_off, n_cfg, cfgs,
                               (const C2 *)wsi, b, s, (const C2 *)tw, (PlanePartial<T> *)pp, (T *)psi_out, clash_out,
                               e_count);
        return hipGetLastError();
    }
    static hipError_t merge(hipStream_t st, const CfgDev *cfgs, int n_cfg, const void *pp, fftdg_partial *out) {
        if (n_cfg <= 0) return hipSuccess;
        hipLaunchKernelGGL((k_merge<T>), dim3((n_cfg + 127) / 128), dim3(128), 0, st, cfgs, n_cfg,
                           (const PlanePartial<T> *)pp, out);
        return hipGetLastError();
    }
};

// Launch sequences for FFT sizes whose planes do not fit in LDS.
template <typename T, int N>
struct LaunchSplit {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    static hipError_t rec_spectra(hipStream_t st, const void *grids, const uint8_t *occ, int n_rec, int n_ch,
                                  const void *tw, void *rxy, void *rspec) {
        hipLaunchKernelGGL((k_rec_rows<T, N>), dim3(n_ch * n_rec), dim3(NT), 0, st, (const T *)grids, occ, n_rec,
                           (const C2 *)tw, (C2 *)rxy);
        hipLaunchKernelGGL((k_rec_cols<T, N>), dim3(n_ch * n_rec * Tile<T, N>::NTILE), dim3(NT), 0, st, n_rec,
                           (const C2 *)tw, (C2 *)rxy);
        const int n_tiles = (G::NP + G::U - 1) / G::U;
        hipLaunchKernelGGL((k_rec_z<T, N>), dim3(n_ch * n_tiles), dim3(NT), 0, st, (const C2 *)rxy, n_rec, n_tiles,
                           (const C2 *)tw, (C2 *)rspec);
        return hipGetLastError();
    }
    static hipError_t fwd(hipStream_t st, bool edf, const int32_t *fwd_off, int n_cfg, int n_items,
                          const CfgDev *cfgs, const int32_t *ulat, const void *gam, const double *thr,
                          const void *tw, void *ws) {
        if (n_items <= 0) return hipSuccess;
        if (edf) {
            hipLaunchKernelGGL((k_fwd_rows<T, N, true>), dim3(n_items), dim3(NT), 0, st, fwd_off, n_cfg, cfgs, ulat,
                               (const T *)gam, thr, (const C2 *)tw, (C2 *)ws);
            hipLaunchKernelGGL((k_fwd_cols<T, N, true>), dim3(n_items * Tile<T, N>::NTILE), dim3(NT), 0, st, fwd_off,
                               n_cfg, cfgs, (const C2 *)tw, (C2 *)ws);
        } else {
            hipLaunchKernelGGL((k_fwd_rows<T, N, false>), dim3(n_items), dim3(NT), 0, st, fwd_off, n_cfg, cfgs, ulat,
                               (const T *)gam, thr, (const C2 *)tw, (C2 *)ws);
            hipLaunchKernelGGL((k_fwd_cols<T, N, false>), dim3(n_items * Tile<T, N>::NTILE), dim3(NT), 0, st, fwd_off,
                               n_cfg, cfgs, (const C2 *)tw, (C2 *)ws);
        }
        return hipGetLastError();
    }
    static hipError_t inv(hipStream_t st, bool occ, const int32_t *inv_off, int n_cfg, int n_items,
                          const CfgDev *cfgs, const void *wsi, double beta, const void *tw, void *pp, void *psi_out,
                          uint8_t *clash_out, unsigned int *e_count) {
        if (n_items <= 0) return hipSuccess;
        const T b = (T)beta, s = (T)(1.0 / ((double)N * N * N));
        if (occ)
            hipLaunchKernelGGL((k_inv_plane<T, N, true>), dim3(n_items), dim3(Whole<T, N>::WT), 0, st, inv_off, n_cfg,
                               cfgs, (const C2 *)wsi, b, s, (const C2 *)tw, (PlanePartial<T> *)pp, (T *)psi_out,
                               clash_out, e_count);
        else
            hipLaunchKernelGGL((k_inv_plane<T, N, false>), dim3(n_items), dim3(Whole<T, N>::WT), 0, st, inv_off, n_cfg,
                               cfgs, (const C2 *)wsi, b, s, (const C2 *)tw, (PlanePartial<T> *)pp, (T *)psi_out,
                               clash_out, e_count);
        return hipGetLastError();
    }
};

template <typename T, int N>
static const KernelSet *make_split_set() {
    static const KernelSet s = {
        N,
        (int)sizeof(typename Cx<T>::t),
        (int)sizeof(PlanePartial<T>),
        Geo<T, N>::NP,
        LaunchSplit<T, N>::rec_spectra,
        LaunchSplit<T, N>::fwd,
        Launch<T, N>::zprod,
        LaunchSplit<T, N>::inv,
        Launch<T, N>::merge,
    };
    return &s;
}

template <typename T, int N>
static const KernelSet *make_set() {
    static const KernelSet s = {
        N,
        (int)sizeof(typename Cx<T>::t),
        (int)sizeof(PlanePartial<T>),
        Geo<T, N>::NP,
        Launch<T, N>::rec_spectra,
        Launch<T, N>::fwd,
        Launch<T, N>::zprod,
        Launch<T, N>::inv,
        Launch<T, N>::merge,
    };
    return &s;
}

const KernelSet *kernel_set(int precision, int n_fft) {
    if (precision == FFTDG_F32) {
        if (n_fft == 32) return make_set<float, 32>();
        if (n_fft == 64) return make_set<float, 64>();
        if (n_fft == 128) return make_set<float, 128>();
        if (n_fft == 256) return make_split_set<float, 256>();
    } else if (precision == FFTDG_F64) {
        if (n_fft == 32) return make_set<double, 32>();
        if (n_fft == 64) return make_set<double, 64>();
    }
    return nullptr;
}

hipError_t launch_reduce(hipStream_t st, const fftdg_partial *p, int64_t n_cfg_total, int n_snap, int n_lig,
                         const int32_t *cfg_off, const double *cfg_w, const double *W, double kT, double h3,
                         double c0, double *B, LigRed *res) {
    hipLaunchKernelGGL(k_reduce, dim3(n_lig), dim3(NT), 0, st, p, n_cfg_total, n_snap, cfg_off, cfg_w, W, kT, h3,
                       c0, B, res);
    return hipGetLastError();
}

hipError_t launch_grid_energies(hipStream_t st, int precision, const void *grids, int n_rec, double h,
                                const double *origin, int n_atoms, const double *lq, const double *ls,
                                const double *le, int n_poses, const double *pose, double *out) {
    if (precision == FFTDG_F64)
        hipLaunchKernelGGL((k_grid_energies<double>), dim3(n_poses), dim3(NT), 0, st, (const double *)grids, n_rec, h,
                           origin[0], origin[1], origin[2], n_atoms, lq, ls, le, pose, out);
    else
        hipLaunchKernelGGL((k_grid_energies<float>), dim3(n_poses), dim3(NT), 0, st, (const float *)grids, n_rec, h,
                           origin[0], origin[1], origin[2], n_atoms, lq, ls, le, pose, out);
    return hipGetLastError();
}

hipError_t launch_pair_energies(hipStream_t st, int n_rec_atoms, const double *rxyz, const double *rq,
                                const double *rs, const double *re, int n_atoms, const double *lq,
                                const double *ls, const double *le, int n_poses, const double *pose, int excl,
                                double *out) {
    hipLaunchKernelGGL(k_pair_energies, dim3(n_poses), dim3(NT), 0, st, n_rec_atoms, rxyz, rq, rs, re, n_atoms, lq,
                       ls, le, pose, excl, out);
    return hipGetLastError();
}

hipError_t launch_sample_translations(hipStream_t st, int precision, const void *psi, const uint8_t *clash, int n,
                                     double beta, const double *u, int nu, int32_t *out_lin, double *out_psi) {
    if (precision == FFTDG_F64)
        hipLaunchKernelGGL((k_sample_translations<double>), dim3(1), dim3(NT), 0, st, (const double *)psi, clash, n,
                           beta, u, nu, out_lin, out_psi);
    else
        hipLaunchKernelGGL((k_sample_translations<float>), dim3(1), dim3(NT), 0, st, (const float *)psi, clash, n,
                           beta, u, nu, out_lin, out_psi);
    return hipGetLastError();
}

hipError_t launch_scan_features(hipStream_t st, const fftdg_partial *p, int64_t n_cfg_total, int n_snap, int n_lig,
                                const int32_t *cfg_off, const double *W, float *feat, int ld, int col0) {
    hipLaunchKernelGGL(k_scan_features, dim3(n_lig), dim3(NT), 0, st, p, n_cfg_total, n_snap, cfg_off, W, feat, ld,
                       col0);
    return hipGetLastError();
}

hipError_t launch_receptor_grids(hipStream_t st, int precision, int n_atoms, const double *xyz, const double *q,
                                 const double *sg, const double *ep, int n_rec, double h, const double *origin,
                                 int mode, double cap, double occ_f, void *grids, uint8_t *occ) {
    const long long n3 = (long long)n_rec * n_rec * n_rec;
    const unsigned nb = (unsigned)((n3 + NT - 1) / NT);
    if (precision == FFTDG_F32)
        hipLaunchKernelGGL(k_receptor_grids<float>, dim3(nb), dim3(NT), 0, st, n_atoms, xyz, q, sg, ep, n_rec, h,
                           origin[0], origin[1], origin[2], mode, cap, occ_f, (float *)grids, occ);
    else
        hipLaunchKernelGGL(k_receptor_grids<double>, dim3(nb), dim3(NT), 0, st, n_atoms, xyz, q, sg, ep, n_rec, h,
                           origin[0], origin[1], origin[2], mode, cap, occ_f, (double *)grids, occ);
    return hipGetLastError();
}

}  // namespace fftdg

// Fused scan path for gfx950 (wave64): energy channels only through the FFT,
// clashes by an exact bitwise test.
//
// Clash test (occupancy mode, Eq. 10).  The overlap count of Eq. 10 is
// positive exactly when some occupied ligand grid point n lands on an
// occupied receptor point n + t (indices mod n_fft over the zero-padded
// receptor grid, the convention the FFT correlation has).  Instead of a
// fourth FFT channel thresholded at 1/2, the test is made on bits:
//   - the ligand's occupied points (union of its atoms' balls, the integer
//     membership test of the occupancy grid) are written as runs along x,
//     one per maximal segment of a (y, z) row (k_lig_runs);
//   - each receptor occupancy row is kept OR-dilated over windows of 2^k
//     points, D_k(x) = OR_{0 <= j < 2^k} O_R(x + j) (k_rec_dilate);
//   - a run of length L starting at x = a meets receptor occupancy at
//     translation t iff D_k(a + t_x) | D_k(a + L - 2^k + t_x) on row
//     (y + t_y, z + t_z), 2^k <= L < 2^(k+1); one 32-bit word answers 32
//     x-translations at once (k_clash).
// The result is the clash mask the FFT threshold reproduces, without its
// rounding: every decision is an integer one.
//
// Energy channels (Eqs. 4-9).  The x/y DFT of a trilinearly spread atom
// factorises,
//   sum_{dx,dy} w_dx w_dy w^(kx (ax+dx) + ky (ay+dy))
//     = w^(kx ax) ((1-fx) + fx w^kx) * w^(ky ay) ((1-fy) + fy w^ky),
// (w = exp(-2 pi i / N)) and the atom reaches only the planes floor(uz)
// (weight 1-fz) and floor(uz)+1 (weight fz).  The z kernel (k_zfused) forms
// each z-pencil's input from these factors (a table per block over its
// pencils and the configuration's atoms, atoms sorted by plane), runs the
// forward z FFT, the product with the receptor spectra summed over the three
// channels (Eq. 9) and the inverse z FFT, and stores only the z-translations
// that have a clash-free translation (all box-valid ones in cap mode or when
// energies are exported).  k_inv_fused finishes the inverse along y and x on
// those planes, skips row pairs without a clash-free translation, and folds
// the clash-free energies into the Eq. 2 partials.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/fftdg.h"
#include "fft_device.hpp"
#include "fused.hpp"
#include "scan_common.hpp"
#include "scan_types.hpp"

namespace fftdg {

// ------------------------------------------------------------ receptor rows
// One thread per row (Z, Y) of the periodic N^3 domain.  Level 0 holds the
// occupancy bits of the row (zero outside the n_rec^3 receptor grid); level
// k ORs level k-1 with itself advanced by 2^(k-1) points (mod N).
template <int N>
__global__ __launch_bounds__(NT) void k_rec_dilate(const uint8_t *__restrict__ occ, int n_rec,
                                                    uint32_t *__restrict__ dil) {
    using D = Dil<N>;
    constexpr int NW = D::NW;
    const int r = (int)blockIdx.x * NT + (int)threadIdx.x;
    if (r >= N * N) return;
    const int Z = r / N, Y = r - (r / N) * N;
    uint32_t v[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) v[w] = 0u;
    if (Z < n_rec && Y < n_rec) {
        const uint8_t *row = occ + ((int64_t)Z * n_rec + Y) * n_rec;
        for (int x = 0; x < n_rec; ++x)
            if (row[x]) v[x >> 5] |= 1u << (x & 31);
    }
#pragma unroll
    for (int k = 0; k < D::K; ++k) {
        if (k > 0) {
            const int s = 1 << (k - 1);  // bit x of the advanced row is bit (x + s) mod N
            uint32_t t[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int p = (32 * w + s) & (N - 1);
                const int q = p >> 5, sh = p & 31;
                const uint32_t lo = v[q], hi = v[(q + 1) % NW];
                t[w] = sh ? ((lo >> sh) | (hi << (32 - sh))) : lo;
            }
#pragma unroll
            for (int w = 0; w < NW; ++w) v[w] |= t[w];
        }
#pragma unroll
        for (int q = 0; q < D::RW; ++q) dil[D::index(k, Z, q, Y)] = v[q % NW];
    }
}

// ------------------------------------------------------------ ligand runs
// Exclusive prefix sum over the block (fixed order), `total` = block sum.
__device__ __forceinline__ int block_excl_scan(int v, int &total, int *sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        base += i < w ? sh[i] : 0;
        tot += sh[i];
    }
    __syncthreads();
    total = tot;
    return base + x - v;
}

__device__ __forceinline__ long long ceildiv16(long long a) { return -floordiv(-a, 65536LL); }

// The ball of atom `a` on row (y, z): [xlo, xhi] in true grid x, or false.
struct RunAtom {
    int Ux, Uy, Uz;
    long long T;
};
__device__ __forceinline__ bool ball_row(const RunAtom &A, int y, int z, long long &xlo, long long &xhi) {
    const long long dz = (long long)z * 65536LL - A.Uz;
    const long long rz = A.T - dz * dz;
    if (rz <= 0) return false;
    const long long dy = (long long)y * 65536LL - A.Uy;
    const long long rem = rz - dy * dy;
    if (rem <= 0) return false;
    const long long s = isqrt_lt(rem);
    xlo = ceildiv16(A.Ux - s);
    xhi = floordiv(A.Ux + s, 65536LL);
    return xlo <= xhi;
}

__device__ __forceinline__ uint32_t pack_run(int z, int y, int a, int len, int N) {
    return ((uint32_t)(z & (N - 1)) << 24) | ((uint32_t)(y & (N - 1)) << 16) | ((uint32_t)(len - 1) << 8) |
           (uint32_t)(a & (N - 1));
}

// One block per scanned configuration.  Runs are written in a fixed order:
// first each atom's chord through the row nearest its centre (its widest
// segment; a subset of the union, so harmless to the OR, and the most likely
// to meet receptor occupancy, which lets the clash test stop early), then
// the maximal segments of the union of the balls on every row of the
// occupancy window, z-major.
template <int N>
__global__ __launch_bounds__(NT) void k_lig_runs(const CfgDev *__restrict__ cfgs, const int32_t *__restrict__ zcfg,
                                                  const int32_t *__restrict__ ulat, const double *__restrict__ thr,
                                                  uint32_t *__restrict__ runs, int32_t *__restrict__ run_count) {
    constexpr int NW = N / 32;
    __shared__ RunAtom at[MAXA];
    __shared__ int sh[NT / 64];
    const int lc = zcfg[blockIdx.x];
    const CfgDev c = cfgs[lc];
    const int n = c.n_atoms;
    for (int a = threadIdx.x; a < n; a += NT) {
        const int32_t *U = ulat + 3 * (c.u_base + a);
        at[a] = RunAtom{U[0], U[1], U[2], (long long)thr[c.atom_base + a]};
    }
    __syncthreads();
    uint32_t *out = runs + c.run_off;
    const int cap = c.run_cap;
    int base = 0, total;
    // chords through the centre rows
    for (int a0 = 0; a0 < n; a0 += NT) {
        const int a = a0 + (int)threadIdx.x;
        long long xlo = 0, xhi = -1;
        int yc = 0, zc = 0;
        bool has = false;
        if (a < n) {
            yc = (int)floordiv((long long)at[a].Uy + 32768LL, 65536LL);
            zc = (int)floordiv((long long)at[a].Uz + 32768LL, 65536LL);
            has = ball_row(at[a], yc, zc, xlo, xhi);
        }
        const int pos = base + block_excl_scan(has ? 1 : 0, total, sh);
        if (has && pos < cap) out[pos] = pack_run(zc, yc, (int)xlo, (int)(xhi - xlo + 1), N);
        base += total;
    }
    // every row of the occupancy window: union of the balls as a bit row
    // relative to xo0 (the window's x extent is at most N), then its runs
    const int nrows = c.Lo * c.Lyo;
    for (int r0 = 0; r0 < nrows; r0 += NT) {
        const int r = r0 + (int)threadIdx.x;
        uint32_t m[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) m[w] = 0u;
        int z = 0, y = 0;
        if (r < nrows) {
            z = c.zo0 + r / c.Lyo;
            y = c.yo0 + r % c.Lyo;
            for (int a = 0; a < n; ++a) {
                long long xlo, xhi;
                if (!ball_row(at[a], y, z, xlo, xhi)) continue;
                const int l = (int)(xlo - c.xo0), h = (int)(xhi - c.xo0);
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    const int lo = max(l, 32 * w), hi = min(h, 32 * w + 31);
                    if (lo <= hi) {
                        const int wid = hi - lo + 1;
                        m[w] |= (wid == 32 ? ~0u : ((1u << wid) - 1u)) << (lo - 32 * w);
                    }
                }
            }
        }
        // runs start where a set bit follows a clear one
        int cnt = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint32_t prev = (m[w] << 1) | (w > 0 ? m[w - 1] >> 31 : 0u);
            cnt += __builtin_popcount(m[w] & ~prev);
        }
        int pos = base + block_excl_scan(cnt, total, sh);
        if (cnt > 0) {
            int x = 0;
            while (x < N) {
                // next set bit at or after x
                int s = N;
                for (int w = x >> 5; w < NW; ++w) {
                    const uint32_t b = m[w] & (w == (x >> 5) ? (~0u << (x & 31)) : ~0u);
                    if (b) {
                        s = 32 * w + __builtin_ctz(b);
                        break;
                    }
                }
                if (s >= N) break;
                // next clear bit after s
                int e = N;
                for (int w = s >> 5; w < NW; ++w) {
                    const uint32_t b = ~m[w] & (w == (s >> 5) ? (~0u << (s & 31)) : ~0u);
                    if (b) {
                        e = 32 * w + __builtin_ctz(b);
                        break;
                    }
                }
                if (pos < cap) out[pos] = pack_run(z, y, c.xo0 + s, e - s, N);
                ++pos;
                x = e;
            }
        }
        base += total;
    }
    if (threadIdx.x == 0) run_count[lc] = base < cap ? base : cap;
}

// ------------------------------------------------------------ clash test
// One wavefront per (configuration, z-translation tz, group of 64 y-
// translations); lane = ty.  Free bits (box-valid and clash-free) of row
// (tz, ty) go to fb[free_off + (tz Vy + ty) W + w], W = ceil(Vx / 32), bit
// tx & 31 of word tx >> 5; live[item_base + tz ny + g] = 1 if the group has
// any.  The run loop stops once every lane's translations all clash.
template <int N>
__global__ __launch_bounds__(NT) void k_clash(const int32_t *__restrict__ item_off, int n_cfg, int n_items,
                                               const CfgDev *__restrict__ cfgs, const uint32_t *__restrict__ runs,
                                               const int32_t *__restrict__ run_count, const uint32_t *__restrict__ dil,
                                               uint32_t *__restrict__ fb, uint8_t *__restrict__ live) {
    using D = Dil<N>;
    constexpr int NW = D::NW;
    const int item = (int)blockIdx.x * (NT / 64) + ((int)threadIdx.x >> 6);
    if (item >= n_items) return;
    const int lane = threadIdx.x & 63;
    const int ic = find_cfg(item_off, n_cfg, item);
    const CfgDev c = cfgs[ic];
    const int Vx = c.V[0], Vy = c.V[1];
    const int ny = (Vy + 63) >> 6;
    const int loc = item - item_off[ic];
    const int tz = loc / ny, g = loc - (loc / ny) * ny;
    const int ty = 64 * g + lane;
    const bool act = ty < Vy;
    const int W = (Vx + 31) >> 5;
    const uint32_t lm = (Vx & 31) ? ((1u << (Vx & 31)) - 1u) : ~0u;
    uint32_t acc[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) acc[w] = 0u;
    const int nr = run_count[ic];
    const uint32_t *rl = runs + c.run_off;
    const auto rsrc = make_rsrc(dil, (int)(D::words() * 4));
    for (int i = 0; i < nr; ++i) {
        const uint32_t e = rl[i];
        const int a = (int)(e & 0xffu), len = (int)((e >> 8) & 0xffu) + 1;
        const int Yo = (int)((e >> 16) & 0xffu), Zo = (int)(e >> 24);
        const int Z = (Zo + tz) & (N - 1);
        const int k = 31 - __builtin_clz((unsigned)len);
        const int Y = (Yo + ty) & (N - 1);
        const int vo = Y * 4;
        const int p1 = a, p2 = (a + len - (1 << k)) & (N - 1);
        const int rb = (k * N + Z) * D::RW;  // row block of level k, slice Z
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int p = h ? p2 : p1;
            const int q0 = p >> 5, sh = p & 31;
            uint32_t v[NW + 1];
#pragma unroll
            for (int j = 0; j <= NW; ++j)
                v[j] = j <= W ? __builtin_amdgcn_raw_buffer_load_b32(rsrc, vo, (rb + q0 + j) * N * 4, 0) : 0u;
#pragma unroll
            for (int w = 0; w < NW; ++w)
                if (w < W) acc[w] |= __builtin_amdgcn_alignbit(v[w + 1], v[w], (unsigned)sh);
        }
        if ((i & 7) == 7) {
            bool full = true;
#pragma unroll
            for (int w = 0; w < NW; ++w)
                if (w < W) full = full && ((w == W - 1) ? ((acc[w] & lm) == lm) : (acc[w] == ~0u));
            if (__all(!act || full)) break;
        }
    }
    bool any = false;
    if (act) {
        uint32_t *o = fb + c.free_off + ((int64_t)tz * Vy + ty) * W;
#pragma unroll
        for (int w = 0; w < NW; ++w)
            if (w < W) {
                const uint32_t f = ~acc[w] & (w == W - 1 ? lm : ~0u);
                o[w] = f;
                any = any || f != 0u;
            }
    }
    const unsigned long long bal = __ballot(any);
    if (lane == 0) live[c.item_base + loc] = bal != 0ull ? 1 : 0;
}

// ------------------------------------------------------------ z pass
// Block -> (tile of P z-pencils, configuration), with the XCD-aware order of
// the plane path's z kernel.  ZHI: the configuration's energy window (L_e
// planes, loaded from plane 0; the correlation of the shifted grid is the
// wanted one shifted by ze0, undone at the store) fits in the lower half of
// the pencil, so the first radix-2 stage is pruned.  CLASH: store only the
// z-translations whose live flag is set; a configuration with none is
// skipped whole.
template <typename T, int N, bool ZHI, bool CLASH>
__global__ __launch_bounds__(NT) void k_zfused(const CfgDev *__restrict__ cfgs, const int32_t *__restrict__ zcfg,
                                                int nz, int n_tiles, int ma, int ac,
                                                const typename Cx<T>::t *__restrict__ rspec,
                                                const typename Cx<T>::t *__restrict__ twg,
                                                typename Cx<T>::t *__restrict__ wsi, const int32_t *__restrict__ ulat,
                                                const T *__restrict__ gam, const uint8_t *__restrict__ live) {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    constexpr int R1 = G::R1, R2 = G::R2, P = G::U, NP = G::NP, H = G::H, PW = G::PW, PAD = G::PAD;
    constexpr int FP = P + 1;  // table row stride (complex): lanes of different planes on distinct banks
    __shared__ C2 buf[4 * G::WREG];
    __shared__ C2 tw[N];
    __shared__ uint32_t lv[N / 32];
    __shared__ int zb[N + 2];
    extern __shared__ __align__(16) unsigned char dyn[];
    const int nb = gridDim.x, b = blockIdx.x;
    const int L = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    if (L >= n_tiles * nz) return;
    const int tile = L / nz, zi = L % nz;
    const CfgDev c = cfgs[zcfg[zi]];
    const int Vz = c.V[2];
    if (threadIdx.x < N / 32) lv[threadIdx.x] = 0u;
    __syncthreads();
    if (CLASH) {
        const int ny = (c.V[1] + 63) >> 6;
        for (int tz = threadIdx.x; tz < Vz; tz += NT) {
            bool l = false;
            for (int g = 0; g < ny; ++g) l = l || live[c.item_base + tz * ny + g] != 0;
            if (l) atomicOr(&lv[tz >> 5], 1u << (tz & 31));
        }
    } else {
        for (int tz = threadIdx.x; tz < Vz; tz += NT) atomicOr(&lv[tz >> 5], 1u << (tz & 31));
    }
    __syncthreads();
    {
        uint32_t any = 0u;
#pragma unroll
        for (int w = 0; w < N / 32; ++w) any |= lv[w];
        if (any == 0u) return;  // block-uniform: no translation of this configuration is clash-free
    }
    // dynamic LDS (ma = most atoms of a ligand in the launch): planes of the
    // atoms in batch order, then sorted by plane: planes, weights, x/y
    // placement; then the factor table F[ac][FP]
    const int n = c.n_atoms;
    int *raz = (int *)dyn;                        // [ma] plane of atom a, batch order
    int *saz = raz + ma;                          // [ma] sorted planes
    int *sxy = saz + ma;                          // [ma][2] ax, ay
    T *swt = (T *)(((uintptr_t)(sxy + 2 * ma) + 15) & ~(uintptr_t)15);  // [ma][6] gamma_ch (1 - fz), gamma_ch fz
    T *sf = swt + 6 * ma;                         // [ma][2] fx, fy
    C2 *F = (C2 *)(((uintptr_t)(sf + 2 * ma) + 15) & ~(uintptr_t)15);
    load_tw<T, N>(tw, twg);
    for (int a = threadIdx.x; a < n; a += NT) raz[a] = ulat[3 * (c.u_base + a) + 2] >> 16;
    __syncthreads();
    for (int a = threadIdx.x; a < n; a += NT) {
        const int az = raz[a];
        int rk = 0;
        for (int o = 0; o < n; ++o) {
            const int bz = raz[o];
            rk += (bz < az || (bz == az && o < a)) ? 1 : 0;
        }
        const int32_t *U = ulat + 3 * (c.u_base + a);
        const T fz = (T)(U[2] & 0xffff) * (T)(1.0 / 65536.0);
        saz[rk] = az;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const T g = gam[3 * (c.atom_base + a) + ch];
            swt[6 * rk + ch] = g * ((T)1 - fz);
            swt[6 * rk + 3 + ch] = g * fz;
        }
        sxy[2 * rk] = U[0] >> 16;
        sxy[2 * rk + 1] = U[1] >> 16;
        sf[2 * rk] = (T)(U[0] & 0xffff) * (T)(1.0 / 65536.0);
        sf[2 * rk + 1] = (T)(U[1] & 0xffff) * (T)(1.0 / 65536.0);
    }
    __syncthreads();
    // zb[j] = number of atoms with plane < ze0 + j - 1 (j = 0 .. Le + 1):
    // plane j of the window receives sorted atoms [zb[j], zb[j + 2])
    for (int j = threadIdx.x; j <= c.Le + 1; j += NT) {
        const int zt = c.ze0 + j - 1;
        int k = 0;
        for (int o = 0; o < n; ++o) k += saz[o] < zt ? 1 : 0;
        zb[j] = k;
    }
    const ZLane<N> zl;
    const int n1 = zl.n1, p = zl.p;
    C2 *ex = buf + zl.w * G::WREG + zl.pl;
    const int pen = tile * P + p;
    const bool ok = pen < NP;
    const int rlane = rs_lane<T, N>(n1, ok ? pen : 0);
    const int nchunk = (n + ac - 1) / ac;
    auto build_table = [&](int e0) {
        const int na = min(ac, n - e0);
        for (int idx = threadIdx.x; idx < na * P; idx += NT) {
            const int e = idx / P, q = idx - (idx / P) * P;
            const int pq = tile * P + q;
            C2 v = C2{(T)0, (T)0};
            if (pq < NP) {
                const int kyq = pq / H, kxq = pq - (pq / H) * H;
                const int ax = sxy[2 * (e0 + e)], ay = sxy[2 * (e0 + e) + 1];
                const T fx = sf[2 * (e0 + e)], fy = sf[2 * (e0 + e) + 1];
                const C2 wx = tw[kxq & (N - 1)], wy = tw[kyq & (N - 1)];
                const C2 ex_ = tw[(kxq * ax) & (N - 1)], ey = tw[(kyq * ay) & (N - 1)];
                const T sxr = (T)1 - fx + fx * wx.x, sxi = fx * wx.y;
                const T syr = (T)1 - fy + fy * wy.x, syi = fy * wy.y;
                const T xr = ex_.x * sxr - ex_.y * sxi, xi = ex_.x * sxi + ex_.y * sxr;
                const T yr = ey.x * syr - ey.y * syi, yi = ey.x * syi + ey.y * syr;
                v = C2{xr * yr - xi * yi, xr * yi + xi * yr};
            }
            F[e * FP + q] = v;
        }
    };
    T er[R2], ei[R2];
#pragma unroll
    for (int i = 0; i < R2; ++i) er[i] = ei[i] = (T)0;
    constexpr int NIN = ZHI ? R2 / 2 : R2;
#pragma unroll 1
    for (int ch = 0; ch < 3; ++ch) {
        T re[R2], im[R2];
#pragma unroll
        for (int i = 0; i < R2; ++i) re[i] = im[i] = (T)0;
        for (int ck = 0; ck < nchunk; ++ck) {
            const int e0 = ck * ac, e1 = min(n, e0 + ac);
            if (ch == 0 || nchunk > 1) {
                __syncthreads();
                build_table(e0);
                __syncthreads();
            }
#pragma unroll
            for (int i = 0; i < NIN; ++i) {
                const int j = n1 + R1 * i;
                if (j < c.Le) {
                    const int zt = c.ze0 + j;
                    const int lo = max(zb[j], e0), hi = min(zb[j + 2], e1);
                    for (int e = lo; e < hi; ++e) {
                        const T wgt = swt[6 * e + ch + (saz[e] == zt ? 0 : 3)];
                        const C2 f = F[(e - e0) * FP + p];
                        re[i] += wgt * f.x;
                        im[i] += wgt * f.y;
                    }
                }
            }
        }
        fft_unit<T, N, false, ZHI>(re, im, n1, ex, PW, tw, true, PAD);
        rprod<T, N, true>(make_rsrc(rspec + (int64_t)ch * N * NP, N * NP * (int)sizeof(C2)), rlane, re, im, er, ei);
    }
    fft_unit_rev<T, N, true>(er, ei, n1, ex, PW, tw, true, PAD);
    // element z of the output is translation t = z - ze0 (mod N); store the
    // live ones (t < Vz); others fall outside the descriptor
    const auto rd = make_rsrc(wsi + c.off_inv, Vz * NP * (int)sizeof(C2));
    const int oor = Vz * NP * (int)sizeof(C2);
#pragma unroll
    for (int i = 0; i < R2; ++i) {
        const int t = (n1 + R1 * i - c.ze0) & (N - 1);
        const bool st = ok && t < Vz && ((lv[t >> 5] >> (t & 31)) & 1u);
        buf_store(rd, st ? (t * NP + pen) * (int)sizeof(C2) : oor, C2{er[i], ei[i]});
    }
}

// ------------------------------------------------------------ inverse xy
// One block per (configuration, box-valid z-translation): inverse y on the
// packed columns, C2R along x on row pairs, Eq. 2 partial over the
// clash-free translations.  CLASH: free bits from k_clash; a plane without
// any is not read (its partial is empty) unless energies are exported.
template <typename T, int N, bool CLASH>
__global__ __launch_bounds__(NT) void k_inv_fused(const int32_t *__restrict__ inv_off, int n_cfg,
                                                   const CfgDev *__restrict__ cfgs,
                                                   const typename Cx<T>::t *__restrict__ wsi, T beta, T inv_n3,
                                                   const typename Cx<T>::t *__restrict__ twg,
                                                   const uint32_t *__restrict__ fb, const uint8_t *__restrict__ live,
                                                   PlanePartial<T> *__restrict__ pp, T *__restrict__ psi_out,
                                                   uint8_t *__restrict__ clash_out,
                                                   unsigned int *__restrict__ e_count) {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    constexpr int R1 = G::R1, R2 = G::R2, M = G::M, S = G::S, U = G::U, NP = G::NP;
    constexpr int NW = N / 32;
    static_assert(N + (R1 - 1) * G::RPAD <= 2 * S, "row-pair exchange must fit in two rows");
    __shared__ C2 Pl[N * S];
    __shared__ C2 tw[N];
    __shared__ LseAcc<T> red[NT / 64];
    const int ic = find_cfg(inv_off, n_cfg, (int)blockIdx.x);
    const CfgDev c = cfgs[ic];
    const int Vx = c.V[0], Vy = c.V[1], tz = (int)blockIdx.x - inv_off[ic];
    const bool exporting = psi_out != nullptr || clash_out != nullptr;
    LseAcc<T> acc;
    acc.init();
    if (CLASH && !exporting) {
        const int ny = (Vy + 63) >> 6;
        bool l = false;
        for (int g = 0; g < ny; ++g) l = l || live[c.item_base + tz * ny + g] != 0;
        if (!l) {  // block-uniform: every translation of the plane clashes
            if (threadIdx.x == 0) {
                PlanePartial<T> o;
                o.m = -(T)INFINITY;
                o.s = (T)0;
                o.psi_min = (T)INFINITY;
                o.n_finite = 0;
                o.argmin = -1;
                pp[c.pp_base + tz] = o;
            }
            return;
        }
    }
    if (threadIdx.x == 0 && e_count) atomicAdd(e_count, 1u);
    load_tw<T, N>(tw, twg);
    const int unit = threadIdx.x / R1, n1 = threadIdx.x % R1;
    const C2 *src = wsi + c.off_inv + (int64_t)tz * NP;
    plane_copy<T, N, true>(Pl, const_cast<C2 *>(src));
    __syncthreads();
    T re[R2], im[R2];
    // inverse y on columns (kx = 0 and N/2 packed into column 0), keep y < Vy
    constexpr int rounds_b = (N / 2 + U - 1) / U;
    for (int rd = 0; rd < rounds_b; ++rd) {
        const int col = unit + U * rd;
        const bool lv = col < N / 2;
        const bool c0 = col == 0;
#pragma unroll
        for (int i = 0; i < R2; ++i) {
            const int ky = n1 + R1 * i;
            re[i] = im[i] = (T)0;
            if (lv) {
                const C2 v = Pl[ky * S + col];
                const C2 bq = c0 ? Pl[ky * S + N / 2] : C2{(T)0, (T)0};
                re[i] = v.x - bq.y;
                im[i] = v.y + bq.x;
            }
        }
        C2 *cp = Pl + (lv ? col : 0);
        fft_unit<T, N, true, false, true>(re, im, n1, cp, S, tw, lv);
        wave_sync();  // column col (and N/2 for col = 0) is private to this unit
        if (lv) {
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
    const int W = (Vx + 31) >> 5;
    const uint32_t *fp = fb + c.free_off + (int64_t)tz * Vy * W;
    // inverse x (C2R) of row pairs (y, y+1), y < Vy
    const int npairs = (Vy + 1) / 2;
    const int rounds_a = (npairs + U - 1) / U;
    for (int rd = 0; rd < rounds_a; ++rd) {
        const int y = 2 * (unit + U * rd);
        const bool lv = y < Vy;
        uint32_t f0[NW], f1[NW];
        bool anyf = false;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            f0[w] = f1[w] = 0u;
            if (CLASH && lv && w < W) {
                f0[w] = fp[(int64_t)y * W + w];
                if (y + 1 < Vy) f1[w] = fp[(int64_t)(y + 1) * W + w];
            }
            anyf = anyf || (f0[w] | f1[w]) != 0u;
        }
        // a wavefront whose row pairs hold no clash-free translation has
        // nothing to add
        if (CLASH && !exporting && !__any(lv && anyf)) continue;
        C2 *row = Pl + (lv ? y * S : 0);
#pragma unroll
        for (int i = 0; i < R2; ++i) {
            const int k = n1 + R1 * i;
            re[i] = im[i] = (T)0;
            if (lv) {
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
        fft_unit<T, N, true>(re, im, n1, row, 1, tw, lv, G::RPAD);
        if (lv) {
            // clash flags in the epilogue's slot layout: bit 2 sl + h is
            // (x, y + h) with x = spec_index(n1, sl / R1, sl % R1)
            uint32_t cb = 0u;
            if (CLASH) {
#pragma unroll
                for (int sl = 0; sl < R2; ++sl) {
                    const int k1 = sl % R1;
                    const int x = spec_index<N>(n1, sl / R1, k1);
                    const int wi = (R2 * k1) >> 5;  // x >> 5 (compile-time)
                    cb |= (uint32_t)(((f0[wi] >> (x & 31)) & 1u) == 0u) << (2 * sl);
                    cb |= (uint32_t)(((f1[wi] >> (x & 31)) & 1u) == 0u) << (2 * sl + 1);
                }
            }
            uint32_t vb;
            (void)row_pair_epilogue<T, N, CLASH>(re, im, n1, y, Vx, Vy, tz, false, cb, inv_n3, beta, psi_out,
                                                clash_out, acc, vb);
        }
    }
    block_partial_store(acc, red, pp + c.pp_base + tz);
}

// ------------------------------------------------------------ launchers
template <typename T, int N>
struct LaunchFused {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    static hipError_t rec_dilate(hipStream_t st, const uint8_t *occ, int n_rec, uint32_t *dil) {
        hipLaunchKernelGGL((k_rec_dilate<N>), dim3((N * N + NT - 1) / NT), dim3(NT), 0, st, occ, n_rec, dil);
        return hipGetLastError();
    }
    static hipError_t lig_runs(hipStream_t st, const CfgDev *cfgs, const int32_t *zcfg, int nz, const int32_t *ulat,
                               const double *thr, uint32_t *runs, int32_t *run_count) {
        if (nz <= 0) return hipSuccess;
        hipLaunchKernelGGL((k_lig_runs<N>), dim3(nz), dim3(NT), 0, st, cfgs, zcfg, ulat, thr, runs, run_count);
        return hipGetLastError();
    }
    static hipError_t clash(hipStream_t st, const int32_t *item_off, int n_cfg, int n_items, const CfgDev *cfgs,
                            const uint32_t *runs, const int32_t *run_count, const uint32_t *dil, uint32_t *fb,
                            uint8_t *live) {
        if (n_items <= 0) return hipSuccess;
        const int nb = (n_items + NT / 64 - 1) / (NT / 64);
        hipLaunchKernelGGL((k_clash<N>), dim3(nb), dim3(NT), 0, st, item_off, n_cfg, n_items, cfgs, runs, run_count,
                           dil, fb, live);
        return hipGetLastError();
    }
    static int atoms_per_table() {
        constexpr int FP = G::U + 1;
        int a = (int)(FUSED_TABLE_BYTES / (FP * sizeof(C2)));
        return a < 1 ? 1 : a;
    }
    static size_t dyn_bytes(int max_atoms) {
        const int ac = max_atoms < atoms_per_table() ? max_atoms : atoms_per_table();
        size_t o = (size_t)max_atoms * 4 * sizeof(int);
        o = (o + 15) & ~(size_t)15;
        o += (size_t)max_atoms * 8 * sizeof(T);
        o = (o + 15) & ~(size_t)15;
        return o + (size_t)ac * (G::U + 1) * sizeof(C2) + 16;
    }
    static hipError_t zpass(hipStream_t st, bool zhalf, bool clash, const CfgDev *cfgs, const int32_t *zcfg, int nz,
                            int max_atoms, const void *rspec, const void *tw, void *wsi, const int32_t *ulat,
                            const void *gam, const uint8_t *live) {
        if (nz <= 0) return hipSuccess;
        const int n_tiles = (G::NP + G::U - 1) / G::U;
        long long nb = (long long)n_tiles * nz;
        nb = (nb + 7) / 8 * 8;
        const int ac = max_atoms < atoms_per_table() ? max_atoms : atoms_per_table();
        const size_t dyn = dyn_bytes(max_atoms);
#define FFTDG_ZF(Z, C)                                                                                           \
    hipLaunchKernelGGL((k_zfused<T, N, Z, C>), dim3((unsigned)nb), dim3(NT), dyn, st, cfgs, zcfg, nz, n_tiles,      \
                       max_atoms, ac,                                                                            \
                       (const C2 *)rspec, (const C2 *)tw, (C2 *)wsi, ulat, (const T *)gam, live)
        if (zhalf && clash) FFTDG_ZF(true, true);
        else if (zhalf) FFTDG_ZF(true, false);
        else if (clash) FFTDG_ZF(false, true);
        else FFTDG_ZF(false, false);
#undef FFTDG_ZF
        return hipGetLastError();
    }
    static hipError_t inv(hipStream_t st, bool clash, const int32_t *inv_off, int n_cfg, int n_items,
                          const CfgDev *cfgs, const void *wsi, double beta, const void *tw, const uint32_t *fb,
                          const uint8_t *live, void *pp, void *psi_out, uint8_t *clash_out, unsigned int *e_count) {
        if (n_items <= 0) return hipSuccess;
        const T b = (T)beta, s = (T)(1.0 / ((double)N * N * N));
        if (clash)
            hipLaunchKernelGGL((k_inv_fused<T, N, true>), dim3(n_items), dim3(NT), 0, st, inv_off, n_cfg, cfgs,
                               (const C2 *)wsi, b, s, (const C2 *)tw, fb, live, (PlanePartial<T> *)pp, (T *)psi_out,
                               clash_out, e_count);
        else
            hipLaunchKernelGGL((k_inv_fused<T, N, false>), dim3(n_items), dim3(NT), 0, st, inv_off, n_cfg, cfgs,
                               (const C2 *)wsi, b, s, (const C2 *)tw, fb, live, (PlanePartial<T> *)pp, (T *)psi_out,
                               clash_out, e_count);
        return hipGetLastError();
    }
};

template <typename T, int N>
static const FusedSet *make_fused() {
    static const FusedSet s = {
        N,
        Dil<N>::words(),
        LaunchFused<T, N>::rec_dilate,
        LaunchFused<T, N>::lig_runs,
        LaunchFused<T, N>::clash,
        LaunchFused<T, N>::zpass,
        LaunchFused<T, N>::inv,
        LaunchFused<T, N>::dyn_bytes,
    };
    return &s;
}

const FusedSet *fused_set(int precision, int n_fft) {
    if (precision == FFTDG_F32) {
        if (n_fft == 32) return make_fused<float, 32>();
        if (n_fft == 64) return make_fused<float, 64>();
        if (n_fft == 128) return make_fused<float, 128>();
    } else if (precision == FFTDG_F64) {
        if (n_fft == 32) return make_fused<double, 32>();
        if (n_fft == 64) return make_fused<double, 64>();
    }
    return nullptr;
}

}  // namespace fftdg

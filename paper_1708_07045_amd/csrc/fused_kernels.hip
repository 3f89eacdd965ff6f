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

#include <type_traits>

#include "../../include/fftdg.h"
#include "fft_device.hpp"
#include "fused.hpp"
#include "scan_common.hpp"
#include "scan_types.hpp"

namespace fftdg {

// ------------------------------------------------------------ receptor rows
// One thread per stored row (Z, Y) of the table.  Level 0 holds the
// occupancy bits of receptor row ((Y - M) mod N, (Z - M) mod N) (zero
// outside the n_rec^3 receptor grid); level k ORs level k-1 with itself
// advanced by 2^(k-1) points (mod N).
template <int N>
__global__ __launch_bounds__(NT) void k_rec_dilate(const uint8_t *__restrict__ occ, int n_rec,
                                                    uint32_t *__restrict__ dil) {
    using D = Dil<N>;
    constexpr int NW = D::NW;
    const int r = (int)blockIdx.x * NT + (int)threadIdx.x;
    if (r >= D::E * D::E) return;
    const int Z = r / D::E, Y = r - (r / D::E) * D::E;
    const int z = (Z - D::M + N) & (N - 1), y = (Y - D::M + N) & (N - 1);
    uint32_t v[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) v[w] = 0u;
    if (z < n_rec && y < n_rec) {
        const uint8_t *row = occ + ((int64_t)z * n_rec + y) * n_rec;
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
        for (int q = 0; q < D::RW; ++q) dil[D::index(k, Z, q, Y)] = v[(q + NW - 1) % NW];
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

// A run of the clash test as two words: the byte offset of its first table
// word for a translation of zero, o = 4 Dil<N>::index(k, z + M, (a + 32) / 32,
// y + M) (the lane adds 4 (t_z RW E + t_y)), and the two window shifts,
// a mod 32 | ((a + len - 2^k) mod 32) << 8 | (second window one word on) << 16,
// with 2^k <= len < 2^(k+1).  The planner keeps z, y, a >= -M and the
// rows and words a translated run reads inside the table.
template <int N>
__device__ __forceinline__ uint2 pack_run(int z, int y, int a, int len) {
    using D = Dil<N>;
    const int ax = a + 32;
    const int k = 31 - __builtin_clz((unsigned)len);
    const int p2 = ax + len - (1 << k);
    const uint32_t off = (uint32_t)(4 * D::index(k, z + D::M, ax >> 5, y + D::M));
    const uint32_t meta = (uint32_t)(ax & 31) | ((uint32_t)(p2 & 31) << 8) | ((uint32_t)((p2 >> 5) > (ax >> 5)) << 16);
    return make_uint2(off, meta);
}
__device__ __forceinline__ int run_pieces(int len) { return (len + RUN_MAX - 1) / RUN_MAX; }
// Write a run as pieces of at most RUN_MAX points from slot pos (slots at
// or past cap are not written); returns the number of pieces.
template <int N>
__device__ __forceinline__ int emit_run(uint2 *out, int pos, int cap, int z, int y, int a, int len) {
    int k = 0;
    for (int o = 0; o < len; o += RUN_MAX, ++k) {
        const int l = len - o < RUN_MAX ? len - o : RUN_MAX;
        if (pos + k < cap) out[pos + k] = pack_run<N>(z, y, a + o, l);
    }
    return k;
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
    uint2 *out = reinterpret_cast<uint2 *>(runs) + c.run_off;
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
        const int len = has ? (int)(xhi - xlo + 1) : 0;
        const int pos = base + block_excl_scan(has ? run_pieces(len) : 0, total, sh);
        if (has) emit_run<N>(out, pos, cap, zc, yc, (int)xlo, len);
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
        // maximal segments of the row (runs start where a set bit follows a
        // clear one), counted in pieces of at most RUN_MAX points
        int cnt = 0;
        for (int pass = 0; pass < 2; ++pass) {
        int pos = pass ? base + block_excl_scan(cnt, total, sh) : 0;
        if (r < nrows) {
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
                if (pass) pos += emit_run<N>(out, pos, cap, z, y, c.xo0 + s, e - s);
                else cnt += run_pieces(e - s);
                x = e;
            }
        }
        }
        base += total;
    }
    if (threadIdx.x == 0) run_count[lc] = base < cap ? base : cap;
}

// ------------------------------------------------------------ clash test
// The test runs in two phases.  Phase 1: one wavefront per (configuration,
// z-translation tz, group of 64 y-translations), lane = ty, tests the atom
// chords and an evenly spread sample of CLASH_R1 runs; rows whose
// translations all clash are done (no free bit), the others are appended to
// the configuration's list of undecided rows.  Phase 2: wavefronts over each
// configuration's list, lane = one undecided row (tz, ty), test every run.
// Only the configurations that still have undecided rows (those near
// clash-free translations) pay for the full run list.
constexpr int CLASH_R1 = 96;

// Runs k in [k0, k1) of one wavefront: run index k itself (phase 2) or the
// k-th of the spread sample (phase 1: the first NCH runs, the atom chords,
// then stride S over the rest).  Lane row (tzl, ty); W output words per
// lane; UR runs in flight (their table words all requested before use).
// Runs are at most 63 points long, so a run's second window starts at most
// one word after its first: the words q1 .. q1 + W + 1 of its row serve both.
template <int N, int W, bool SAMPLE>
__device__ __forceinline__ void clash_runs(const uint2 *__restrict__ rl, int nr, int k1, int NCH, int S, int tzl,
                                           int ty, bool act, uint32_t lm, __amdgpu_buffer_rsrc_t rsrc,
                                           uint32_t *acc) {
    using D = Dil<N>;
    // runs in flight (their table words all requested before use): few, so
    // that the kernel's 42 VGPRs let two of its wavefronts sit beside the z
    // kernel's three on a SIMD when it runs on the second stream
    constexpr int UR = W <= 1 ? 6 : (W == 2 ? 4 : (W == 3 ? 3 : 2));
    // phase 1: position m of the strided walk over the runs after the chords
    int m = 0;
    const int R = nr - NCH;
    auto run_index = [&](int k) {
        if (!SAMPLE || k < NCH) return k;
        const int i = NCH + m;
        m += S;
        if (m >= R) m -= R;
        return i;
    };
    const int vo = (tzl * (D::RW * D::E) + ty) * 4;  // the lane's part of every table offset
    auto test = [&](auto urc, int k) {
        constexpr int U = decltype(urc)::value;
        uint32_t v[U][W + 2];
        uint32_t meta[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint2 e = rl[run_index(k + u)];
            meta[u] = e.y;
#pragma unroll
            for (int j = 0; j < W + 2; ++j)
                v[u][j] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, vo, (int)e.x + j * (D::E * 4), 0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned sh1 = meta[u] & 31u, sh2 = (meta[u] >> 8) & 31u;
            const bool hi2 = (meta[u] >> 16) != 0u;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint32_t o1 = __builtin_amdgcn_alignbit(v[u][w + 1], v[u][w], sh1);
                const uint32_t lo = hi2 ? v[u][w + 1] : v[u][w], hi = hi2 ? v[u][w + 2] : v[u][w + 1];
                acc[w] |= o1 | __builtin_amdgcn_alignbit(hi, lo, sh2);
            }
        }
    };
    auto all_full = [&]() {
        bool full = true;
#pragma unroll
        for (int w = 0; w < W; ++w) full = full && ((w == W - 1) ? ((acc[w] & lm) == lm) : (acc[w] == ~0u));
        return __all(!act || full) != 0;
    };
    int k = 0;
    for (; k + UR <= k1; k += UR) {
        test(std::integral_constant<int, UR>{}, k);
        if (all_full()) return;
    }
    for (; k < k1; ++k) test(std::integral_constant<int, 1>{}, k);
}

template <int N, bool SAMPLE>
__device__ __forceinline__ void clash_dispatch(int W, const uint2 *rl, int nr, int k1, int NCH, int S, int tzl,
                                               int ty, bool act, uint32_t lm, __amdgpu_buffer_rsrc_t rsrc,
                                               uint32_t *acc) {
    constexpr int NW = N / 32;
    switch (W) {  // wave-uniform
    case 1: clash_runs<N, 1, SAMPLE>(rl, nr, k1, NCH, S, tzl, ty, act, lm, rsrc, acc); break;
    case 2: if constexpr (NW >= 2) clash_runs<N, 2, SAMPLE>(rl, nr, k1, NCH, S, tzl, ty, act, lm, rsrc, acc); break;
    case 3: if constexpr (NW >= 3) clash_runs<N, 3, SAMPLE>(rl, nr, k1, NCH, S, tzl, ty, act, lm, rsrc, acc); break;
    case 4: if constexpr (NW >= 4) clash_runs<N, 4, SAMPLE>(rl, nr, k1, NCH, S, tzl, ty, act, lm, rsrc, acc); break;
    default: break;
    }
}

// Phase 1.  Free bits (box-valid and clash-free) of a decided row (tz, ty)
// go to fb[free_off + (tz Vy + ty) W + w], W = ceil(Vx / 32), bit tx & 31 of
// word tx >> 5; an undecided row leaves its clash bits so far there and is
// appended to the list at surv_off as (tz << 16 | ty), scnt[local config]
// counting.  live[item_base + tz ny + g] = 1 iff the group has a free bit
// once decided (0 until phase 2 decides its undecided rows).
template <int N>
__global__ __launch_bounds__(NT) void k_clash1(const int32_t *__restrict__ item_off, int n_cfg, int n_items,
                                                const CfgDev *__restrict__ cfgs, const uint32_t *__restrict__ runs,
                                                const int32_t *__restrict__ run_count,
                                                const uint32_t *__restrict__ dil, uint32_t *__restrict__ fb,
                                                uint8_t *__restrict__ live, uint32_t *__restrict__ surv,
                                                int32_t *__restrict__ scnt) {
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
    const int k1 = min(nr, CLASH_R1);
    const int NCH = min(nr, 32);
    // stride of the spread sample: near 0.618 of the runs after the chords
    const int S = max(1, (nr - NCH) * 618 / 1000) % max(1, nr - NCH);
    const auto rsrc = make_rsrc(dil, (int)(D::words() * 4));
    clash_dispatch<N, true>(W, reinterpret_cast<const uint2 *>(runs) + c.run_off, nr, k1, NCH, S, tz, ty, act, lm,
                            rsrc, acc);
    const bool final = k1 == nr;  // every run tested: the row is decided either way
    bool full = true, any = false;
#pragma unroll
    for (int w = 0; w < NW; ++w)
        if (w < W) {
            const uint32_t f = ~acc[w] & (w == W - 1 ? lm : ~0u);
            full = full && f == 0u;
        }
    if (act) {
        uint32_t *o = fb + c.free_off + ((int64_t)tz * Vy + ty) * W;
#pragma unroll
        for (int w = 0; w < NW; ++w)
            if (w < W) {
                const uint32_t f = ~acc[w] & (w == W - 1 ? lm : ~0u);
                o[w] = (final || full) ? f : acc[w];
                any = any || f != 0u;
            }
    }
    const bool und = act && !full && !final;
    const unsigned long long um = __ballot(und);
    if (um) {
        int base = 0;
        if (lane == 0) base = atomicAdd(&scnt[ic], __popcll(um));
        base = __shfl(base, 0);
        if (und) surv[c.surv_off + base + __popcll(um & ((1ull << lane) - 1ull))] = ((uint32_t)tz << 16) | (uint32_t)ty;
    }
    const unsigned long long bal = __ballot(final && any);
    if (lane == 0) live[c.item_base + loc] = bal != 0ull ? 1 : 0;
}

// Phase 2: wavefront (configuration, w) takes undecided rows [64 w, 64 w +
// 64) of the configuration's list and tests every run.
template <int N>
__global__ __launch_bounds__(NT) void k_clash2(const int32_t *__restrict__ item2_off, int n_cfg, int n_items,
                                                const CfgDev *__restrict__ cfgs, const uint32_t *__restrict__ runs,
                                                const int32_t *__restrict__ run_count,
                                                const uint32_t *__restrict__ dil, uint32_t *__restrict__ fb,
                                                uint8_t *__restrict__ live, const uint32_t *__restrict__ surv,
                                                const int32_t *__restrict__ scnt) {
    using D = Dil<N>;
    constexpr int NW = D::NW;
    const int item = (int)blockIdx.x * (NT / 64) + ((int)threadIdx.x >> 6);
    if (item >= n_items) return;
    const int lane = threadIdx.x & 63;
    const int ic = find_cfg(item2_off, n_cfg, item);
    const int wv = item - item2_off[ic];
    const int cnt = scnt[ic];
    if (64 * wv >= cnt) return;  // wave-uniform
    const CfgDev c = cfgs[ic];
    const int Vx = c.V[0], Vy = c.V[1];
    const int ny = (Vy + 63) >> 6;
    const int idx = 64 * wv + lane;
    const bool act = idx < cnt;
    const uint32_t ent = act ? surv[c.surv_off + idx] : 0u;
    const int tz = (int)(ent >> 16), ty = (int)(ent & 0xffffu);
    const int W = (Vx + 31) >> 5;
    const uint32_t lm = (Vx & 31) ? ((1u << (Vx & 31)) - 1u) : ~0u;
    uint32_t *o = fb + c.free_off + ((int64_t)tz * Vy + ty) * W;
    uint32_t acc[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) acc[w] = (act && w < W) ? o[w] : 0u;
    const int nr = run_count[ic];
    const auto rsrc = make_rsrc(dil, (int)(D::words() * 4));
    clash_dispatch<N, false>(W, reinterpret_cast<const uint2 *>(runs) + c.run_off, nr, nr, 0, 1, tz, ty, act, lm,
                             rsrc, acc);
    bool any = false;
    if (act) {
#pragma unroll
        for (int w = 0; w < NW; ++w)
            if (w < W) {
                const uint32_t f = ~acc[w] & (w == W - 1 ? lm : ~0u);
                o[w] = f;
                any = any || f != 0u;
            }
        if (any) live[c.item_base + tz * ny + (ty >> 6)] = 1;  // same value from every writer
    }
}

__global__ void k_zero32(int32_t *__restrict__ p, int n) {
    const int i = (int)blockIdx.x * NT + (int)threadIdx.x;
    if (i < n) p[i] = 0;
}

// ------------------------------------------------------------ z pass
// A placed atom as the energy inputs use it: x/y lattice position and
// fraction, and its channel weights on its two planes, gamma_ch (1 - fz)
// (plane floor(uz)) and gamma_ch fz (plane floor(uz) + 1).
template <typename T>
struct ZAtom {
    T fx, fy;
    int32_t ax, ay;
    T w[6];
};

// One wavefront per scanned configuration of a chunk: its atoms sorted by
// plane (ties in atom order) into zat[zi][.], and zbt[zi][j] = number of
// atoms on planes below ze0 + j - 1 (j = 0 .. Le + 1): plane j of the energy
// window receives the sorted atoms [zbt[j], zbt[j + 2]), those before
// zbt[j + 1] with weight gamma fz, the rest with gamma (1 - fz).
template <typename T, int N>
__global__ __launch_bounds__(NT) void k_zprep(const CfgDev *__restrict__ cfgs, const int32_t *__restrict__ zcfg,
                                               int nz, int ma, const int32_t *__restrict__ ulat,
                                               const T *__restrict__ gam, ZAtom<T> *__restrict__ zat,
                                               int32_t *__restrict__ zbt) {
    __shared__ int saz[NT / 64][MAXA];
    const int wv = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int zi = (int)blockIdx.x * (NT / 64) + wv;
    if (zi >= nz) return;  // per-wavefront work only, no block barrier below
    const CfgDev c = cfgs[zcfg[zi]];
    const int n = c.n_atoms;
    int *az = saz[wv];
    for (int a = lane; a < n; a += 64) az[a] = ulat[3 * (c.u_base + a) + 2] >> 16;
    wave_sync();
    for (int a = lane; a < n; a += 64) {
        const int z = az[a];
        int rk = 0;
        for (int o = 0; o < n; ++o) rk += (az[o] < z || (az[o] == z && o < a)) ? 1 : 0;
        const int32_t *U = ulat + 3 * (c.u_base + a);
        const T fz = (T)(U[2] & 0xffff) * (T)(1.0 / 65536.0);
        ZAtom<T> r;
        r.fx = (T)(U[0] & 0xffff) * (T)(1.0 / 65536.0);
        r.fy = (T)(U[1] & 0xffff) * (T)(1.0 / 65536.0);
        r.ax = U[0] >> 16;
        r.ay = U[1] >> 16;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const T g = gam[3 * (c.atom_base + a) + ch];
            r.w[ch] = g * ((T)1 - fz);
            r.w[3 + ch] = g * fz;
        }
        zat[(int64_t)zi * ma + rk] = r;
    }
    for (int j = lane; j <= c.Le + 1; j += 64) {
        const int zt = c.ze0 + j - 1;
        int k = 0;
        for (int o = 0; o < n; ++o) k += az[o] < zt ? 1 : 0;
        zbt[(int64_t)zi * (N + 2) + j] = k;
    }
}

// Block -> (tile of P z-pencils, configuration), with the XCD-aware order
// of the plane path's z kernel.  ZHI: the configuration's energy window
// (L_e planes, loaded from plane 0; the correlation of the shifted grid is
// the wanted one shifted by ze0, undone at the store) fits in the lower half
// of the pencil, so the first radix-2 stage is pruned.  CLASH: store only
// the z-translations whose live flag is set; a configuration with none is
// skipped whole.
template <typename T, int N, bool ZHI, bool CLASH>
__global__ __launch_bounds__(NT) void k_zfused(const CfgDev *__restrict__ cfgs, const int32_t *__restrict__ zcfg,
                                                int nz, int n_tiles, int ma, int ac,
                                                const ZAtom<T> *__restrict__ zat, const int32_t *__restrict__ zbt,
                                                const typename Cx<T>::t *__restrict__ rspec,
                                                const typename Cx<T>::t *__restrict__ twg,
                                                typename Cx<T>::t *__restrict__ wsi, const uint8_t *__restrict__ live) {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    constexpr int R1 = G::R1, R2 = G::R2, P = G::U, NP = G::NP, H = G::H, PW = G::PW, PAD = G::PAD;
    constexpr int FP = P + 1;  // table row stride (complex): lanes of different planes on distinct banks
    static_assert(R2 <= 16 && NT % P == 0, "store masks and table columns");
    __shared__ C2 buf[4 * G::WREG];
    __shared__ C2 tw[N];
    __shared__ uint32_t lv[N / 32];
    __shared__ int4 pd[N];        // plane j: atoms [x, z) of plane j - 1 (to y) and of plane j
    __shared__ uint32_t smask[R1];  // bit i: FFT lane n1 stores its output slot i
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
    // dynamic LDS (ma = most atoms of a ligand in the launch): per sorted
    // atom its x/y placement, its channel weights [ch][corner][atom], then
    // the factor table F[ac][FP]
    const int n = c.n_atoms;
    int2 *sxy = (int2 *)dyn;                                                  // [ma] ax, ay
    T *sfr = (T *)(((uintptr_t)(sxy + ma) + 15) & ~(uintptr_t)15);           // [ma][2] fx, fy
    T *swt = sfr + 2 * ma;                                                    // [6][ma]
    C2 *F = (C2 *)(((uintptr_t)(swt + 6 * ma) + 15) & ~(uintptr_t)15);       // [ac][FP]
    load_tw<T, N>(tw, twg);
    for (int a = threadIdx.x; a < n; a += NT) {
        const ZAtom<T> A = zat[(int64_t)zi * ma + a];
        sxy[a] = make_int2(A.ax, A.ay);
        sfr[2 * a] = A.fx;
        sfr[2 * a + 1] = A.fy;
#pragma unroll
        for (int k = 0; k < 6; ++k) swt[k * ma + a] = A.w[k];  // k = corner * 3 + ch: (1 - fz) for 0..2, fz for 3..5
    }
    for (int j = threadIdx.x; j < c.Le; j += NT) {
        const int32_t *zr = zbt + (int64_t)zi * (N + 2) + j;
        pd[j] = make_int4(zr[0], zr[1], zr[2], 0);
    }
    if (threadIdx.x < R1) {
        // FFT lane n1 holds output z = n1 + R1 i, translation (z - ze0) mod N
        uint32_t m = 0u;
#pragma unroll
        for (int i = 0; i < R2; ++i) {
            const int tt = ((int)threadIdx.x + R1 * i - c.ze0) & (N - 1);
            m |= (uint32_t)(tt < Vz && ((lv[tt >> 5] >> (tt & 31)) & 1u)) << i;
        }
        smask[threadIdx.x] = m;
    }
    __syncthreads();
    const ZLane<N> zl;
    const int n1 = zl.n1, p = zl.p;
    C2 *ex = buf + zl.w * G::WREG + zl.pl;
    const int nchunk = (n + ac - 1) / ac;
    const int pen = tile * P + p;
    const bool ok = pen < NP;
    const int rlane = rs_lane<T, N>(n1, ok ? pen : 0);
    auto build_table = [&](int e0) {
        const int na = min(ac, n - e0);
        const int q = (int)threadIdx.x % P;
        const int pq = tile * P + q;
        const bool okq = pq < NP;
        const int kyq = okq ? pq / H : 0, kxq = okq ? pq - (pq / H) * H : 0;
        const C2 wx = tw[kxq & (N - 1)], wy = tw[kyq & (N - 1)];
        for (int e = (int)threadIdx.x / P; e < na; e += NT / P) {
            const int2 axy = sxy[e0 + e];
            const T fx = sfr[2 * (e0 + e)], fy = sfr[2 * (e0 + e) + 1];
            const C2 ex_ = tw[(kxq * axy.x) & (N - 1)], ey = tw[(kyq * axy.y) & (N - 1)];
            const T sxr = (T)1 - fx + fx * wx.x, sxi = fx * wx.y;
            const T syr = (T)1 - fy + fy * wy.x, syi = fy * wy.y;
            const T xr = ex_.x * sxr - ex_.y * sxi, xi = ex_.x * sxi + ex_.y * sxr;
            const T yr = ey.x * syr - ey.y * syi, yi = ey.x * syi + ey.y * syr;
            F[e * FP + q] = okq ? C2{xr * yr - xi * yi, xr * yi + xi * yr} : C2{(T)0, (T)0};
        }
    };
    T er[R2], ei[R2];
#pragma unroll
    for (int i = 0; i < R2; ++i) er[i] = ei[i] = (T)0;
    // Inputs of channel ch: the wavefront computes the values (plane j,
    // pencil pl) of its PW pencils, j-major, into its own exchange region
    // (free until the transform), element j of pencil pl at
    // j PW + (j / R2) PAD + pl; each lane then reads its slots.
    C2 *wbuf = buf + zl.w * G::WREG;
    const int lane = threadIdx.x & 63;
    const int fcol = zl.w * PW;  // first table column of this wavefront's pencils
    constexpr int NIN = ZHI ? R2 / 2 : R2;
#pragma unroll 1
    for (int ch = 0; ch < 3; ++ch) {
        T re[R2], im[R2];
#pragma unroll
        for (int i = 0; i < R2; ++i) re[i] = im[i] = (T)0;
        const T *w1 = swt + (3 + ch) * ma, *w0 = swt + ch * ma;  // weights gamma fz, gamma (1 - fz)
        for (int ck = 0; ck < nchunk; ++ck) {
            const int e0 = ck * ac, e1 = min(n, e0 + ac);
            if (ch == 0 || nchunk > 1) {
                __syncthreads();
                build_table(e0);
                __syncthreads();
            }
            wave_sync();  // the region may still be read by the previous transform
            for (int idx = lane; idx < PW * c.Le; idx += 64) {
                const int j = idx / PW, pl = idx - (idx / PW) * PW;
                const int4 r = pd[j];
                const C2 *fp = F + (fcol + pl) - e0 * FP;
                T ar = (T)0, ai = (T)0;
                for (int e = max(r.x, e0); e < min(r.y, e1); ++e) {  // atoms of plane j - 1: weight gamma fz
                    const C2 f = fp[e * FP];
                    ar += w1[e] * f.x;
                    ai += w1[e] * f.y;
                }
                for (int e = max(r.y, e0); e < min(r.z, e1); ++e) {  // atoms of plane j: weight gamma (1 - fz)
                    const C2 f = fp[e * FP];
                    ar += w0[e] * f.x;
                    ai += w0[e] * f.y;
                }
                C2 &slot = wbuf[j * PW + (j / R2) * PAD + pl];
                if (ck == 0) slot = C2{ar, ai};
                else slot = C2{slot.x + ar, slot.y + ai};
            }
        }
        wave_sync();
#pragma unroll
        for (int i = 0; i < NIN; ++i) {
            const int j = n1 + R1 * i;
            if (j < c.Le) {
                const C2 v = ex[j * PW + (j / R2) * PAD];
                re[i] = v.x;
                im[i] = v.y;
            }
        }
        fft_unit<T, N, false, ZHI>(re, im, n1, ex, PW, tw, true, PAD);
        rprod<T, N, true>(make_rsrc(rspec + (int64_t)ch * N * NP, N * NP * (int)sizeof(C2)), rlane, re, im, er, ei);
    }
    fft_unit_rev<T, N, true>(er, ei, n1, ex, PW, tw, true, PAD);
    // element z = n1 + R1 i of the output is translation t = z - ze0 (mod N);
    // the live ones (t < Vz) are stored, the others fall outside the
    // descriptor
    const auto rd = make_rsrc(wsi + c.off_inv, Vz * NP * (int)sizeof(C2));
    const int oor = Vz * NP * (int)sizeof(C2);
    const uint32_t sm = ok ? smask[n1] : 0u;
#pragma unroll
    for (int i = 0; i < R2; ++i) {
        const int tt = (n1 + R1 * i - c.ze0) & (N - 1);
        buf_store(rd, ((sm >> i) & 1u) ? (tt * NP + pen) * (int)sizeof(C2) : oor, C2{er[i], ei[i]});
    }
}

// z pass from energy planes in device memory (the direct per-atom x/y DFT of
// the forward pass writes plane p of channel ch at off_fwd + (ch L_e + p)
// NP): the same transforms, product and stores as k_zfused, with the next
// channel's planes loaded while the current one is transformed.  Planes at
// or past L_e lie beyond the load descriptor and read as zero.
template <typename T, int N, bool ZHI, bool CLASH>
__global__ __launch_bounds__(NT) void k_zplanes(const CfgDev *__restrict__ cfgs, const int32_t *__restrict__ zcfg,
                                                 int nz, int n_tiles, const typename Cx<T>::t *__restrict__ ws,
                                                 const typename Cx<T>::t *__restrict__ rspec,
                                                 const typename Cx<T>::t *__restrict__ twg,
                                                 typename Cx<T>::t *__restrict__ wsi, const uint8_t *__restrict__ live) {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    constexpr int R1 = G::R1, R2 = G::R2, P = G::U, NP = G::NP, PW = G::PW, PAD = G::PAD;
    static_assert(R2 <= 16, "store masks");
    __shared__ C2 buf[4 * G::WREG];
    __shared__ C2 tw[N];
    __shared__ uint32_t lv[N / 32];
    __shared__ uint32_t smask[R1];  // bit i: FFT lane n1 stores its output slot i
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
    load_tw<T, N>(tw, twg);
    if (threadIdx.x < R1) {
        uint32_t m = 0u;
#pragma unroll
        for (int i = 0; i < R2; ++i) {
            const int tt = ((int)threadIdx.x + R1 * i - c.ze0) & (N - 1);
            m |= (uint32_t)(tt < Vz && ((lv[tt >> 5] >> (tt & 31)) & 1u)) << i;
        }
        smask[threadIdx.x] = m;
    }
    __syncthreads();
    const ZLane<N> zl;
    const int n1 = zl.n1, p = zl.p;
    C2 *ex = buf + zl.w * G::WREG + zl.pl;
    const int pen = tile * P + p;
    const bool ok = pen < NP;
    const int rlane = rs_lane<T, N>(n1, ok ? pen : 0);
    const int po = ok ? pen : NP * N;  // out of every descriptor's range
    constexpr int NIN = ZHI ? R2 / 2 : R2;
    C2 pf[NIN];
    auto fetch = [&](int ch) {
        const auto rs = make_rsrc(ws + c.off_fwd + (int64_t)ch * c.Le * NP, c.Le * NP * (int)sizeof(C2));
#pragma unroll
        for (int i = 0; i < NIN; ++i) pf[i] = buf_load(rs, ((n1 + R1 * i) * NP + po) * (int)sizeof(C2), (C2 *)nullptr);
    };
    T er[R2], ei[R2];
#pragma unroll
    for (int i = 0; i < R2; ++i) er[i] = ei[i] = (T)0;
    fetch(0);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        T re[R2], im[R2];
#pragma unroll
        for (int i = 0; i < R2; ++i) {
            re[i] = i < NIN ? pf[i].x : (T)0;
            im[i] = i < NIN ? pf[i].y : (T)0;
        }
        if (ch < 2) fetch(ch + 1);
        fft_unit<T, N, false, ZHI>(re, im, n1, ex, PW, tw, true, PAD);
        rprod<T, N, true>(make_rsrc(rspec + (int64_t)ch * N * NP, N * NP * (int)sizeof(C2)), rlane, re, im, er, ei);
    }
    fft_unit_rev<T, N, true>(er, ei, n1, ex, PW, tw, true, PAD);
    const auto rd = make_rsrc(wsi + c.off_inv, Vz * NP * (int)sizeof(C2));
    const int oor = Vz * NP * (int)sizeof(C2);
    const uint32_t sm = ok ? smask[n1] : 0u;
#pragma unroll
    for (int i = 0; i < R2; ++i) {
        const int tt = (n1 + R1 * i - c.ze0) & (N - 1);
        buf_store(rd, ((sm >> i) & 1u) ? (tt * NP + pen) * (int)sizeof(C2) : oor, C2{er[i], ei[i]});
    }
}

// ------------------------------------------------------------ inverse xy
// One block per (configuration, box-valid z-translation): inverse y on the
// packed columns, C2R along x on row pairs, Eq. 2 partial over the
// clash-free translations.  CLASH: free bits from k_clash; a plane without
// any is not read (its partial is empty) unless energies are exported.
// WT threads per plane (N = 128: 512, 64 units with one packed column and
// one row pair each, two planes per CU at 4 wavefronts per SIMD).
template <int N>
__host__ __device__ constexpr int inv_fused_threads() {
    return N == 128 ? 512 : NT;
}
template <typename T, int N, bool CLASH, int WT = inv_fused_threads<N>()>
__global__ __launch_bounds__(WT, WT == 512 ? 4 : 1) void k_inv_fused(const int32_t *__restrict__ inv_off, int n_cfg,
                                                   const CfgDev *__restrict__ cfgs,
                                                   const typename Cx<T>::t *__restrict__ wsi, T beta, T inv_n3,
                                                   const typename Cx<T>::t *__restrict__ twg,
                                                   const uint32_t *__restrict__ fb, const uint8_t *__restrict__ live,
                                                   PlanePartial<T> *__restrict__ pp, T *__restrict__ psi_out,
                                                   uint8_t *__restrict__ clash_out,
                                                   unsigned int *__restrict__ e_count) {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    constexpr int R1 = G::R1, R2 = G::R2, M = G::M, S = G::S, U = WT / R1, NP = G::NP;
    constexpr int NW = N / 32;
    static_assert(N + (R1 - 1) * G::RPAD <= 2 * S, "row-pair exchange must fit in two rows");
    __shared__ C2 Pl[N * S];
    __shared__ C2 tw[N];
    __shared__ LseAcc<T> red[WT / 64];
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
    plane_copy<T, N, true, WT>(Pl, const_cast<C2 *>(src));
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
    block_partial_store<T, WT>(acc, red, pp + c.pp_base + tz);
}

// ------------------------------------------------------------ launchers
template <typename T, int N>
struct LaunchFused {
    using C2 = typename Cx<T>::t;
    using G = Geo<T, N>;
    static hipError_t rec_dilate(hipStream_t st, const uint8_t *occ, int n_rec, uint32_t *dil) {
        constexpr int rows = Dil<N>::E * Dil<N>::E;
        hipLaunchKernelGGL((k_rec_dilate<N>), dim3((rows + NT - 1) / NT), dim3(NT), 0, st, occ, n_rec, dil);
        return hipGetLastError();
    }
    static hipError_t lig_runs(hipStream_t st, const CfgDev *cfgs, const int32_t *zcfg, int nz, const int32_t *ulat,
                               const double *thr, uint32_t *runs, int32_t *run_count) {
        if (nz <= 0) return hipSuccess;
        hipLaunchKernelGGL((k_lig_runs<N>), dim3(nz), dim3(NT), 0, st, cfgs, zcfg, ulat, thr, runs, run_count);
        return hipGetLastError();
    }
    static hipError_t clash(hipStream_t st, const int32_t *item_off, const int32_t *item2_off, int n_cfg,
                            int n_items, int n_items2, const CfgDev *cfgs, const uint32_t *runs,
                            const int32_t *run_count, const uint32_t *dil, uint32_t *fb, uint8_t *live,
                            uint32_t *surv, int32_t *scnt) {
        if (n_items <= 0) return hipSuccess;
        hipLaunchKernelGGL(k_zero32, dim3((n_cfg + NT - 1) / NT), dim3(NT), 0, st, scnt, n_cfg);
        hipLaunchKernelGGL((k_clash1<N>), dim3((n_items + NT / 64 - 1) / (NT / 64)), dim3(NT), 0, st, item_off,
                           n_cfg, n_items, cfgs, runs, run_count, dil, fb, live, surv, scnt);
        if (n_items2 > 0)
            hipLaunchKernelGGL((k_clash2<N>), dim3((n_items2 + NT / 64 - 1) / (NT / 64)), dim3(NT), 0, st,
                               item2_off, n_cfg, n_items2, cfgs, runs, run_count, dil, fb, live, surv, scnt);
        return hipGetLastError();
    }
    static int atoms_per_table() {
        constexpr int FP = G::U + 1;
        int a = (int)(FUSED_TABLE_BYTES / (FP * sizeof(C2)));
        return a < 1 ? 1 : a;
    }
    static size_t dyn_bytes(int max_atoms) {
        const int ac = max_atoms < atoms_per_table() ? max_atoms : atoms_per_table();
        size_t o = (size_t)max_atoms * 2 * sizeof(int);
        o = (o + 15) & ~(size_t)15;
        o += (size_t)max_atoms * 8 * sizeof(T);
        o = (o + 15) & ~(size_t)15;
        return o + (size_t)ac * (G::U + 1) * sizeof(C2) + 16;
    }
    static hipError_t zprep(hipStream_t st, const CfgDev *cfgs, const int32_t *zcfg, int nz, int max_atoms,
                            const int32_t *ulat, const void *gam, void *zat, int32_t *zbt) {
        if (nz <= 0) return hipSuccess;
        hipLaunchKernelGGL((k_zprep<T, N>), dim3((nz + NT / 64 - 1) / (NT / 64)), dim3(NT), 0, st, cfgs, zcfg, nz,
                           max_atoms, ulat, (const T *)gam, (ZAtom<T> *)zat, zbt);
        return hipGetLastError();
    }
    static hipError_t zpass(hipStream_t st, bool zhalf, bool clash, const CfgDev *cfgs, const int32_t *zcfg, int nz,
                            int max_atoms, const void *zat, const int32_t *zbt, const void *rspec, const void *tw,
                            void *wsi, const uint8_t *live) {
        if (nz <= 0) return hipSuccess;
        const int n_tiles = (G::NP + G::U - 1) / G::U;
        long long nb = (long long)n_tiles * nz;
        nb = (nb + 7) / 8 * 8;
        const int ac = max_atoms < atoms_per_table() ? max_atoms : atoms_per_table();
        const size_t dyn = dyn_bytes(max_atoms);
#define FFTDG_ZF(Z, C)                                                                                            \
    hipLaunchKernelGGL((k_zfused<T, N, Z, C>), dim3((unsigned)nb), dim3(NT), dyn, st, cfgs, zcfg, nz, n_tiles,      \
                       max_atoms, ac, (const ZAtom<T> *)zat, zbt, (const C2 *)rspec, (const C2 *)tw, (C2 *)wsi, live)
        if (zhalf && clash) FFTDG_ZF(true, true);
        else if (zhalf) FFTDG_ZF(true, false);
        else if (clash) FFTDG_ZF(false, true);
        else FFTDG_ZF(false, false);
#undef FFTDG_ZF
        return hipGetLastError();
    }
    static hipError_t zplanes(hipStream_t st, bool zhalf, bool clash, const CfgDev *cfgs, const int32_t *zcfg,
                              int nz, const void *ws, const void *rspec, const void *tw, void *wsi,
                              const uint8_t *live) {
        if (nz <= 0) return hipSuccess;
        const int n_tiles = (G::NP + G::U - 1) / G::U;
        long long nb = (long long)n_tiles * nz;
        nb = (nb + 7) / 8 * 8;
#define FFTDG_ZP(Z, C)                                                                                     \
    hipLaunchKernelGGL((k_zplanes<T, N, Z, C>), dim3((unsigned)nb), dim3(NT), 0, st, cfgs, zcfg, nz, n_tiles, \
                       (const C2 *)ws, (const C2 *)rspec, (const C2 *)tw, (C2 *)wsi, live)
        if (zhalf && clash) FFTDG_ZP(true, true);
        else if (zhalf) FFTDG_ZP(true, false);
        else if (clash) FFTDG_ZP(false, true);
        else FFTDG_ZP(false, false);
#undef FFTDG_ZP
        return hipGetLastError();
    }
    static hipError_t inv(hipStream_t st, bool clash, const int32_t *inv_off, int n_cfg, int n_items,
                          const CfgDev *cfgs, const void *wsi, double beta, const void *tw, const uint32_t *fb,
                          const uint8_t *live, void *pp, void *psi_out, uint8_t *clash_out, unsigned int *e_count) {
        if (n_items <= 0) return hipSuccess;
        const T b = (T)beta, s = (T)(1.0 / ((double)N * N * N));
        if (clash)
            hipLaunchKernelGGL((k_inv_fused<T, N, true>), dim3(n_items), dim3(inv_fused_threads<N>()), 0, st, inv_off,
                               n_cfg, cfgs,
                               (const C2 *)wsi, b, s, (const C2 *)tw, fb, live, (PlanePartial<T> *)pp, (T *)psi_out,
                               clash_out, e_count);
        else
            hipLaunchKernelGGL((k_inv_fused<T, N, false>), dim3(n_items), dim3(inv_fused_threads<N>()), 0, st, inv_off,
                               n_cfg, cfgs,
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
        Dil<N>::M,
        LaunchFused<T, N>::rec_dilate,
        LaunchFused<T, N>::lig_runs,
        LaunchFused<T, N>::clash,
        LaunchFused<T, N>::zprep,
        sizeof(ZAtom<T>),
        LaunchFused<T, N>::zpass,
        LaunchFused<T, N>::zplanes,
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

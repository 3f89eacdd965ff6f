// Device helpers shared by the scan kernels (gfx950, wave64): plane and
// pencil geometry, work lookup, raw buffer access with hardware range
// checks, LDS plane copies, the receptor-spectrum product of the z pass and
// the max-shifted log-sum-exp partials of Eq. 2.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fft_device.hpp"
#include "scan_types.hpp"

namespace fftdg {

constexpr int NT = 256;
constexpr int MAXA = 256;

template <typename T, int N>
struct Geo {
    static constexpr int R1 = Shape<N>::R1, R2 = Shape<N>::R2, M = R2 / R1;
    static constexpr int H = N / 2 + 1;  // half-spectrum columns
    // LDS row stride (complex elements) of the xy kernels: a column pass has
    // R1 lanes per unit on consecutive rows and the units of a wavefront on
    // consecutive columns; 2*S = 8 (mod 64) words staggers successive rows
    // by 8 banks so every bank is hit exactly twice by a wavefront's 512 B
    // (two cycles, the minimum).
    static constexpr int S = N == 256 ? 132 : (N == 128 ? 68 : (N == 64 ? 36 : 24));
    // pad (complex elements per block of R2) of the row-pair exchanges,
    // moving the lanes of a unit onto distinct bank pairs; the exchange of
    // rows r, r+1 then spans N + (R1-1)*RPAD <= 2*S elements
    static constexpr int RPAD = N == 32 ? 0 : 1;
    static constexpr int NP = N * H;     // complex values per half-plane
    static constexpr int U = NT / R1;    // FFT units per workgroup
    // z-pencil kernels: each wavefront owns PW whole pencils (R1 lanes each);
    // its exchange region holds N elements per pencil plus PAD complex per
    // block of R2 elements.  Element e of pencil pl sits at e PW + (e / R2)
    // PAD + pl.  The 64 lanes reading at once differ in n1 (block e / R2)
    // and pl, so their complex offsets differ by n1 PAD + pl (mod the bank
    // count): PAD = 64 / R1 makes those 64 offsets distinct, every bank is
    // hit equally often and a read takes the minimum number of LDS passes
    // (N = 32 keeps 8: its 16 pencils per wave already spread the offsets).
    static constexpr int PW = 64 / R1;
    static constexpr int PAD = R1 == 16 ? 4 : 8;
    // Receptor spectra, per channel: element (k, pencil), with the PW
    // pencils of a z-kernel wavefront kept together, [pencil / PW][k][PW]:
    // the R1 lanes of a pencil read consecutive k, so each receptor load of
    // a wavefront is one contiguous run.  When a lane's outputs come in
    // adjacent pairs k, k + 1 (M = 2) and FP32, the pairs are interleaved,
    // [pencil / PW][k / 2][PW][2], so one 16-byte load brings both.
    static constexpr bool KPAIR = M == 2 && sizeof(T) == 4;
    static_assert(NP % (64 / R1) == 0, "pencil groups tile the half spectrum");
    __host__ __device__ static constexpr int rs_index(int k, int pen) {
        return KPAIR ? ((pen / PW) * (N / 2) + k / 2) * (2 * PW) + 2 * (pen % PW) + (k & 1)
                     : ((pen / PW) * N + k) * PW + pen % PW;
    }
    static constexpr int WREG = N * PW + R1 * PAD;
};

// Lane layout of the z-pencil kernels: wave w, lane l -> pencil w*PW + l%PW
// of the tile, FFT lane n1 = l / PW.
template <int N>
struct ZLane {
    int w, n1, pl, p;
    __device__ ZLane() {
        constexpr int PW = 64 / Shape<N>::R1;
        w = threadIdx.x >> 6;
        const int l = threadIdx.x & 63;
        n1 = l / PW;
        pl = l - n1 * PW;
        p = w * PW + pl;
    }
};

__device__ __forceinline__ int pmod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}
__device__ __forceinline__ long long floordiv(long long a, long long b) {
    long long q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}
// largest s >= 0 with s*s < rem (rem >= 1)
__device__ __forceinline__ long long isqrt_lt(long long rem) {
    long long s = (long long)sqrt((double)rem);
    while (s > 0 && s * s >= rem) --s;
    while ((s + 1) * (s + 1) < rem) ++s;
    return s;
}

// XCD-aware block order for any grid size: workgroups land on the 8 XCDs
// round-robin (block b on XCD b mod 8), so XCD x is given the contiguous
// logical range [x q + min(x, r), ...) of its blocks, nb = 8 q + r;
// neighbouring logical blocks (e.g. the column tiles of one plane, whose
// rows straddle the same cache lines) then share one L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// Largest i in [0, n) with off[i] <= b, for a running count off[0..n]
// (off[0] = 0 <= b < off[n]); configurations without work repeat a value.
__device__ __forceinline__ int find_cfg(const int32_t *__restrict__ off, int n, int b) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

template <typename T, int N>
__device__ __forceinline__ void load_tw(typename Cx<T>::t *tw, const typename Cx<T>::t *g) {
    for (int i = threadIdx.x; i < N; i += NT) tw[i] = g[i];
}

// Raw buffer access (stride 0): the descriptor covers [base, base + bytes);
// reads at offsets beyond it return 0 and writes there are dropped by the
// hardware, which the z kernel uses to window planes without branches.
// Every descriptor spans only memory owned by the configuration at hand.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, bytes, 0x00020000);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float2 buf_load(__amdgpu_buffer_rsrc_t r, int off, float2 *) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ double2 buf_load(__amdgpu_buffer_rsrc_t r, int off, double2 *) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
// soff: a wave-uniform part of the offset, carried in an SGPR.  Only the
// VGPR part is range-checked, so the sum must lie inside the descriptor.
__device__ __forceinline__ float2 buf_load(__amdgpu_buffer_rsrc_t r, int off, int soff, float2 *) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
}
__device__ __forceinline__ double2 buf_load(__amdgpu_buffer_rsrc_t r, int off, int soff, double2 *) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, soff, 0));
}
__device__ __forceinline__ float4 buf_load4(__amdgpu_buffer_rsrc_t r, int off, int soff) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, off, soff, 0));
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, int off, float2 v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, int off, double2 v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, 0);
}

// Copy one contiguous half-plane [N][H] between global memory and the LDS
// layout [N][S].  Elements travel in aligned pairs (16 B for FP32) and every
// load of a thread is issued before the first LDS store, so a plane costs
// one memory round trip instead of one per element.  g must be 16-byte
// aligned for FP32 (planes start at multiples of NP, which is even).  NTH
// threads take part.
template <typename T, int N, bool TO_LDS, int NTH = NT>
__device__ __forceinline__ void plane_copy(typename Cx<T>::t *Pl, typename Cx<T>::t *g) {
    using C2 = typename Cx<T>::t;
    constexpr int H = N / 2 + 1, S = Geo<T, N>::S, NP = N * H;
    constexpr int NPAIR = NP / 2;
    constexpr int PER = (NPAIR + NTH - 1) / NTH;
    struct alignas(2 * sizeof(C2)) Pair {
        C2 a, b;
    };
    Pair v[PER];
    if (TO_LDS) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int q = threadIdx.x + j * NTH;
            if (q < NPAIR) v[j] = reinterpret_cast<const Pair *>(g)[q];
        }
    }
    // (row, column) of element 2q, q = threadIdx.x + j NTH, stepped by 2 NTH
    // elements per j instead of divided out per element
    constexpr int DY = (2 * NTH) / H, DX = (2 * NTH) % H;
    int y0 = (2 * (int)threadIdx.x) / H, x0 = 2 * (int)threadIdx.x - y0 * H;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int q = threadIdx.x + j * NTH;
        if (q < NPAIR) {
            const bool wrap = x0 + 1 == H;
            const int o0 = y0 * S + x0, o1 = wrap ? (y0 + 1) * S : o0 + 1;
            if (TO_LDS) {
                Pl[o0] = v[j].a;
                Pl[o1] = v[j].b;
            } else {
                v[j].a = Pl[o0];
                v[j].b = Pl[o1];
            }
        }
        x0 += DX;
        y0 += DY;
        if (x0 >= H) {
            x0 -= H;
            ++y0;
        }
    }
    if (!TO_LDS) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int q = threadIdx.x + j * NTH;
            if (q < NPAIR) reinterpret_cast<Pair *>(g)[q] = v[j];
        }
    }
}

// Receptor-spectrum reads of the z kernel.  Lane n1 of pencil pr0 holds the
// spectral slots i R1 + k1, k = R2 k1 + M n1 + i; rs_lane is the lane part of
// their offsets (bytes), the rest is wave-uniform and travels in the SGPR
// offset.  rprod forms R * conj(L) of one channel for all slots: ACC adds
// it to (er, ei), otherwise it overwrites (lr, li) in place.
template <typename T, int N>
__device__ __forceinline__ int rs_lane(int n1, int pr0) {
    using G = Geo<T, N>;
    constexpr int PW = G::PW;
    return (G::KPAIR ? ((pr0 / PW) * (N / 2) + n1) * (2 * PW) + 2 * (pr0 % PW)
                     : ((pr0 / PW) * N + G::M * n1) * PW + pr0 % PW) *
           (int)sizeof(typename Cx<T>::t);
}

template <typename T, int N, bool ACC>
__device__ __forceinline__ void rprod(__amdgpu_buffer_rsrc_t rr, int rlane, T *lr, T *li, T *er, T *ei) {
    using G = Geo<T, N>;
    using C2 = typename Cx<T>::t;
    constexpr int R1 = G::R1, R2 = G::R2, M = G::M, KS = G::PW;  // KS: element stride of k
    auto put = [&](int sl, T rx, T ry) {
        const T a = lr[sl], b = li[sl];
        if (ACC) {
            er[sl] += rx * a + ry * b;
            ei[sl] += ry * a - rx * b;
        } else {
            lr[sl] = rx * a + ry * b;
            li[sl] = ry * a - rx * b;
        }
    };
    if constexpr (G::KPAIR) {
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) {
            const float4 r2 = buf_load4(rr, rlane, R2 * k1 * KS * (int)sizeof(C2));  // k and k + 1
            put(k1, r2.x, r2.y);
            put(R1 + k1, r2.z, r2.w);
        }
    } else {
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) {
                const C2 r = buf_load(rr, rlane, (R2 * k1 + i) * KS * (int)sizeof(C2), (C2 *)nullptr);
                put(i * R1 + k1, r.x, r.y);
            }
    }
}

template <typename T>
struct LseAcc {
    T m, s, pmin;
    int n, amin;
    __device__ void init() {
        m = -(T)INFINITY;
        s = (T)0;
        pmin = (T)INFINITY;
        n = 0;
        amin = -1;
    }
    __device__ void add(T x, T psi, int lin) {
        if (x > m) {
            s = s * exp(m - x) + (T)1;
            m = x;
        } else {
            s += exp(x - m);
        }
        if (psi < pmin || (psi == pmin && lin < amin)) {
            pmin = psi;
            amin = lin;
        }
        ++n;
    }
    __device__ void merge(const LseAcc &o) {
        if (o.n == 0) return;
        if (n == 0) {
            *this = o;
            return;
        }
        const T mm = m > o.m ? m : o.m;
        s = s * exp(m - mm) + o.s * exp(o.m - mm);
        m = mm;
        if (o.pmin < pmin || (o.pmin == pmin && o.amin < amin)) {
            pmin = o.pmin;
            amin = o.amin;
        }
        n += o.n;
    }
};

// Workgroup reduction of the per-thread partials in a fixed tree: a
// butterfly over the lanes of each wavefront (shuffles, no barrier), then
// thread 0 merges the wavefronts' results in order and stores the plane
// partial.  red holds one entry per wavefront of the NTH-thread workgroup.
template <typename T, int NTH = NT>
__device__ __forceinline__ void block_partial_store(LseAcc<T> a, LseAcc<T> *red, PlanePartial<T> *out) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        LseAcc<T> o;
        o.m = __shfl_xor(a.m, off);
        o.s = __shfl_xor(a.s, off);
        o.pmin = __shfl_xor(a.pmin, off);
        o.n = __shfl_xor(a.n, off);
        o.amin = __shfl_xor(a.amin, off);
        a.merge(o);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        LseAcc<T> r = red[0];
        for (int w = 1; w < NTH / 64; ++w) r.merge(red[w]);
        PlanePartial<T> o;
        o.m = r.m;
        o.s = r.s;
        o.psi_min = r.pmin;
        o.n_finite = r.n;
        o.argmin = r.amin;
        *out = o;
    }
}

__device__ __forceinline__ float lse_exp(float d) { return __builtin_amdgcn_exp2f(d * 1.4426950408889634f); }
__device__ __forceinline__ double lse_exp(double d) { return exp(d); }

// Outputs of one lane after the C2R transform of storage rows (y, y+1):
// slot (i R1 + k1) holds x = spec_index(n1, i, k1) of row y in re and of
// row y+1 in im.  Flag bit (i R1 + k1) * 2 + h stands for (x, y + h).
// The energies and occupancies are scaled by inv_n3 in place.  `valid`
// receives the bits of the box-valid translations.  The occupancy pass
// returns the clash flags (C >= 1/2, Eq. 10) of the valid translations; the
// energy pass takes in `clash` the translations to leave out (bits outside
// `valid` are ignored), exports if asked, and folds the rest into the Eq. 2
// partial in two sweeps over registers (the minimum energy, whose -beta
// multiple is the largest exponent, then the sum of exponentials), keeping
// the lowest linear index among equal minima.
template <typename T, int N, bool OCC>
__device__ __forceinline__ uint32_t row_pair_epilogue(T *re, T *im, int n1, int y, int Vx, int Vy, int tz,
                                                      bool occ_pass, uint32_t clash, T inv_n3, T beta,
                                                      T *__restrict__ psi_out, uint8_t *__restrict__ clash_out,
                                                      LseAcc<T> &acc, uint32_t &valid) {
    constexpr int R1 = Shape<N>::R1, R2 = Shape<N>::R2;
    static_assert(2 * R2 <= 32, "one flag word per row pair");
    // slot s = i R1 + k1; value of (x, y + h) in (h ? im : re)[s]; bit 2 s + h
    uint32_t vb = 0;
#pragma unroll
    for (int sl = 0; sl < R2; ++sl) {
        const int x = spec_index<N>(n1, sl / R1, sl % R1);
        re[sl] *= inv_n3;
        im[sl] *= inv_n3;
        vb |= (uint32_t)(x < Vx && y < Vy) << (2 * sl);
        vb |= (uint32_t)(x < Vx && y + 1 < Vy) << (2 * sl + 1);
    }
    valid = vb;
    if (OCC && occ_pass) {
        uint32_t cb = 0;
#pragma unroll
        for (int sl = 0; sl < R2; ++sl) {
            cb |= (uint32_t)(re[sl] >= (T)0.5) << (2 * sl);
            cb |= (uint32_t)(im[sl] >= (T)0.5) << (2 * sl + 1);
        }
        return cb & vb;
    }
    if (psi_out || clash_out) {
#pragma unroll
        for (int sl = 0; sl < R2; ++sl)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int x = spec_index<N>(n1, sl / R1, sl % R1), b = 2 * sl + h;
                if ((vb >> b) & 1u) {
                    const int lin = (tz * Vy + y + h) * Vx + x;
                    if (psi_out) psi_out[lin] = h ? im[sl] : re[sl];
                    if (clash_out) clash_out[lin] = OCC ? (uint8_t)((clash >> b) & 1u) : (uint8_t)0;
                }
            }
    }
    const uint32_t use = vb & ~(OCC ? clash : 0u);
    if (use == 0u) return 0u;
    // minimum psi (its -beta multiple is the maximum of the exponents): the
    // first minimum in (h, x) order, which is the order of the linear index,
    // so the lowest index among equal minima; the index is formed once
    constexpr int M = R2 / R1;
    T pm = (T)INFINITY;
    int best = -1;  // flag bit 2 sl + h of the minimum
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1)
#pragma unroll
            for (int i = 0; i < M; ++i) {
                const int sl = i * R1 + k1;  // x = spec_index(n1, i, k1), increasing in (k1, i)
                const T v = h ? im[sl] : re[sl];
                const bool better = ((use >> (2 * sl + h)) & 1u) && (v < pm || (best < 0 && v == pm));
                pm = better ? v : pm;
                best = better ? 2 * sl + h : best;
            }
    const int sb = best >> 1;
    const int am = best < 0 ? 0x7fffffff
                            : (tz * Vy + y + (best & 1)) * Vx + spec_index<N>(n1, sb / R1, sb % R1);
    const T ml = -beta * pm;
    T sm = (T)0;
#pragma unroll
    for (int sl = 0; sl < R2; ++sl)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const T e = lse_exp(-beta * (h ? im[sl] : re[sl]) - ml);
            sm += ((use >> (2 * sl + h)) & 1u) ? e : (T)0;
        }
    LseAcc<T> o;
    o.m = ml;
    o.s = sm;
    o.pmin = pm;
    o.amin = am;
    o.n = __builtin_popcount(use);
    acc.merge(o);
    return 0u;
}

}  // namespace fftdg

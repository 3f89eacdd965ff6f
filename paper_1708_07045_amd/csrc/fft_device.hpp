// Device FFT building blocks for gfx950 (wave64).
//
// A length-N complex DFT, N = R1 * R2 (R2 = M * R1), is computed by a "unit"
// of R1 lanes.  Lane n1 holds x[n1 + R1*n2], n2 = 0..R2-1, in registers.
// With n = n1 + R1 n2 and k = R2 k1 + k2:
//     X[R2 k1 + k2] = sum_n1 w_R1^(n1 k1) * [ w_N^(n1 k2) * sum_n2 x[n1 + R1 n2] w_R2^(n2 k2) ]
// Pass 1: each lane does an R2-point DFT in registers and the twiddle;
// one exchange through LDS; pass 2: each lane does M R1-point DFTs.
// After the forward routine lane j holds X[R2 k1 + j*M + i] in slot i*R1 + k1
// (the "spectral layout"); the reverse routine takes that layout back to the
// natural one.  Twiddles w_N^k come from a table computed on the host in
// FP64 (cos/sin of 2 pi k / N) and rounded once to the working precision;
// the constants of the in-register DFTs are cos(2 pi k/16) written out.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fftdg {

template <typename T> struct Cx;
template <> struct Cx<float> { using t = float2; };
template <> struct Cx<double> { using t = double2; };

template <int N> struct Shape;
template <> struct Shape<32> { static constexpr int R1 = 4, R2 = 8; };
template <> struct Shape<64> { static constexpr int R1 = 8, R2 = 8; };
template <> struct Shape<128> { static constexpr int R1 = 8, R2 = 16; };
template <> struct Shape<256> { static constexpr int R1 = 16, R2 = 16; };

// cos(2 pi k / 16)
__host__ __device__ constexpr double cos16(int k) {
    switch (k & 15) {
    case 0: return 1.0;
    case 1: return 0.92387953251128675613;
    case 2: return 0.70710678118654752440;
    case 3: return 0.38268343236508977173;
    case 4: return 0.0;
    case 5: return -0.38268343236508977173;
    case 6: return -0.70710678118654752440;
    case 7: return -0.92387953251128675613;
    case 8: return -1.0;
    case 9: return -0.92387953251128675613;
    case 10: return -0.70710678118654752440;
    case 11: return -0.38268343236508977173;
    case 12: return 0.0;
    case 13: return 0.38268343236508977173;
    case 14: return 0.70710678118654752440;
    default: return 0.92387953251128675613;
    }
}
// sin(2 pi k / 16) = cos(2 pi (k - 4) / 16)
__host__ __device__ constexpr double sin16(int k) { return cos16(k - 4); }

__host__ __device__ constexpr int bitrev(int i, int R) {
    int r = 0;
    for (int b = 1; b < R; b <<= 1) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

// (br + i bi) * w16^(+-k): forward uses exp(-2 pi i k/16), inverse exp(+...).
template <bool INV, typename T>
__device__ __forceinline__ void tw16(int k, T br, T bi, T &tr, T &ti) {
    k &= 15;
    if (k == 0) {
        tr = br;
        ti = bi;
    } else if (k == 4) {  // -i (fwd) / +i (inv)
        if (!INV) { tr = bi; ti = -br; } else { tr = -bi; ti = br; }
    } else if (k == 8) {
        tr = -br;
        ti = -bi;
    } else if (k == 12) {  // +i (fwd) / -i (inv)
        if (!INV) { tr = -bi; ti = br; } else { tr = bi; ti = -br; }
    } else {
        const T c = (T)cos16(k);
        const T s = INV ? (T)sin16(k) : (T)(-sin16(k));
        tr = br * c - bi * s;
        ti = br * s + bi * c;
    }
}

// In-register R-point DFT (R in {2,4,8,16}), natural order in and out.
// ZHI: inputs R/2..R-1 are zero (not read); the first radix-2 stage, which
// pairs input n with n + R/2, then reduces to copies.
template <int R, bool INV, typename T, bool ZHI = false>
__device__ __forceinline__ void dft_reg(T *re, T *im) {
    T xr[R], xi[R];
#pragma unroll
    for (int i = 0; i < (ZHI ? R / 2 : R); ++i) {
        xr[bitrev(i, R)] = re[i];
        xi[bitrev(i, R)] = im[i];
    }
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
#pragma unroll
        for (int i = 0; i < R; i += len) {
            if (ZHI && len == 2) {  // bitrev(n + R/2) = bitrev(n) + 1
                xr[i + 1] = xr[i];
                xi[i + 1] = xi[i];
                continue;
            }
#pragma unroll
            for (int j = 0; j < len / 2; ++j) {
                T tr, ti;
                tw16<INV>(j * (16 / len), xr[i + j + len / 2], xi[i + j + len / 2], tr, ti);
                const T ar = xr[i + j], ai = xi[i + j];
                xr[i + j] = ar + tr;
                xi[i + j] = ai + ti;
                xr[i + j + len / 2] = ar - tr;
                xi[i + j + len / 2] = ai - ti;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
        re[i] = xr[i];
        im[i] = xi[i];
    }
}

template <typename T>
__device__ __forceinline__ void cmul_tw(T &r, T &i, typename Cx<T>::t w, bool conj) {
    const T wi = conj ? -w.y : w.y;
    const T nr = r * w.x - i * wi;
    const T ni = r * wi + i * w.x;
    r = nr;
    i = ni;
}

// Orders LDS traffic between the lanes of one wavefront.  A wavefront's LDS
// instructions execute in program order, so only the compiler has to be kept
// from moving loads and stores across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Forward-structured length-N transform by one unit (R1 lanes).
//   in : lane n1 holds x[n1 + R1*n2] in (re,im)[n2]
//   out: lane j holds X[R2*k1 + j*M + i] in (re,im)[i*R1 + k1]
// INV selects the sign of the exponent (no scaling).
// ex[e * es + (e / R2) * pad], e in [0, N): this unit's private LDS exchange
// area (the padding moves the blocks read by different lanes to different
// LDS banks).  The R1
// lanes of a unit must belong to one wavefront: the exchange is ordered with
// wave_sync(), not with a workgroup barrier.  `live` = false makes the unit
// skip its LDS traffic.
// ZHI: the inputs x[z], z >= N/2 (slots n2 >= R2/2) are zero and not read.
// ROT: element e = b R2 + r of the exchange goes to slot b R2 + (r + b) mod
// R2 instead of e (pad unused), a rotation inside each block of R2: for an
// exchange strided through a column of a plane, whose stride puts the
// blocks the R1 lanes read at once on the same bank, it gives them distinct
// banks.
template <typename T, int N, bool INV, bool ZHI = false, bool ROT = false>
__device__ __forceinline__ void fft_unit(T *re, T *im, int n1, typename Cx<T>::t *ex, int es,
                                         const typename Cx<T>::t *tw, bool live, int pad = 0) {
    using C2 = typename Cx<T>::t;
    constexpr int R1 = Shape<N>::R1, R2 = Shape<N>::R2, M = R2 / R1;
    auto slot = [&](int e) {
        return ROT ? ((e / R2) * R2 + (e % R2 + e / R2) % R2) * es : e * es + (e / R2) * pad;
    };
    dft_reg<R2, INV, T, ZHI>(re, im);
#pragma unroll
    for (int k2 = 1; k2 < R2; ++k2) cmul_tw(re[k2], im[k2], tw[n1 * k2], INV);
    wave_sync();  // the exchange area may still be read by a previous step
    if (live) {
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) {
            const int e = k2 * R1 + n1;
            ex[slot(e)] = C2{re[k2], im[k2]};
        }
    }
    wave_sync();
    if (live) {
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int a = 0; a < R1; ++a) {
                const int e = (n1 * M + i) * R1 + a;
                C2 v = ex[slot(e)];
                re[i * R1 + a] = v.x;
                im[i * R1 + a] = v.y;
            }
    }
#pragma unroll
    for (int i = 0; i < M; ++i) dft_reg<R1, INV>(re + i * R1, im + i * R1);
}

// fft_unit for shapes with R1 == R2 (N = 256), twiddles from a per-lane table
// tw2[n1 TW2S + k2] = w_N^(n1 k2) (TW2S = R2 + 1: the lanes' rows on distinct
// banks) and the padded exchange layout: every LDS access of a lane is one
// base address plus an immediate offset, so the routine holds two address
// registers instead of one per element.
template <int N>
struct LaneTw {
    static constexpr int S = Shape<N>::R2 + 1;     // row stride
    static constexpr int SIZE = Shape<N>::R1 * S;  // complex entries
};
template <typename T, int N, bool INV>
__device__ __forceinline__ void fft_unit_lt(T *re, T *im, int n1, typename Cx<T>::t *ex, int es,
                                            const typename Cx<T>::t *tw2, bool live, int pad) {
    using C2 = typename Cx<T>::t;
    constexpr int R1 = Shape<N>::R1, R2 = Shape<N>::R2;
    static_assert(R1 == R2, "one output slot per lane and k1");
    dft_reg<R2, INV, T>(re, im);
    const C2 *tr = tw2 + n1 * LaneTw<N>::S;
#pragma unroll
    for (int k2 = 1; k2 < R2; ++k2) cmul_tw(re[k2], im[k2], tr[k2], INV);
    wave_sync();  // the exchange area may still be read by a previous step
    if (live) {
        C2 *w = ex + n1 * es;  // element k2 R1 + n1 of block k2
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) w[k2 * (R1 * es + pad)] = C2{re[k2], im[k2]};
    }
    wave_sync();
    if (live) {
        const C2 *r = ex + n1 * (R1 * es + pad);  // block n1
#pragma unroll
        for (int a = 0; a < R1; ++a) {
            const C2 v = r[a * es];
            re[a] = v.x;
            im[a] = v.y;
        }
    }
    dft_reg<R1, INV>(re, im);
}

// Reverse of fft_unit's layouts: input in the spectral layout (lane j holds
// X[R2*k1 + j*M + i] in slot i*R1 + k1), output natural (lane n1 holds
// x[n1 + R1*n2] in slot n2).  Same transform definition as fft_unit.
template <typename T, int N, bool INV>
__device__ __forceinline__ void fft_unit_rev(T *re, T *im, int n1, typename Cx<T>::t *ex, int es,
                                             const typename Cx<T>::t *tw, bool live, int pad = 0) {
    using C2 = typename Cx<T>::t;
    constexpr int R1 = Shape<N>::R1, R2 = Shape<N>::R2, M = R2 / R1;
    // R1-point DFT over k1 for each of this lane's k2 = j*M + i, giving
    // Z[a][k2] (a = output index n1'), then twiddle w_N^(a k2).
#pragma unroll
    for (int i = 0; i < M; ++i) {
        dft_reg<R1, INV>(re + i * R1, im + i * R1);
        const int k2 = n1 * M + i;
#pragma unroll
        for (int a = 1; a < R1; ++a) cmul_tw(re[i * R1 + a], im[i * R1 + a], tw[a * k2], INV);
    }
    wave_sync();
    if (live) {
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int a = 0; a < R1; ++a) {
                const int e = (n1 * M + i) * R1 + a;
                ex[e * es + (e / R2) * pad] = C2{re[i * R1 + a], im[i * R1 + a]};
            }
    }
    wave_sync();
    if (live) {
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) {
            const int e = k2 * R1 + n1;
            C2 v = ex[e * es + (e / R2) * pad];
            re[k2] = v.x;
            im[k2] = v.y;
        }
    }
    dft_reg<R2, INV>(re, im);
}

// Output index held in slot (i*R1 + k1) by lane j after fft_unit.
template <int N>
__device__ __forceinline__ int spec_index(int j, int i, int k1) {
    constexpr int R2 = Shape<N>::R2, M = Shape<N>::R2 / Shape<N>::R1;
    return R2 * k1 + j * M + i;
}

}  // namespace fftdg

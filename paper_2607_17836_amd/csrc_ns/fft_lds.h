// Complex FFT of N = 64, 128, ..., 4096 FP64 points held in LDS, computed by
// one workgroup of N / 8 threads.
//
// Stockham autosort formulation (Govindaraju et al., "High performance
// discrete Fourier transforms on graphics processors", SC 2008): pass p of
// radix R reads butterfly j's R inputs at stride N / R, twists input r by
// exp(-+2 pi i r k / (Ns R)) with k = j mod Ns (Ns = product of the earlier
// radices), applies the R-point DFT and writes the outputs at stride Ns
// starting from (j - k) R + k; after the last pass the result is in natural
// order.  Radix-8 passes and a last 2 or 4 where log2 N is not a multiple of
// 3 (64 = 8 8, 128 = 8 8 2, 256 = 8 8 4, 512 = 8 8 8, 1024 = 8 8 8 2,
// 2048 = 8 8 8 4, 4096 = 8 8 8 8).  Each pass first reads all of a
// thread's inputs into registers, then (after a barrier) writes, so one LDS
// buffer suffices.  Forward: exp(-2 pi i jk / N); inverse: exp(+2 pi i jk / N),
// unnormalised.  Twiddles come from a table W[m] = exp(-2 pi i m / N).
#pragma once

#include <hip/hip_runtime.h>

namespace ns_fft {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// z * (-i) for the forward transform, z * (+i) for the inverse.
template <bool INV>
__device__ __forceinline__ double2 rot90(double2 z)
{
    return INV ? make_double2(-z.y, z.x) : make_double2(z.y, -z.x);
}

template <bool INV>
__device__ __forceinline__ void dft2(double2 *v)
{
    const double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

// 4-point DFT in natural order.
template <bool INV>
__device__ __forceinline__ void dft4(double2 *v)
{
    const double2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const double2 t2 = cadd(v[1], v[3]), t3 = rot90<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
}

// 8-point DFT in natural order: 4-point DFTs of the even and odd inputs,
// combined with the eighth roots of unity.
template <bool INV>
__device__ __forceinline__ void dft8(double2 *v)
{
    constexpr double c = 0.70710678118654752440;   // sqrt(1/2)
    double2 e[4] = {v[0], v[2], v[4], v[6]};
    double2 o[4] = {v[1], v[3], v[5], v[7]};
    dft4<INV>(e);
    dft4<INV>(o);
    // w^s = exp(-+2 pi i s / 8)
    const double2 o1 = INV ? make_double2(c * (o[1].x - o[1].y), c * (o[1].x + o[1].y))
                           : make_double2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
    const double2 o2 = rot90<INV>(o[2]);
    const double2 o3 = INV ? make_double2(-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y))
                           : make_double2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
}

template <int R, bool INV>
__device__ __forceinline__ void dft(double2 *v)
{
    if constexpr (R == 8) dft8<INV>(v);
    else if constexpr (R == 4) dft4<INV>(v);
    else dft2<INV>(v);
}

// One Stockham pass of radix R with Ns = product of the earlier radices.
// Entered and left with the block synchronised.
template <int N, int R, bool INV>
__device__ __forceinline__ void pass(double2 *buf, int Ns, const double2 *__restrict__ W)
{
    constexpr int T = N / 8;          // threads
    constexpr int B = N / R / T;      // butterflies per thread
    const int t = threadIdx.x;
    double2 v[B][R];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + b * T;
        const int k = j & (Ns - 1);
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = buf[j + r * (N / R)];
        if (Ns > 1) {
            const int step = N / (Ns * R);
#pragma unroll
            for (int r = 1; r < R; ++r) {
                double2 w = W[r * k * step];
                if (INV) w.y = -w.y;
                v[b][r] = cmul(v[b][r], w);
            }
        }
        dft<R, INV>(v[b]);
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = t + b * T;
        const int k = j & (Ns - 1);
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) buf[base + r * Ns] = v[b][r];
    }
    __syncthreads();
}

// In-place N-point transform of buf by the whole block (blockDim.x == N / 8).
// The caller synchronises the block after filling buf; the block is
// synchronised on return.
template <int N, bool INV>
__device__ __forceinline__ void fft(double2 *buf, const double2 *__restrict__ W)
{
    static_assert(N >= 64 && N <= 4096 && (N & (N - 1)) == 0, "built-in transform sizes");
    pass<N, 8, INV>(buf, 1, W);
    pass<N, 8, INV>(buf, 8, W);
    if constexpr (N == 128) pass<N, 2, INV>(buf, 64, W);
    if constexpr (N == 256) pass<N, 4, INV>(buf, 64, W);
    if constexpr (N >= 512) pass<N, 8, INV>(buf, 64, W);
    if constexpr (N == 1024) pass<N, 2, INV>(buf, 512, W);
    if constexpr (N == 2048) pass<N, 4, INV>(buf, 512, W);
    if constexpr (N == 4096) pass<N, 8, INV>(buf, 512, W);
}

}  // namespace ns_fft

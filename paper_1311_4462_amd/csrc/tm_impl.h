// Internal definitions shared by the HIP kernels and the host runtime.
// Field layouts are those documented in include/tm.h.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "../../include/tm.h"

namespace twm {

constexpr int kMaxProblems = 8;   // problems per batched launch

// Doublet hop kernels can put the two flavours of a site on a lane pair
// (build with TM_ND_SPLIT=1); measured 2-4% slower than one thread per site,
// so off by default.
#ifndef TM_ND_SPLIT
#define TM_ND_SPLIT 0
#endif
constexpr bool kNdSplit = TM_ND_SPLIT != 0;
constexpr int kBlock = 256;       // default threads per block
// Device scratch of the allocation-free operator call: 256 MiB per GPU
// (the odd temporary of the 32^3 x 64 FP32 doublet operator is 192 MiB).
constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;

// ------------------------------------------------------------------ complex

template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ cx<T> cjmul(cx<T> a, cx<T> b)
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.im, a.re}; }
template <typename T>
__device__ __forceinline__ cx<T> times_mi(cx<T> a) { return {a.im, -a.re}; }

// ------------------------------------------------------------------ precision

template <int P>
struct Prec;

template <>
struct Prec<TM_FP64> {
    using real = double;
    static constexpr int kChunkBytes = 16;   // one complex
    static constexpr int kCplxPerChunk = 1;
    static constexpr bool kScaled = false;
};
template <>
struct Prec<TM_FP32> {
    using real = float;
    static constexpr int kChunkBytes = 16;   // two complex (float4)
    static constexpr int kCplxPerChunk = 2;
    static constexpr bool kScaled = false;
};
template <>
struct Prec<TM_FP16> {
    using real = float;
    static constexpr int kChunkBytes = 16;   // four complex as eight fp16
    static constexpr int kCplxPerChunk = 4;
    static constexpr bool kScaled = true;
};
template <>
struct Prec<TM_BF16> {
    using real = float;
    static constexpr int kChunkBytes = 16;   // four complex as eight bf16
    static constexpr int kCplxPerChunk = 4;
    static constexpr bool kScaled = true;
};

template <int P>
constexpr int nchunks() { return 12 / Prec<P>::kCplxPerChunk; }

// bytes of the chunk part of one parity field, rounded to 256
__host__ __device__ inline size_t chunk_bytes(int prec, long vh, int nf, int nrhs)
{
    const size_t nch = (prec == TM_FP64) ? 12 : (prec == TM_FP32 ? 6 : 3);   // 16-byte chunks
    size_t b = 16 * nch * (size_t)vh * nf * nrhs;
    return (b + 255) & ~(size_t)255;
}
__host__ __device__ inline size_t spinor_field_bytes(int prec, long vh, int nf, int nrhs)
{
    size_t b = chunk_bytes(prec, vh, nf, nrhs);
    if (prec == TM_FP16 || prec == TM_BF16) b += (((size_t)vh * nf * nrhs * 4) + 255) & ~(size_t)255;
    return b;
}

// fp16 / bf16 scalar conversions
__device__ __forceinline__ float h2f(uint16_t h)
{
    _Float16 v;
    __builtin_memcpy(&v, &h, 2);
    return (float)v;
}
__device__ __forceinline__ uint16_t f2h(float f)
{
    _Float16 v = (_Float16)f;
    uint16_t h;
    __builtin_memcpy(&h, &v, 2);
    return h;
}
__device__ __forceinline__ float b2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ uint16_t f2b(float f)
{
    // round to nearest even; inputs are finite and |f| <= 1 after scaling
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <int P>
__device__ __forceinline__ float half_to_f(uint16_t v)
{
    if constexpr (P == TM_FP16) return h2f(v); else return b2f(v);
}
template <int P>
__device__ __forceinline__ uint16_t f_to_half(float v)
{
    if constexpr (P == TM_FP16) return f2h(v); else return f2b(v);
}

// Non-temporal vector loads (streamed data that is read once per launch).
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef unsigned int nt_u2 __attribute__((ext_vector_type(2)));
typedef unsigned int nt_u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double2 ld_nt(const double2 *p)
{
    nt_d2 v = __builtin_nontemporal_load((const nt_d2 *)p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ float4 ld_nt(const float4 *p)
{
    nt_f4 v = __builtin_nontemporal_load((const nt_f4 *)p);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 ld_nt(const float2 *p)
{
    nt_f2 v = __builtin_nontemporal_load((const nt_f2 *)p);
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ uint2 ld_nt(const uint2 *p)
{
    nt_u2 v = __builtin_nontemporal_load((const nt_u2 *)p);
    return make_uint2(v.x, v.y);
}
__device__ __forceinline__ uint4 ld_nt(const uint4 *p)
{
    nt_u4 v = __builtin_nontemporal_load((const nt_u4 *)p);
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint32_t ld_nt(const uint32_t *p)
{
    return __builtin_nontemporal_load(p);
}

// Non-temporal vector stores (streamed results no kernel of the launch reads).
__device__ __forceinline__ void st_nt(double2 *p, double2 v)
{
    __builtin_nontemporal_store((nt_d2){v.x, v.y}, (nt_d2 *)p);
}
__device__ __forceinline__ void st_nt(float4 *p, float4 v)
{
    __builtin_nontemporal_store((nt_f4){v.x, v.y, v.z, v.w}, (nt_f4 *)p);
}
__device__ __forceinline__ void st_nt(uint4 *p, uint4 v)
{
    __builtin_nontemporal_store((nt_u4){v.x, v.y, v.z, v.w}, (nt_u4 *)p);
}
template <bool NT, typename T>
__device__ __forceinline__ T lds_(const T *p)
{
    if constexpr (NT) return ld_nt(p); else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void sts_(T *p, T v)
{
    if constexpr (NT) st_nt(p, v); else *p = v;
}

// Streams of a hop launch accessed non-temporally (HopBatch::nt_streams):
// each is touched once per launch, so it need not displace the neighbour
// spinors that several threads re-read from L2.
constexpr int kNtOut = 1;     // output stores
constexpr int kNtX = 2;       // xpay operand loads
constexpr int kNtTime = 4;    // time-neighbour loads (their other users run a time slice later)

// ------------------------------------------------------------------ spinor access
//
// A parity field of nrhs x nf sites-vectors: chunk array + optional scales.
// Site vector element k = 3*spin + colour.

struct SpinorPtr {
    void *data;      // chunk array
    float *scale;    // per (rhs, flavour, site) scale (half precisions)
};

// Addressing: every (rhs, flavour, chunk) row starts at a wave-uniform base
// pointer, and a lane adds the 32-bit offset cb * chunk bytes, so a load
// needs one VGPR for the offset whatever the chunk (scalar base + vector
// offset addressing).
template <typename T>
__device__ __forceinline__ const T *at(const void *base, uint32_t off)
{
    return (const T *)((const char *)base + off);
}
template <typename T>
__device__ __forceinline__ T *at_w(void *base, uint32_t off)
{
    return (T *)((char *)base + off);
}

template <int P>
struct SpinorIO {
    using real = typename Prec<P>::real;
    static constexpr int CB = Prec<P>::kChunkBytes;
    static constexpr int NCH = nchunks<P>();

    __device__ static __forceinline__ const char *row(const SpinorPtr &s, uint32_t vh, uint32_t vec,
                                                      int chunk)
    {
        return (const char *)s.data + ((size_t)vec * NCH + chunk) * vh * CB;
    }

    // Load complex elements [K0, K0 + N) (multiples of the chunk size) of
    // vector vec = rhs * nf + flavour at site cb.
    template <int K0, int N, bool NT = false>
    __device__ static __forceinline__ void load(cx<real> *v, const SpinorPtr &s, uint32_t vh,
                                                uint32_t vec, uint32_t cb)
    {
        const uint32_t off = cb * CB;
        if constexpr (P == TM_FP64) {
#pragma unroll
            for (int k = 0; k < N; k++) {
                double2 c = lds_<NT>(at<double2>(row(s, vh, vec, K0 + k), off));
                v[k] = mk(c.x, c.y);
            }
        } else if constexpr (P == TM_FP32) {
#pragma unroll
            for (int k = 0; k < N / 2; k++) {
                float4 c = lds_<NT>(at<float4>(row(s, vh, vec, K0 / 2 + k), off));
                v[2 * k] = mk(c.x, c.y);
                v[2 * k + 1] = mk(c.z, c.w);
            }
        } else {
            // 16-byte chunks of four complex: elements 0-3 | 4-7 | 8-11; the
            // upper spin pair (0-5) is chunk 0 and the low half of chunk 1.
            const float sc = *at<float>(s.scale + (size_t)vec * vh, cb * 4u);
            if constexpr (K0 == 0 && N == 12) {
#pragma unroll
                for (int k = 0; k < 3; k++) unpack4(v + 4 * k, lds_<NT>(at<uint4>(row(s, vh, vec, k), off)), sc);
            } else if constexpr (K0 == 0 && N == 6) {
                unpack4(v, *at<uint4>(row(s, vh, vec, 0), off), sc);
                unpack2(v + 4, *at<uint2>(row(s, vh, vec, 1), off), sc);
            } else {
                static_assert(K0 == 6 && N == 6, "half-precision loads: full site or one spin pair");
                unpack2(v, *at<uint2>(row(s, vh, vec, 1), off + 8u), sc);
                unpack4(v + 2, *at<uint4>(row(s, vh, vec, 2), off), sc);
            }
        }
    }

    // As load, but half-precision values come without the site scale, which
    // is returned in sc (FP32 / FP64: sc = 1), so that a caller that is linear
    // in v applies it once to its result.
    template <int K0, int N, bool NT = false>
    __device__ static __forceinline__ void load_unscaled(cx<real> *v, const SpinorPtr &s, uint32_t vh,
                                                         uint32_t vec, uint32_t cb, real &sc)
    {
        if constexpr (P == TM_FP64 || P == TM_FP32) {
            load<K0, N, NT>(v, s, vh, vec, cb);
            sc = (real)1;
        } else {
            const uint32_t off = cb * CB;
            sc = *at<float>(s.scale + (size_t)vec * vh, cb * 4u);
            if constexpr (K0 == 0 && N == 12) {
#pragma unroll
                for (int k = 0; k < 3; k++) unpack4(v + 4 * k, *at<uint4>(row(s, vh, vec, k), off), 1.0f);
            } else if constexpr (K0 == 0 && N == 6) {
                unpack4(v, lds_<NT>(at<uint4>(row(s, vh, vec, 0), off)), 1.0f);
                unpack2(v + 4, lds_<NT>(at<uint2>(row(s, vh, vec, 1), off)), 1.0f);
            } else {
                static_assert(K0 == 6 && N == 6, "half-precision loads: full site or one spin pair");
                unpack2(v, lds_<NT>(at<uint2>(row(s, vh, vec, 1), off + 8u)), 1.0f);
                unpack4(v + 2, lds_<NT>(at<uint4>(row(s, vh, vec, 2), off)), 1.0f);
            }
        }
    }

    // Half precision: the stored words of complex elements [K0, K0 + N)
    // (real part in the low 16 bits) and the site scale.
    template <int K0, int N, bool NT = false>
    __device__ static __forceinline__ void load_words(uint32_t *w, const SpinorPtr &s, uint32_t vh,
                                                      uint32_t vec, uint32_t cb, float &sc)
    {
        static_assert(P == TM_FP16 || P == TM_BF16, "stored words: half precision");
        const uint32_t off = cb * CB;
        sc = *at<float>(s.scale + (size_t)vec * vh, cb * 4u);
        auto put4 = [](uint32_t *o, uint4 c) {
            o[0] = c.x;
            o[1] = c.y;
            o[2] = c.z;
            o[3] = c.w;
        };
        if constexpr (K0 == 0 && N == 12) {
#pragma unroll
            for (int k = 0; k < 3; k++) put4(w + 4 * k, *at<uint4>(row(s, vh, vec, k), off));
        } else if constexpr (K0 == 0 && N == 6) {
            put4(w, lds_<NT>(at<uint4>(row(s, vh, vec, 0), off)));
            const uint2 c = lds_<NT>(at<uint2>(row(s, vh, vec, 1), off));
            w[4] = c.x;
            w[5] = c.y;
        } else {
            static_assert(K0 == 6 && N == 6, "half-precision loads: full site or one spin pair");
            const uint2 c = lds_<NT>(at<uint2>(row(s, vh, vec, 1), off + 8u));
            w[0] = c.x;
            w[1] = c.y;
            put4(w + 2, lds_<NT>(at<uint4>(row(s, vh, vec, 2), off)));
        }
    }

    __device__ static __forceinline__ void unpack2(cx<real> *v, uint2 c, float sc)
    {
        v[0] = mk(sc * half_to_f<P>(c.x & 0xffff), sc * half_to_f<P>(c.x >> 16));
        v[1] = mk(sc * half_to_f<P>(c.y & 0xffff), sc * half_to_f<P>(c.y >> 16));
    }
    __device__ static __forceinline__ void unpack4(cx<real> *v, uint4 c, float sc)
    {
        unpack2(v, make_uint2(c.x, c.y), sc);
        unpack2(v + 2, make_uint2(c.z, c.w), sc);
    }
    __device__ static __forceinline__ uint32_t pack1(cx<real> a, float inv)
    {
        return (uint32_t)f_to_half<P>(a.re * inv) | ((uint32_t)f_to_half<P>(a.im * inv) << 16);
    }

    // Store the full site vector (12 complex); NT: non-temporal stores.
    template <bool NT = false>
    __device__ static __forceinline__ void store(const SpinorPtr &s, uint32_t vh, uint32_t vec,
                                                 uint32_t cb, const cx<real> *v)
    {
        const uint32_t off = cb * CB;
        if constexpr (P == TM_FP64) {
#pragma unroll
            for (int k = 0; k < 12; k++)
                sts_<NT>(at_w<double2>((void *)row(s, vh, vec, k), off), make_double2(v[k].re, v[k].im));
        } else if constexpr (P == TM_FP32) {
#pragma unroll
            for (int k = 0; k < 6; k++)
                sts_<NT>(at_w<float4>((void *)row(s, vh, vec, k), off),
                         make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im));
        } else {
            float m = 0.f;
#pragma unroll
            for (int k = 0; k < 12; k++) m = fmaxf(m, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
            const float inv = (m > 0.f) ? 1.0f / m : 0.f;
#pragma unroll
            for (int k = 0; k < 3; k++)
                sts_<NT>(at_w<uint4>((void *)row(s, vh, vec, k), off),
                         make_uint4(pack1(v[4 * k], inv), pack1(v[4 * k + 1], inv), pack1(v[4 * k + 2], inv),
                                    pack1(v[4 * k + 3], inv)));
            *at_w<float>(s.scale + (size_t)vec * vh, cb * 4u) = m;
        }
    }
};

// Link loads: non-temporal (NT) or ordinary.
template <bool NT, typename T>
__device__ __forceinline__ T ldl(const T *p)
{
    if constexpr (NT) return ld_nt(p); else return *p;
}

// ------------------------------------------------------------------ links
//
// Links of one parity: [mu][elem-chunk][cb].  recon 12 stores rows 0, 1 (6
// complex), recon 18 all 9.  Chunking: FP64 one complex per 16-byte chunk;
// FP32 recon 12 two complex per float4, recon 18 one complex per float2;
// FP16/BF16 recon 12 two complex per 8 bytes, recon 18 one complex per 4 bytes.

__host__ __device__ inline size_t link_elem_bytes(int prec)
{
    return prec == TM_FP64 ? 16 : (prec == TM_FP32 ? 8 : 4);
}
__host__ __device__ inline size_t gauge_parity_bytes(int prec, int recon, long vh)
{
    size_t b = link_elem_bytes(prec) * (recon == 12 ? 6 : (recon == 8 ? 4 : 9)) * 4 * (size_t)vh;
    return (b + 255) & ~(size_t)255;
}

// conj(p q - r s), each part one FMA chain of four terms.
template <typename T>
__device__ __forceinline__ cx<T> conj_cross(cx<T> p, cx<T> q, cx<T> r, cx<T> s)
{
    T re = p.re * q.re;
    re = fma(-p.im, q.im, re);
    re = fma(-r.re, s.re, re);
    re = fma(r.im, s.im, re);
    T im = r.re * s.im;
    im = fma(r.im, s.re, im);
    im = fma(-p.re, q.im, im);
    im = fma(-p.im, q.re, im);
    return mk(re, im);
}

// Link rows of one parity (all [mu][cb], 16-byte rows first):
//   FP64       NE rows of one complex (double2)
//   FP32  12:  3 rows of two complex (float4)
//   FP32  18:  4 rows of two complex (float4), then 1 row of one complex (float2)
//   FP32   8:  2 rows of two complex (float4)
//   half  12:  1 row of four complex (16 B), then 1 row of two complex (8 B)
//   half  18:  2 rows of four complex (16 B), then 1 row of one complex (4 B)
//   half   8:  1 row of four complex (16 B)
// Stored elements, row-major: 12 -> rows 0 and 1; 18 -> all nine; 8 -> a2, a3,
// b1 and (arg a1, arg c1) as the real and imaginary part of the fourth slot
// (a, b, c the rows of the link).
template <int P, int RECON, bool NT = true>
struct LinkIO {
    using real = typename Prec<P>::real;
    // half-precision 8-real links: phase = k * pi / 32767, k a 16-bit integer
    static constexpr double kPhaseStepD = 3.14159265358979323846 / 32767.0;
    static constexpr real kPhaseStep = (real)kPhaseStepD;
    static constexpr int NE = (RECON == 12) ? 6 : (RECON == 8 ? 4 : 9);
    static constexpr int NR32 = NE / 2;         // FP32 16-byte rows (two complex each)
    static constexpr int NR16 = NE / 4;         // half 16-byte rows (four complex each)
    static constexpr int T16 = NE % 4;          // half tail: complex per site

    // start of the 16-byte row k, and of the narrow tail row
    __device__ static __forceinline__ const char *row16(const void *base, uint32_t vh, int mu, int k,
                                                        int nrow)
    {
        return (const char *)base + ((size_t)mu * nrow + k) * vh * 16;
    }
    __device__ static __forceinline__ const char *tail(const void *base, uint32_t vh, int mu, int nrow16,
                                                       int tbytes)
    {
        return (const char *)base + (size_t)4 * nrow16 * vh * 16 + (size_t)mu * vh * tbytes;
    }

    __device__ static __forceinline__ cx<real> h2c(uint32_t c)
    {
        return mk(half_to_f<P>(c & 0xffff), half_to_f<P>(c >> 16));
    }

    // 8-real links.  Unit norm of row a and of column 1 give |a1|^2 = 1 - N,
    // N = |a2|^2 + |a3|^2, and |c1|^2 = N - |b1|^2.  Orthogonality of a to b
    // and c, with b = conj(c x a) and c = conj(a x b) (det U = 1), leaves a
    // 2x2 linear system for each of (b2, b3) and (c2, c3), of determinant N:
    //   b2 = -(a3* c1* + a1* a2 b1) / N     b3 = (a2* c1* - a1* a3 b1) / N
    //   c2 =  (a3* b1* - a1* a2 c1) / N     c3 = -(a2* b1* + a1* a3 c1) / N
    // Links with N = 0 (a1 of modulus one) cannot be represented; the gauge
    // upload rejects them.
    __device__ static __forceinline__ void recon8(cx<real> (&u)[3][3], cx<real> a2, cx<real> a3,
                                                  cx<real> b1, real tha, real thc)
    {
        const real n = a2.re * a2.re + a2.im * a2.im + a3.re * a3.re + a3.im * a3.im;
        const real ra = sqrt(fmax(real(1) - n, real(0)));
        const real rc = sqrt(fmax(n - (b1.re * b1.re + b1.im * b1.im), real(0)));
        real sa, ca, sc, cc;
        if constexpr (sizeof(real) == 8) {
            sincos(tha, &sa, &ca);
            sincos(thc, &sc, &cc);
        } else {
            // hardware sine / cosine: absolute error ~1e-6 on [-pi, pi]
            __sincosf(tha, &sa, &ca);
            __sincosf(thc, &sc, &cc);
        }
        const cx<real> a1 = mk(ra * ca, ra * sa), c1 = mk(rc * cc, rc * sc);
        const real in = real(1) / n;
        const cx<real> a2b1 = cjmul(a1, cmul(a2, b1)), a3b1 = cjmul(a1, cmul(a3, b1));
        const cx<real> a2c1 = cjmul(a1, cmul(a2, c1)), a3c1 = cjmul(a1, cmul(a3, c1));
        const cx<real> a3c1s = conjg(cmul(a3, c1)), a2c1s = conjg(cmul(a2, c1));
        const cx<real> a3b1s = conjg(cmul(a3, b1)), a2b1s = conjg(cmul(a2, b1));
        u[0][0] = a1;
        u[0][1] = a2;
        u[0][2] = a3;
        u[1][0] = b1;
        u[1][1] = (-in) * (a3c1s + a2b1);
        u[1][2] = in * (a2c1s - a3b1);
        u[2][0] = c1;
        u[2][1] = in * (a3b1s - a2c1);
        u[2][2] = (-in) * (a2b1s + a3c1);
    }

    __device__ static __forceinline__ void load(cx<real> (&u)[3][3], const void *base, uint32_t vh,
                                                int mu, uint32_t cb)
    {
        cx<real> e[9];
        const uint32_t o16 = cb * 16u;
        if constexpr (P == TM_FP64) {
#pragma unroll
            for (int k = 0; k < NE; k++) {
                double2 c = ldl<NT>(at<double2>(row16(base, vh, mu, k, NE), o16));
                e[k] = mk(c.x, c.y);
            }
        } else if constexpr (P == TM_FP32) {
#pragma unroll
            for (int k = 0; k < NR32; k++) {
                float4 c = ldl<NT>(at<float4>(row16(base, vh, mu, k, NR32), o16));
                e[2 * k] = mk(c.x, c.y);
                e[2 * k + 1] = mk(c.z, c.w);
            }
            if constexpr (NE % 2 == 1) {
                float2 c = ldl<NT>(at<float2>(tail(base, vh, mu, NR32, 8), cb * 8u));
                e[NE - 1] = mk(c.x, c.y);
            }
        } else {
#pragma unroll
            for (int k = 0; k < NR16; k++) {
                uint4 c = ldl<NT>(at<uint4>(row16(base, vh, mu, k, NR16), o16));
                e[4 * k] = h2c(c.x);
                e[4 * k + 1] = h2c(c.y);
                e[4 * k + 2] = h2c(c.z);
                if constexpr (RECON == 8)
                    e[3] = mk(kPhaseStep * (real)(int16_t)(c.w & 0xffff), kPhaseStep * (real)(int16_t)(c.w >> 16));
                else
                    e[4 * k + 3] = h2c(c.w);
            }
            if constexpr (T16 == 2) {
                uint2 c = ldl<NT>(at<uint2>(tail(base, vh, mu, NR16, 8), cb * 8u));
                e[4 * NR16] = h2c(c.x);
                e[4 * NR16 + 1] = h2c(c.y);
            } else if constexpr (T16 == 1) {
                uint32_t c = ldl<NT>(at<uint32_t>(tail(base, vh, mu, NR16, 4), cb * 4u));
                e[4 * NR16] = h2c(c);
            }
        }
        if constexpr (RECON == 8) {
            recon8(u, e[0], e[1], e[2], e[3].re, e[3].im);
        } else {
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int b = 0; b < 3; b++) u[a][b] = e[3 * a + b];
            if constexpr (RECON == 12) {
                // third row of an SU(3) matrix: conj(row0 x row1)
                u[2][0] = conj_cross(u[0][1], u[1][2], u[0][2], u[1][1]);
                u[2][1] = conj_cross(u[0][2], u[1][0], u[0][0], u[1][2]);
                u[2][2] = conj_cross(u[0][0], u[1][1], u[0][1], u[1][0]);
            } else {
#pragma unroll
                for (int b = 0; b < 3; b++) u[2][b] = e[6 + b];
            }
        }
    }

    // Write the stored elements of one link given in full (row-major, nine
    // complex, FP64).
    __device__ static __forceinline__ void store(void *base, uint32_t vh, int mu, uint32_t cb,
                                                 const double2 *full)
    {
        double2 e[9];
        if constexpr (RECON == 8) {
            e[0] = full[1];
            e[1] = full[2];
            e[2] = full[3];
            e[3] = make_double2(atan2(full[0].y, full[0].x), atan2(full[6].y, full[6].x));
        } else {
            for (int k = 0; k < NE; k++) e[k] = full[k];
        }
        char *b = (char *)base;
        const uint32_t o16 = cb * 16u;
        if constexpr (P == TM_FP64) {
            for (int k = 0; k < NE; k++)
                *at_w<double2>((void *)row16(b, vh, mu, k, NE), o16) = e[k];
        } else if constexpr (P == TM_FP32) {
            for (int k = 0; k < NR32; k++)
                *at_w<float4>((void *)row16(b, vh, mu, k, NR32), o16) =
                    make_float4((float)e[2 * k].x, (float)e[2 * k].y, (float)e[2 * k + 1].x, (float)e[2 * k + 1].y);
            if constexpr (NE % 2 == 1)
                *at_w<float2>((void *)tail(b, vh, mu, NR32, 8), cb * 8u) =
                    make_float2((float)e[NE - 1].x, (float)e[NE - 1].y);
        } else {
            auto c2h = [](double2 v) {
                return (uint32_t)f_to_half<P>((float)v.x) | ((uint32_t)f_to_half<P>((float)v.y) << 16);
            };
            // 16-bit fixed-point phases: a float16 / bfloat16 angle near pi
            // would carry an error of up to 2e-3 / 8e-3 rad
            auto ph = [](double2 v) {
                auto q = [](double t) { return (uint32_t)(uint16_t)(int16_t)__double2int_rn(t / kPhaseStepD); };
                return q(v.x) | (q(v.y) << 16);
            };
            for (int k = 0; k < NR16; k++)
                *at_w<uint4>((void *)row16(b, vh, mu, k, NR16), o16) =
                    make_uint4(c2h(e[4 * k]), c2h(e[4 * k + 1]), c2h(e[4 * k + 2]),
                               RECON == 8 ? ph(e[3]) : c2h(e[4 * k + 3]));
            if constexpr (T16 == 2)
                *at_w<uint2>((void *)tail(b, vh, mu, NR16, 8), cb * 8u) =
                    make_uint2(c2h(e[4 * NR16]), c2h(e[4 * NR16 + 1]));
            else if constexpr (T16 == 1)
                *at_w<uint32_t>((void *)tail(b, vh, mu, NR16, 4), cb * 4u) = c2h(e[4 * NR16]);
        }
    }
};

// ------------------------------------------------------------------ twist
//
// R v = v + i ta g5 t3 v + b t1 v;  R^-1 v = c (v - i ta g5 t3 v - b t1 v),
// c = 1 / (1 + ta^2 - b^2).  ta carries the flavour sign (one flavour) and the
// dagger sign.  g5 swaps the upper (k < 6) and lower (k >= 6) spin pairs.
struct Twist {
    double ta, b, c;
};

template <typename T, int NF>
__device__ __forceinline__ void apply_twist(cx<T> (&v)[NF][12], const Twist &tw, bool inverse)
{
    const T ta = (T)tw.ta, b = (T)tw.b;
    const T s = inverse ? (T)-1 : (T)1;
    const T c = inverse ? (T)tw.c : (T)1;
    cx<T> o[NF][12];
#pragma unroll
    for (int f = 0; f < NF; f++) {
        const T t3 = (f == 0) ? ta : -ta;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const int kk = (k < 6) ? k + 6 : k - 6;
            cx<T> r = v[f][k] + (s * t3) * times_i(v[f][kk]);
            if constexpr (NF == 2) r = r + (s * b) * v[1 - f][k];
            o[f][k] = c * r;
        }
    }
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
        for (int k = 0; k < 12; k++) v[f][k] = o[f][k];
}

// ------------------------------------------------------------------ clover
//
// Twisted clover (the future work of Sec. 4): R(x) = A(x) + i a g5 t3 + b t1.
// A commutes with g5, so in the chiral basis (g5 = diag(1, 1, -1, -1)) it is
// two Hermitian 6x6 blocks A_+, A_- on (spin pair, colour).  Per block the
// doublet twist is [[A + i a chi, b], [b, A - i a chi]] in flavour space, whose
// inverse is B [[A - i a chi, -b], [-b, A + i a chi]] with the Hermitian
// B = (A^2 + a^2 - b^2)^-1 (A commutes with the scalars).  Stored per site:
// A_+, A_-, B_+, B_-, each as 36 reals (6 real diagonal entries, then the 15
// upper off-diagonal entries (i < j, row-major) as re, im), in 16-byte chunk
// rows [block][chunk][cb] (FP64: 18 chunks per block, FP32: 9).
// The internal basis maps to the chiral one by psi_+ = (psi_0,1 + psi_2,3),
// psi_- = (psi_0,1 - psi_2,3) (times 1/sqrt 2, applied as 1/2 on the way back).

__host__ __device__ inline size_t clover_parity_bytes(int prec, long vh)
{
    return (size_t)4 * 36 * (prec == TM_FP64 ? 8 : 4) * vh;
}

template <int P>
struct CloverIO {
    using real = typename Prec<P>::real;
    static constexpr int NCH = (P == TM_FP64) ? 18 : 9;   // 16-byte chunks per block

    __device__ static __forceinline__ void load(real (&d)[36], const void *base, uint32_t vh, int blk,
                                                uint32_t cb)
    {
        const uint32_t o16 = cb * 16u;
        if constexpr (P == TM_FP64) {
#pragma unroll
            for (int k = 0; k < NCH; k++) {
                const double2 c = *at<double2>((const char *)base + ((size_t)blk * NCH + k) * vh * 16, o16);
                d[2 * k] = c.x;
                d[2 * k + 1] = c.y;
            }
        } else {
#pragma unroll
            for (int k = 0; k < NCH; k++) {
                const float4 c = *at<float4>((const char *)base + ((size_t)blk * NCH + k) * vh * 16, o16);
                d[4 * k] = c.x;
                d[4 * k + 1] = c.y;
                d[4 * k + 2] = c.z;
                d[4 * k + 3] = c.w;
            }
        }
    }

    __device__ static __forceinline__ void store(void *base, uint32_t vh, int blk, uint32_t cb,
                                                 const double (&d)[36])
    {
        const uint32_t o16 = cb * 16u;
        for (int k = 0; k < NCH; k++) {
            char *row = (char *)base + ((size_t)blk * NCH + k) * vh * 16;
            if constexpr (P == TM_FP64)
                *at_w<double2>(row, o16) = make_double2(d[2 * k], d[2 * k + 1]);
            else
                *at_w<float4>(row, o16) = make_float4((float)d[4 * k], (float)d[4 * k + 1],
                                                      (float)d[4 * k + 2], (float)d[4 * k + 3]);
        }
    }
};

// w = H v for a packed Hermitian 6x6 H
template <typename T>
__device__ __forceinline__ void herm6_mv(cx<T> (&w)[6], const T (&h)[36], const cx<T> (&v)[6])
{
#pragma unroll
    for (int i = 0; i < 6; i++) w[i] = h[i] * v[i];
    int o = 6;
#pragma unroll
    for (int i = 0; i < 6; i++)
#pragma unroll
        for (int j = i + 1; j < 6; j++) {
            const cx<T> e = mk(h[o], h[o + 1]);
            o += 2;
            w[i] = w[i] + cmul(e, v[j]);
            w[j] = w[j] + cjmul(e, v[i]);
        }
}

// w_chi <- R w_chi or R^-1 w_chi on one chiral block (all flavours)
template <int P, int NF>
__device__ __forceinline__ void clover_block(cx<typename Prec<P>::real> (&w)[NF][6], const void *clov,
                                             uint32_t vh, uint32_t cb, int chi, const Twist &tw,
                                             bool inverse)
{
    using T = typename Prec<P>::real;
    const T s = inverse ? (T)-1 : (T)1;
    const T sg = chi == 0 ? (T)1 : (T)-1;                // g5 on this block
    const T b = (T)tw.b;
    T h[36];
    CloverIO<P>::load(h, clov, vh, chi, cb);
    cx<T> u[NF][6];
#pragma unroll
    for (int f = 0; f < NF; f++) {
        herm6_mv(u[f], h, w[f]);
        const T t3 = (f == 0 ? (T)tw.ta : (T)-tw.ta) * sg * s;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            u[f][k] = u[f][k] + t3 * times_i(w[f][k]);
            if constexpr (NF == 2) u[f][k] = u[f][k] + (s * b) * w[1 - f][k];
        }
    }
    if (inverse) {
        CloverIO<P>::load(h, clov, vh, 2 + chi, cb);
#pragma unroll
        for (int f = 0; f < NF; f++) herm6_mv(w[f], h, u[f]);
    } else {
#pragma unroll
        for (int f = 0; f < NF; f++)
#pragma unroll
            for (int k = 0; k < 6; k++) w[f][k] = u[f][k];
    }
}

// v <- R v or R^-1 v (R^+ / R^-+ through the sign of tw.ta) with the clover
// term of this site.
template <int P, int NF>
__device__ __forceinline__ void apply_clover(cx<typename Prec<P>::real> (&v)[NF][12], const void *clov,
                                             uint32_t vh, uint32_t cb, const Twist &tw, bool inverse)
{
    using T = typename Prec<P>::real;
    cx<T> wp[NF][6], wm[NF][6];
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
        for (int k = 0; k < 6; k++) {
            wp[f][k] = v[f][k] + v[f][k + 6];
            wm[f][k] = v[f][k] - v[f][k + 6];
        }
    clover_block<P, NF>(wp, clov, vh, cb, 0, tw, inverse);
    clover_block<P, NF>(wm, clov, vh, cb, 1, tw, inverse);
    // back to the internal basis, the two 1/sqrt 2 factors as one 1/2
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
        for (int k = 0; k < 6; k++) {
            v[f][k] = (T)0.5 * (wp[f][k] + wm[f][k]);
            v[f][k + 6] = (T)0.5 * (wp[f][k] - wm[f][k]);
        }
}

// ------------------------------------------------------------------ reductions

// CG scalars per right-hand side, device resident.
constexpr int kHistory = 16;   // iterated residuals kept per rhs (ring)
struct CGScalars {
    double rr;       // |r|^2 of the iterated residual
    double rr_old;
    double pap;      // |M p|^2 = <p, M^+ M p>
    double alpha;
    double beta;
    double stop2;    // stop when rr <= stop2
    double maxrr;    // largest rr since the last residual replacement
    double rr_upd;   // true |r|^2 at the last residual replacement (0: none yet)
    double stall_f2; // squared stall factor: a replacement whose true |r|^2 is
                     // not below stall_f2 * rr_upd made no progress
    double hist[kHistory];   // |r|^2 of the last iterations, hist[i % kHistory]
    int niter;       // iterations this rhs was active in
    int stall;       // consecutive replacements without progress
    int active;      // 0 once converged (updates become no-ops)
    int pending;     // converged in the iterated residual, not yet verified
};

enum FinOp { FIN_NONE = 0, FIN_STORE = 1, FIN_ALPHA = 2, FIN_BETA = 3, FIN_STORE_RR = 4, FIN_RELIABLE = 5 };

// Two-stage deterministic reduction: every block of the producing kernel
// stores its partial sum per vector; a separate one-block finish kernel adds
// the partials in a fixed order and applies the finishing operation.  (No
// atomics and no device-scope fences in the producing kernel: on a multi-XCD
// part each such fence writes back the XCD's L2.)
struct Reduce {
    double *partials;      // [nvec][nblk]
    double *out;           // FIN_STORE destination [nvec]
    CGScalars *cg;         // FIN_ALPHA / FIN_BETA state [nvec]
    int op;
    int nvec;              // filled for the finish kernel
    int nblk;
};

struct FinishBatch {
    int nprob;
    const int *gate;       // nullable: skip the launch when *gate == 0
    Reduce r[kMaxProblems];
};

// Device-side decision whether the next reliable update runs (mixed CG with
// captured iterations): any active rhs whose rr fell below delta^2 maxrr, or
// any rhs whose iterated residual converged and awaits verification.
struct DecideArgs {
    int nprob;
    int nrhs[kMaxProblems];
    CGScalars *cg[kMaxProblems];
    double delta2;
    int *gate;
    int *count;            // number of updates decided (for reporting)
};

// Device-side run flag of a CG iteration: set when some rhs is still active
// (or, with reliable updates, awaits its verifying update); every launch of
// the iteration is gated by it, so iterations enqueued past convergence (the
// rest of a captured graph, the rest of a host check period) do nothing.
// iters counts the iterations that ran; once it reaches maxiter the flag
// stays clear, so a check period never runs past the iteration limit.
struct RunArgs {
    int nprob;
    int nrhs[kMaxProblems];
    const CGScalars *cg[kMaxProblems];
    int with_pending;
    int maxiter;
    int *run;
    int *iters;
};

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the block; result valid in thread 0.  Deterministic order.
template <int BS>
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < BS / 64; i++) s += sh[i];
    }
    __syncthreads();
    return s;
}

// ------------------------------------------------------------------ hop descriptors

struct HopProblem {
    int X[4];            // Lx, Ly, Lz, Lt
    int vh;              // sites per parity
    int nrhs;
    int blk_start;       // first logical block of this problem
    int nsb;             // site blocks
    int ngrp;            // rhs groups
    int out_parity;
    int zc;              // z-planes per brick of the processing order (0: lexicographic)
    int ts;              // time slices per slab of the processing order (zc > 0)
    double tsign;        // factor on hops across the t boundary
    Twist tw;            // twist (dagger sign folded in)
    double k;            // epilogue coefficient
    const void *gauge[2];   // links of parity 0 / 1
    const void *clov;       // clover blocks of the output parity (twisted clover)
    SpinorPtr in, out, x;
    // nullable: CG residual update in the epilogue, out = out - alpha A with
    // A the epilogue's result and alpha of each rhs read from here
    const CGScalars *upd;
    Reduce red;
};

struct HopBatch {
    int nprob;
    int total_blocks;
    const int *gate;     // nullable: skip the launch when *gate == 0
    int epi;             // tm_epilogue
    int xcd_remap;       // 1: give every XCD a contiguous range of blocks
    int nt_streams;      // kNtOut | kNtX | kNtTime: streams accessed non-temporally
    HopProblem p[kMaxProblems];
};

// Map hardware workgroup id to a logical block so that each of the 8 XCDs
// (which receive workgroups round-robin) gets one contiguous range.
__device__ __forceinline__ int xcd_logical_block(int i, int g)
{
    const int q = g >> 3, r = g & 7;
    const int k = i & 7, j = i >> 3;
    return k * q + (k < r ? k : r) + j;
}

}  // namespace twm

// Error reporting and the matrix-core policies of the mode products (FP64/FP32
// MFMA and split BF16), with the vector and LDS helpers they use.
//
// Part of libetdds: included, in order, by library.hpp (each translation
// unit that includes it holds its own copy); internal linkage throughout.
#pragma once

namespace {

etd_status fail(etd_status s, const std::string& m) {
    g_err = m;
    return s;
}

etd_status hip_fail(hipError_t e, const char* where) {
    g_err = std::string(where) + ": " + hipGetErrorString(e);
    return ETD_EHIP;
}

#define HIP_TRY(expr, where)                     \
    do {                                         \
        hipError_t e_ = (expr);                  \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Vec4;
template <>
struct Vec4<double> {
    typedef f64x4 type;
};
template <>
struct Vec4<float> {
    typedef f32x4 type;
};

// Row, within a 16x16 result tile, of accumulator register e in lane group
// g = lane/16 (the column is lane%16).  The FP64 16x16x4 MFMA interleaves the
// four lane groups (row g + 4e); the FP32 one stacks them (row 4g + e).  The A
// and B operand layouts are the same for both: A[i][k] in lane i + 16k,
// B[k][j] in lane j + 16k.
template <typename T>
__device__ __forceinline__ int acc_row(int g, int e);
template <>
__device__ __forceinline__ int acc_row<double>(int g, int e) { return g + 4 * e; }
template <>
__device__ __forceinline__ int acc_row<float>(int g, int e) { return 4 * g + e; }

__device__ __forceinline__ f64x4 mfma4(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T, int N>
using vec_t = T __attribute__((ext_vector_type(N)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// KL contiguous elements from LDS, read in 16-byte pieces.
template <typename T, int KL>
__device__ __forceinline__ vec_t<T, KL> lds_vec(const T* p) {
    constexpr int PER = 16 / int(sizeof(T));
    vec_t<T, KL> v;
#pragma unroll
    for (int i = 0; i < KL / PER; ++i) {
        const vec_t<T, PER> w = *reinterpret_cast<const vec_t<T, PER>*>(p + i * PER);
#pragma unroll
        for (int j = 0; j < PER; ++j) v[i * PER + j] = w[j];
    }
    return v;
}

// How one 16x16 block of a mode product is computed.  A K block of KB
// contracted indices is consumed in NSUB matrix-core steps; lane (i, g) of the
// A operand holds P[row i][k0 .. k0+KL), k0 = KB*kb + KL*g, and lane (j, g) of
// the B operand the same k range of column j.  row(g, e) gives the tile row of
// accumulator register e in lane group g.
//
// Native: FP64 or FP32 16x16x4 MFMA, K block 16, four steps of 4.
//
// elem is the type of the state (fields, LDS tiles, diagonals, epilogues) and
// acc the type the matrix cores accumulate in.
template <typename T>
struct NativeMma {
    typedef T elem;
    typedef T acc;
    static constexpr int KB = 16, KL = 4, NSUB = 4;
    static constexpr bool SPLIT_B = false;
    typedef vec_t<T, 4> A;
    typedef vec_t<T, 4> B;
    // row-major P: lane (i, g) of row block rb reads P[16 rb + i][KL g ..]
    __device__ static long a_off(int NP, int rb, int li, int lg) { return long(16 * rb + li) * NP + KL * lg; }
    __device__ static long a_kstep(int) { return KB; }
    __device__ static A load_a(const void* P, int, long off) {
        return *reinterpret_cast<const A*>(static_cast<const T*>(P) + off);
    }
    __device__ static B prep(const vec_t<T, 4>& b) { return b; }
    __device__ static void step(vec_t<T, 4>& acc, const A& a, const B& b, int e) { acc = mfma4(a[e], b[e], acc); }
    __device__ static int row(int g, int e) { return acc_row<T>(g, e); }
};

// FP64 state with FP32 products: the fields, the tiles in LDS, the
// diagonals and every epilogue stay FP64; P is held in FP32 and each B
// fragment is rounded to FP32 as it is read, for the FP32 16x16x4 MFMA with
// FP32 accumulation.  The increment form keeps the rounded quantity a
// correction to the FP64 state.
struct F64F32Mma {
    typedef double elem;
    typedef float acc;
    static constexpr int KB = 16, KL = 4, NSUB = 4;
    static constexpr bool SPLIT_B = false;
    typedef vec_t<float, 4> A;
    typedef vec_t<float, 4> B;
    __device__ static long a_off(int NP, int rb, int li, int lg) { return long(16 * rb + li) * NP + KL * lg; }
    __device__ static long a_kstep(int) { return KB; }
    __device__ static A load_a(const void* P, int, long off) {
        return *reinterpret_cast<const A*>(static_cast<const float*>(P) + off);
    }
    __device__ static B prep(const vec_t<double, 4>& b) { return __builtin_convertvector(b, B); }
    __device__ static void step(vec_t<float, 4>& acc, const A& a, const B& b, int e) { acc = mfma4(a[e], b[e], acc); }
    __device__ static int row(int g, int e) { return acc_row<float>(g, e); }
};

// Split BF16: both operands are written x = hi + mid + lo with bfloat16
// pieces (hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid), each
// subtraction exact in FP32); the product keeps the six terms whose weight is
// at least 2^-16 of hi*hi (lo*hi, mid*mid, hi*lo, mid*hi, hi*mid, hi*hi, the
// small ones first) on the BF16 16x16x32 MFMA with FP32 accumulation.  P's
// pieces are split once on the host and stored in fragment order: for row
// block rb and K block kb, one contiguous chunk of three planes (hi, mid, lo)
// x 64 lanes x 8 values, lane i + 16 g holding P[16 rb + i][32 kb + 8 g ..
// +8], so each plane of a fragment is one fully used 1 KB run (row-major
// planes would touch sixteen half-used lines per load).  The data's pieces
// are split on the fly (an FP64 state is rounded to FP32 first).
template <typename S>
struct Bf16x6MmaOn {
    typedef S elem;
    typedef float acc;
    static constexpr int KB = 32, KL = 8, NSUB = 6;
    static constexpr bool SPLIT_B = true;
    struct A {
        bf16x8 p[3];   // hi, mid, lo
    };
    typedef A B;
    static constexpr int CHUNK = 3 * 64 * 8;   // bf16 values per (row block, K block)
    __device__ static long a_off(int NP, int rb, int li, int lg) {
        return long(rb) * (NP / KB) * CHUNK + 8 * (li + 16 * lg);
    }
    __device__ static long a_kstep(int) { return CHUNK; }
    __device__ static A load_a(const void* P, int, long off) {
        const __bf16* q = static_cast<const __bf16*>(P) + off;
        A a;
        a.p[0] = *reinterpret_cast<const bf16x8*>(q);
        a.p[1] = *reinterpret_cast<const bf16x8*>(q + 512);
        a.p[2] = *reinterpret_cast<const bf16x8*>(q + 1024);
        return a;
    }
    // Pairs of elements go through two-wide conversions, so that each packed
    // round-to-nearest conversion serves two values and lands in place.
    __device__ static B prep(const vec_t<S, 8>& xs) {
        const vec_t<float, 8> x = __builtin_convertvector(xs, vec_t<float, 8>);
        typedef float f2 __attribute__((ext_vector_type(2)));
        typedef __bf16 b2 __attribute__((ext_vector_type(2)));
        B b;
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
            const f2 v = {x[e], x[e + 1]};
            const b2 h = __builtin_convertvector(v, b2);
            const f2 r1 = v - __builtin_convertvector(h, f2);
            const b2 m = __builtin_convertvector(r1, b2);
            const b2 l = __builtin_convertvector(r1 - __builtin_convertvector(m, f2), b2);
            b.p[0][e] = h[0];
            b.p[0][e + 1] = h[1];
            b.p[1][e] = m[0];
            b.p[1][e + 1] = m[1];
            b.p[2][e] = l[0];
            b.p[2][e + 1] = l[1];
        }
        return b;
    }
    __device__ static void step(f32x4& acc, const A& a, const B& b, int t) {
        switch (t) {
        case 0: acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[2], b.p[0], acc, 0, 0, 0); break;
        case 1: acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[1], b.p[1], acc, 0, 0, 0); break;
        case 2: acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[0], b.p[2], acc, 0, 0, 0); break;
        case 3: acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[1], b.p[0], acc, 0, 0, 0); break;
        case 4: acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[0], b.p[1], acc, 0, 0, 0); break;
        default: acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[0], b.p[0], acc, 0, 0, 0); break;
        }
    }
    __device__ static int row(int g, int e) { return 4 * g + e; }
};
typedef Bf16x6MmaOn<float> Bf16x6Mma;

}  // namespace

// Spectral ETD2RK-DS stepper for gfx950: stage kernels and the C ABI.
//
// One step of the Pade-based scheme (Sec. 3.1; Algorithms 1-2), written in the
// increment form Q(z) g = Q(0) g + P diag(Q(tau lambda) - Q(0)) P g, with P
// the symmetric orthogonal eigenvector matrix of the direction (so the forward
// product P^T and the backward product P are the same matrix):
//
//   outer stage(s)  (3-D: z then y; 2-D: y)
//       w_a = g_a + P diag(q1 - 1) P g_a      for g = [U, f(t_n, U)] (first)
//                                              or g = [w1, w2]       (middle)
//   x stage (fused, Algorithm 2 steps 3.5.1-3.5.7)
//       c   = (q1 - 1) .* (P w3) + tau (q2 - 1) .* (P w4)
//       W   = w3 + tau w4 + P c
//       d   = f(t_{n+1}, W) - w4
//       U+  = W + tau d / 2 + tau P ((q3 - 1/2) .* (P d))
//
// which is Q1 w3 + tau Q2 w4 and W + tau Q3 (F1 - w4) rearranged.  Every
// product is a dense mode-d contraction with P and runs on the MFMA units
// (FP64 or FP32 16x16x4).  A workgroup owns a tile of 16 grid lines (x stage)
// or 16 columns (outer stages) over the whole contracted direction, so the
// forward product, the Hadamard scaling and the backward product stay on chip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "etdds.h"
#include "plan.hpp"

using namespace etdds;

// Optional per-stage timing: HIP events recorded on the caller's stream
// around every stage launch (diagnostics; not thread-safe).
struct StageTimer {
    bool on = false;
    std::vector<hipEvent_t> pool;    // reusable events
    size_t used = 0;                 // events recorded since the last read
    std::vector<int> kind;           // stage kind of interval i = (ev[2i], ev[2i+1])
};

struct etd_plan {
    Plan p;
    mutable StageTimer timer;
};

namespace {

thread_local std::string g_err;

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
template <typename T>
struct NativeMma {
    typedef T elem;
    static constexpr int KB = 16, KL = 4, NSUB = 4;
    static constexpr bool SPLIT_B = false;
    typedef vec_t<T, 4> A;
    typedef vec_t<T, 4> B;
    __device__ static A load_a(const void* P, int, long off) {
        return *reinterpret_cast<const A*>(static_cast<const T*>(P) + off);
    }
    __device__ static B prep(const vec_t<T, 4>& b) { return b; }
    __device__ static void step(vec_t<T, 4>& acc, const A& a, const B& b, int e) { acc = mfma4(a[e], b[e], acc); }
    __device__ static int row(int g, int e) { return acc_row<T>(g, e); }
};

// Split BF16: both operands are written x = hi + mid + lo with bfloat16
// pieces (hi = bf16(x), mid = bf16(x - hi), lo = bf16(x - hi - mid), each
// subtraction exact in FP32); the product keeps the six terms whose weight is
// at least 2^-16 of hi*hi (lo*hi, mid*mid, hi*lo, mid*hi, hi*mid, hi*hi, the
// small ones first) on the BF16 16x16x32 MFMA with FP32 accumulation.  P's
// pieces are split once on the host (three planes of NP*NP); the data's are
// split on the fly.
struct Bf16x6Mma {
    typedef float elem;
    static constexpr int KB = 32, KL = 8, NSUB = 6;
    static constexpr bool SPLIT_B = true;
    struct A {
        bf16x8 p[3];   // hi, mid, lo
    };
    typedef A B;
    __device__ static A load_a(const void* P, int NP, long off) {
        const __bf16* q = static_cast<const __bf16*>(P) + off;
        const long plane = long(NP) * NP;
        A a;
        a.p[0] = *reinterpret_cast<const bf16x8*>(q);
        a.p[1] = *reinterpret_cast<const bf16x8*>(q + plane);
        a.p[2] = *reinterpret_cast<const bf16x8*>(q + 2 * plane);
        return a;
    }
    // Pairs of elements go through two-wide conversions, so that each packed
    // round-to-nearest conversion serves two values and lands in place.
    __device__ static B prep(const vec_t<float, 8>& x) {
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

// ---------------------------------------------------------------------------
// Reactions (pointwise source terms of the examples and workloads)
// ---------------------------------------------------------------------------

struct RxnArgs {
    int kind;
    double p[4];
    double ac_rate;        // -lam + kappa * sum_d mu_d + q (AC_MMS)
    double ac_mu;          // sum_d mu_d, d psi / d kappa per unit ue (AC_MMS)
    double exp_lt;         // e^{-lam t} at the stage's time (AC_MMS)
    const double* sines;   // [3][kMaxPadded] sin(pi (x_i - lo)/L), 0 on the padding
    double tau;            // the instance's time step (grouped launches form t from it)
};

// Exact solution and psi of the manufactured Allen-Cahn problem at node
// (x, y, z).  psi depends on kappa and q through ac_rate: d psi / d kappa =
// ac_mu ue, d psi / d q = ue.
__device__ __forceinline__ double ac_ue(const RxnArgs& r, int x, int y, int z) {
    return r.exp_lt * r.sines[x] * r.sines[kMaxPadded + y] * r.sines[2 * kMaxPadded + z];
}

__device__ __forceinline__ double ac_psi(const RxnArgs& r, int x, int y, int z) {
    const double ue = ac_ue(r, x, y, z);
    return r.ac_rate * ue - ue * (1.0 - ue * ue);
}

template <typename T>
__device__ __forceinline__ T react1(const RxnArgs& r, T u, int x, int y, int z) {
    switch (r.kind) {
    case ETD_RXN_LINEAR: return T(r.p[0]) * u;
    case ETD_RXN_FISHER: return T(r.p[0]) * u * (T(1) - u);
    case ETD_RXN_ALLEN_CAHN: return u - u * u * u;
    case ETD_RXN_AC_MMS: return u * (T(1) - u * u) + T(ac_psi(r, x, y, z));
    case ETD_RXN_SATURATING: return T(r.p[0]) * u / (T(1) - u);
    default: return T(0);
    }
}

template <typename T>
__device__ __forceinline__ void react2(const RxnArgs& r, T u, T v, T& fu, T& fv) {
    if (r.kind == ETD_RXN_FHN_CUBIC) {
        fu = u * (T(1) - u) * (u - T(r.p[0])) - v;
        fv = T(r.p[1]) * (u - T(r.p[2]) * v);
    } else {
        fu = u - u * u * u / T(3) - v;
        fv = T(r.p[0]) * (u - T(r.p[1]) * v);
    }
}

// Reaction on NC components at one node: f[c] from u[c].
template <typename T, int NC>
__device__ __forceinline__ void react(const RxnArgs& r, const T* u, T* f, int x, int y, int z) {
    if constexpr (NC == 1) {
        f[0] = react1<T>(r, u[0], x, y, z);
    } else {
        react2<T>(r, u[0], u[1], f[0], f[1]);
    }
}

// J(u)^T g: the transposed pointwise Jacobian of the reaction applied to g
// (the adjoint of a perturbation of u; the forcing of AC_MMS does not depend
// on u).
template <typename T, int NC>
__device__ __forceinline__ void react_jt(const RxnArgs& r, const T* u, const T* g, T* out) {
    if constexpr (NC == 1) {
        T d;
        switch (r.kind) {
        case ETD_RXN_LINEAR: d = T(r.p[0]); break;
        case ETD_RXN_FISHER: d = T(r.p[0]) * (T(1) - T(2) * u[0]); break;
        case ETD_RXN_ALLEN_CAHN:
        case ETD_RXN_AC_MMS: d = T(1) - T(3) * u[0] * u[0]; break;
        case ETD_RXN_SATURATING: {
            const T om = T(1) - u[0];
            d = T(r.p[0]) / (om * om);
            break;
        }
        default: d = T(0);
        }
        out[0] = d * g[0];
    } else {
        T fu_u, fu_v, fv_u, fv_v;
        if (r.kind == ETD_RXN_FHN_CUBIC) {
            // fu = u(1-u)(u-a) - v, fv = eps (u - gam v)
            fu_u = (T(-3) * u[0] + T(2) * (T(1) + T(r.p[0]))) * u[0] - T(r.p[0]);
            fu_v = T(-1);
            fv_u = T(r.p[1]);
            fv_v = -T(r.p[1]) * T(r.p[2]);
        } else {
            // fu = u - u^3/3 - v, fv = eps (u - alpha v)
            fu_u = T(1) - u[0] * u[0];
            fu_v = T(-1);
            fv_u = T(r.p[0]);
            fv_v = -T(r.p[0]) * T(r.p[1]);
        }
        out[0] = fu_u * g[0] + fv_u * g[1];
        out[1] = fu_v * g[0] + fv_v * g[1];
    }
}

// ---------------------------------------------------------------------------
// Shared pieces of the stage kernels
// ---------------------------------------------------------------------------

// acc[r][q] += P[16(rb0+r) .. +16][:] . B_q over the whole contracted length
// NP (a multiple of M::KB).  The A operand comes straight from the row-major P
// in global memory (L2-resident; each lane reads its KL contiguous entries)
// and is double-buffered in registers one K block ahead; bload(q, k0) returns
// the KL values of B fragment q for contracted indices k0 .. k0+KL of this
// lane's column.
template <typename M, int RB, int NQ, typename BL>
__device__ __forceinline__ void gemm(const void* __restrict__ P, int NP, int rb0, int li, int lg,
                                     vec_t<typename M::elem, 4> (&acc)[RB][NQ], BL bload) {
    const int nkb = NP / M::KB;
    long off[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) off[r] = long(16 * (rb0 + r) + li) * NP + M::KL * lg;
    typename M::A a_cur[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) a_cur[r] = M::load_a(P, NP, off[r]);
    for (int kb = 0; kb < nkb; ++kb) {
        const int kn = min(kb + 1, nkb - 1) * M::KB;
        typename M::A a_nxt[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) a_nxt[r] = M::load_a(P, NP, off[r] + kn);
        if constexpr (M::SPLIT_B) {
            // split B fragments one at a time (each expands to three pieces)
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const typename M::B b = M::prep(bload(q, kb * M::KB + M::KL * lg));
#pragma unroll
                for (int t = 0; t < M::NSUB; ++t)
#pragma unroll
                    for (int r = 0; r < RB; ++r) M::step(acc[r][q], a_cur[r], b, t);
            }
        } else {
            typename M::B b[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) b[q] = M::prep(bload(q, kb * M::KB + M::KL * lg));
#pragma unroll
            for (int t = 0; t < M::NSUB; ++t)
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int q = 0; q < NQ; ++q) M::step(acc[r][q], a_cur[r], b[q], t);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) a_cur[r] = a_nxt[r];
    }
}

template <typename T, int RB, int NQ>
__device__ __forceinline__ void zero(typename Vec4<T>::type (&acc)[RB][NQ]) {
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[r][q] = typename Vec4<T>::type{0, 0, 0, 0};
}

// 16-byte vector of T
template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
    typedef double __attribute__((ext_vector_type(2))) type;
    static constexpr int n = 2;
};
template <>
struct Vec16<float> {
    typedef float __attribute__((ext_vector_type(4))) type;
    static constexpr int n = 4;
};

// ---------------------------------------------------------------------------
// Outer-mode stage: contraction along a strided direction (z, or y)
// ---------------------------------------------------------------------------

struct OuterArgs {
    const void* in0;     // first: U; middle: w1
    const void* in1;     // middle: w2
    void* out0;          // Q1 applied to in0
    void* out1;          // Q1 applied to f(in0) (first) or in1 (middle)
    const void* P;       // NP x NP row-major
    const void* diag;    // q1 - 1 of this direction, component 0
    long diag_cstride;   // elements between components' diagonals
    int NP;              // padded length of the contracted direction
    int ncb;             // 16-column blocks per batch
    long sk;             // element stride of the contracted index
    long sb;             // batch stride
    long sc;             // component stride
    int npx, npy;        // padded x and y extents (node decoding)
    int dim;
    RxnArgs rxn;
    const void* other;   // split systems: the other component's field (first stage), else null
    int comp;            // split systems: the component this launch handles
};

// Reaction of component `comp` of a two-component system at one node, the
// other component being read from `other` (split processing).
template <typename T>
__device__ __forceinline__ T react_coupled(const RxnArgs& r, int comp, T mine, T theirs) {
    T fu, fv;
    if (comp == 0) react2<T>(r, mine, theirs, fu, fv);
    else react2<T>(r, theirs, mine, fu, fv);
    return comp == 0 ? fu : fv;
}

// Workgroup: NP/(16 RB) waves over one tile of 16*CB columns; wave w owns
// output row blocks RB*w .. RB*w+RB-1 for all CB column blocks (each P
// fragment feeds 2*NC*CB MFMAs).  LDS: [2*NC arrays][16*CB columns][NP + pad]
// of T (the contracted index contiguous, so a lane's B fragment is one
// vector read), first the inputs (and f of them), then the scaled spectral
// coefficients.
// One thread's share of an outer tile's global inputs: ITER 16-byte vectors
// of each loaded array (the workgroup has exactly 4 NP / RB threads).
template <typename M, int NC, bool FIRST, int RB, int CB>
struct OuterRegs {
    typedef typename Vec16<typename M::elem>::type TV;
    static constexpr int ITER = 4 * RB * CB / Vec16<typename M::elem>::n;
    static constexpr int NLOAD = FIRST ? NC : 2 * NC;
    TV v[ITER][NLOAD];
    TV other[(FIRST && NC == 1) ? ITER : 1];
};

template <typename M, int NC, bool FIRST, int RB, int CB>
__device__ __forceinline__ void outer_load(const OuterArgs& a, long tile, OuterRegs<M, NC, FIRST, RB, CB>& g) {
    typedef typename M::elem T;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    constexpr int NCOL = 16 * CB;
    constexpr int VPR = NCOL / VN;
    const int nvec = a.NP * VPR;
    const long gbase = (tile / a.ncb) * a.sb + long(tile % a.ncb) * NCOL;
    const T* __restrict__ in0 = static_cast<const T*>(a.in0);
    const T* __restrict__ in1 = static_cast<const T*>(a.in1);
#pragma unroll
    for (int i = 0; i < OuterRegs<M, NC, FIRST, RB, CB>::ITER; ++i) {
        const int v = threadIdx.x + i * blockDim.x;
        if (v >= nvec) break;
        const int k = v / VPR, j0 = (v - k * VPR) * VN;
        const long gi = gbase + long(k) * a.sk + j0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            g.v[i][c] = *reinterpret_cast<const TV*>(in0 + gi + c * a.sc);
            if constexpr (!FIRST) g.v[i][NC + c] = *reinterpret_cast<const TV*>(in1 + gi + c * a.sc);
        }
        if constexpr (FIRST && NC == 1)
            if (a.other) g.other[i] = *reinterpret_cast<const TV*>(static_cast<const T*>(a.other) + gi);
    }
}

// Registers -> LDS (and, in the first stage, f of them).  LDS: [2*NC
// arrays][16*CB columns][NP + pad], the contracted index contiguous.
template <typename M, int NC, bool FIRST, int RB, int CB>
__device__ __forceinline__ void outer_store(const OuterArgs& a, long tile, const OuterRegs<M, NC, FIRST, RB, CB>& g) {
    typedef typename M::elem T;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    constexpr int NCOL = 16 * CB;
    constexpr int VPR = NCOL / VN;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* X = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = NCOL * RS;
    const int nvec = NP * VPR;
    const int cb = int(tile % a.ncb);
#pragma unroll
    for (int i = 0; i < OuterRegs<M, NC, FIRST, RB, CB>::ITER; ++i) {
        const int v = threadIdx.x + i * blockDim.x;
        if (v >= nvec) break;
        const int k = v / VPR, j0 = (v - k * VPR) * VN;
        if constexpr (FIRST) {
            TV f[NC];
#pragma unroll
            for (int t = 0; t < VN; ++t) {
                int x, y, z;
                const int col = cb * NCOL + j0 + t;
                if (a.dim == 3) {
                    z = k;
                    y = col / a.npx;
                    x = col - y * a.npx;
                } else {
                    z = 0;
                    y = k;
                    x = col;
                }
                T uu[NC], ff[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) uu[c] = g.v[i][c][t];
                if constexpr (NC == 1) {
                    if (a.other) ff[0] = react_coupled<T>(a.rxn, a.comp, uu[0], g.other[i][t]);
                    else react<T, NC>(a.rxn, uu, ff, x, y, z);
                } else {
                    react<T, NC>(a.rxn, uu, ff, x, y, z);
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) f[c][t] = ff[c];
            }
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int t = 0; t < VN; ++t) {
                    X[c * AST + (j0 + t) * RS + k] = g.v[i][c][t];
                    X[(NC + c) * AST + (j0 + t) * RS + k] = f[c][t];
                }
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int t = 0; t < VN; ++t) {
                    X[c * AST + (j0 + t) * RS + k] = g.v[i][c][t];
                    X[(NC + c) * AST + (j0 + t) * RS + k] = g.v[i][NC + c][t];
                }
        }
    }
}

// Workgroup: NP/(16 RB) waves over one tile of 16*CB columns; wave w owns
// output row blocks RB*w .. RB*w+RB-1 for all CB column blocks (each P
// fragment feeds 2*NC*CB MFMAs).  Runs on a staged tile: the inputs (and f
// of them) in LDS, then the scaled spectral coefficients.
template <typename M, int NC, bool FIRST, int RB, int CB>
__device__ __forceinline__ void outer_compute(const OuterArgs& a, long tile) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    constexpr int NCOL = 16 * CB;         // columns per tile
    constexpr int NA = 2 * NC;
    constexpr int NQ = NA * CB;           // B fragments per K block
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* X = reinterpret_cast<T*>(smem_raw);

    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));     // LDS stride between columns
    const int AST = NCOL * RS;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const int cb = int(tile % a.ncb);
    const long bt = tile / a.ncb;
    const long gbase = bt * a.sb + long(cb) * NCOL;
    const void* __restrict__ P = a.P;

    const int rb0 = RB * w;
    // fragment qq = array (qq / CB), column block (qq % CB)
    auto bfrag = [&](int qq, int k0) {
        return lds_vec<T, M::KL>(X + (qq / CB) * AST + ((qq % CB) * 16 + li) * RS + k0);
    };
    // element (row of accumulator register e of block rb0+r, column li of block qq%CB) of array qq/CB
    auto at = [&](int qq, int r, int e) -> T& {
        return X[(qq / CB) * AST + ((qq % CB) * 16 + li) * RS + 16 * (rb0 + r) + M::row(lg, e)];
    };
    T4 acc[RB][NQ];
    T4 res[RB][NQ];
    zero<T, RB, NQ>(acc);

    // ---- forward product S = P g (all arrays share the A operand) ----
    gemm<M, RB, NQ>(P, NP, rb0, li, lg, acc, bfrag);
    // the inputs at this wave's output rows, for the increment-form epilogue
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int qq = 0; qq < NQ; ++qq)
#pragma unroll
            for (int e = 0; e < 4; ++e) res[r][qq][e] = at(qq, r, e);
    __syncthreads();

    // ---- Hadamard scaling by q1 - 1, coefficients back to LDS ----
    const T* __restrict__ dg = static_cast<const T*>(a.diag);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int qq = 0; qq < NQ; ++qq) {
            const T* dc = dg + ((qq / CB) % NC) * a.diag_cstride + 16 * (rb0 + r);
#pragma unroll
            for (int e = 0; e < 4; ++e) at(qq, r, e) = acc[r][qq][e] * dc[M::row(lg, e)];
        }
    zero<T, RB, NQ>(acc);
    __syncthreads();

    // ---- backward product P S and the increment-form epilogue ----
    gemm<M, RB, NQ>(P, NP, rb0, li, lg, acc, bfrag);
    T* __restrict__ out0 = static_cast<T*>(a.out0);
    T* __restrict__ out1 = static_cast<T*>(a.out1);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int qq = 0; qq < NQ; ++qq) {
            const int q = qq / CB;
            T* o = (q < NC ? out0 : out1) + (q % NC) * a.sc + gbase + (qq % CB) * 16 + li;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = 16 * (rb0 + r) + M::row(lg, e);
                o[long(row) * a.sk] = res[r][qq][e] + acc[r][qq][e];
            }
        }
}

// One tile, staged and computed.
template <typename M, int NC, bool FIRST, int RB, int CB>
__device__ __forceinline__ void outer_tile(const OuterArgs& a, long tile) {
    OuterRegs<M, NC, FIRST, RB, CB> g;
    outer_load<M, NC, FIRST, RB, CB>(a, tile, g);
    outer_store<M, NC, FIRST, RB, CB>(a, tile, g);
    __syncthreads();
    outer_compute<M, NC, FIRST, RB, CB>(a, tile);
}

template <typename M, int NC, bool FIRST, int RB, int CB, int MAXT>
__global__ __launch_bounds__(MAXT) void outer_stage(OuterArgs a) {
    outer_tile<M, NC, FIRST, RB, CB>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// x stage: contraction along the contiguous direction, both RK stages fused
// ---------------------------------------------------------------------------

struct XArgs {
    const void* w3;
    const void* w4;
    void* out;
    const void* P;
    const void* diag;     // slot X1 of component 0
    long diag_sstride;    // elements between slots X1, X2, X3
    long diag_cstride;    // elements between components
    int NP;
    long sc;              // component stride
    int npy;              // padded y extent (line -> (y, z))
    double tau;
    RxnArgs rxn;          // at t_{n+1}
    void* Wout;           // when set, W is also written there (the adjoint's replay)
};

// Workgroup: NP/(16 RB) waves over 16*CB consecutive x-lines.  Wave w owns
// the spectral/physical x rows of blocks RB*w .. RB*w+RB-1 of every product,
// for all CB line blocks.  LDS: [2*NC][16*CB lines][NP + pad]; arrays 0..NC-1
// hold w3, then c, then e; arrays NC..2NC-1 hold w4, then d.
// One thread's share of an x tile's inputs (w3 and w4 of every component):
// ITER 16-byte vectors of each (the workgroup has exactly 4 NP / RB threads).
template <typename M, int NC, int RB, int CB>
struct XRegs {
    static constexpr int ITER = 4 * RB * CB / Vec16<typename M::elem>::n;
    typename Vec16<typename M::elem>::type v[ITER][2 * NC];
};

// The tile's lines are one contiguous run of 16*CB*NP elements per array.
template <typename M, int NC, int RB, int CB>
__device__ __forceinline__ void x_load(const XArgs& a, long tile, XRegs<M, NC, RB, CB>& g) {
    typedef typename M::elem T;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    const int nvec = 16 * CB * a.NP / VN;
    const long base = tile * 16 * CB * long(a.NP);
    const T* __restrict__ w3 = static_cast<const T*>(a.w3);
    const T* __restrict__ w4 = static_cast<const T*>(a.w4);
#pragma unroll
    for (int i = 0; i < XRegs<M, NC, RB, CB>::ITER; ++i) {
        const int v = threadIdx.x + i * blockDim.x;
        if (v >= nvec) break;
        const long gi = base + long(v) * VN;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            g.v[i][c] = *reinterpret_cast<const TV*>(w3 + c * a.sc + gi);
            g.v[i][NC + c] = *reinterpret_cast<const TV*>(w4 + c * a.sc + gi);
        }
    }
}

// LDS: [2*NC][16*CB lines][NP + pad]; arrays 0..NC-1 hold w3, NC..2NC-1 w4.
template <typename M, int NC, int RB, int CB>
__device__ __forceinline__ void x_store(const XArgs& a, const XRegs<M, NC, RB, CB>& g) {
    typedef typename M::elem T;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* R = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = 16 * CB * RS;
    const int nvec = 16 * CB * NP / VN;
    const int vpl = NP / VN;
#pragma unroll
    for (int i = 0; i < XRegs<M, NC, RB, CB>::ITER; ++i) {
        const int v = threadIdx.x + i * blockDim.x;
        if (v >= nvec) break;
        const int j = v / vpl, x = (v - j * vpl) * VN;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            *reinterpret_cast<TV*>(R + c * AST + j * RS + x) = g.v[i][c];
            *reinterpret_cast<TV*>(R + (NC + c) * AST + j * RS + x) = g.v[i][NC + c];
        }
    }
}

// Workgroup: NP/(16 RB) waves over 16*CB consecutive x-lines.  Wave w owns
// the spectral/physical x rows of blocks RB*w .. RB*w+RB-1 of every product,
// for all CB line blocks.  Runs on a staged tile; arrays 0..NC-1 then hold
// c, then e, and arrays NC..2NC-1 hold d.
template <typename M, int NC, int RB, int CB>
__device__ __forceinline__ void x_compute(const XArgs& a, long tile) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    constexpr int NA = 2 * NC;
    constexpr int NL = 16 * CB;           // lines per tile
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* R = reinterpret_cast<T*>(smem_raw);

    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = NL * RS;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const long line0 = tile * NL;
    const void* __restrict__ P = a.P;
    const T tau = T(a.tau);

    const int rb0 = RB * w;
    // B fragment qq of arrays q0..: array q0 + qq/CB, line li + 16 (qq%CB), x = k0 .. k0+KL
    auto bfrag_from = [&](int q0) {
        return [&, q0](int qq, int k0) {
            return lds_vec<T, M::KL>(R + (q0 + qq / CB) * AST + (li + 16 * (qq % CB)) * RS + k0);
        };
    };
    // element (line li + 16 cb, x row of accumulator register e of block rb0+r) of array q
    auto at = [&](int q, int cb, int r, int e) -> T& {
        return R[q * AST + (li + 16 * cb) * RS + 16 * (rb0 + r) + M::row(lg, e)];
    };
    const T* __restrict__ dg = static_cast<const T*>(a.diag);

    // res[r][q*CB + cb]: w3 (q < NC) and w4 (q >= NC) at this wave's x rows
    T4 res[RB][NA * CB];
    {
        // ---- b1 = P w3, b2 = P w4 ----
        T4 acc[RB][NA * CB];
        zero<T, RB, NA * CB>(acc);
        gemm<M, RB, NA * CB>(P, NP, rb0, li, lg, acc, bfrag_from(0));
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int qq = 0; qq < NA * CB; ++qq)
#pragma unroll
                for (int e = 0; e < 4; ++e) res[r][qq][e] = at(qq / CB, qq % CB, r, e);
        __syncthreads();
        // ---- c = (q1 - 1) b1 + tau (q2 - 1) b2 into arrays 0..NC-1 ----
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const T* d1 = dg + c * a.diag_cstride + 16 * (rb0 + r);
                const T* d2 = d1 + a.diag_sstride;
#pragma unroll
                for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int k = M::row(lg, e);
                        at(c, cb, r, e) = d1[k] * acc[r][c * CB + cb][e] + d2[k] * acc[r][(NC + c) * CB + cb][e];
                    }
            }
        __syncthreads();
    }

    // ---- W = w3 + tau w4 + P c; d = f(W) - w4; V = W + tau d/2 ----
    T4 acc[RB][NC * CB];
    zero<T, RB, NC * CB>(acc);
    gemm<M, RB, NC * CB>(P, NP, rb0, li, lg, acc, bfrag_from(0));
    T4 V[RB][NC * CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const long line = line0 + li + 16 * cb;
        const int ly = int(line % a.npy), lz = int(line / a.npy);
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                T Wv[NC], F[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    Wv[c] = res[r][c * CB + cb][e] + tau * res[r][(NC + c) * CB + cb][e] + acc[r][c * CB + cb][e];
                react<T, NC>(a.rxn, Wv, F, 16 * (rb0 + r) + M::row(lg, e), ly, lz);
                if (a.Wout) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        static_cast<T*>(a.Wout)[c * a.sc + line * NP + 16 * (rb0 + r) + M::row(lg, e)] = Wv[c];
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const T d = F[c] - res[r][(NC + c) * CB + cb][e];
                    at(NC + c, cb, r, e) = d;
                    V[r][c * CB + cb][e] = Wv[c] + T(0.5) * tau * d;
                }
            }
    }
    zero<T, RB, NC * CB>(acc);
    __syncthreads();

    // ---- e = (q3 - 1/2) .* (P d) into arrays 0..NC-1 ----
    gemm<M, RB, NC * CB>(P, NP, rb0, li, lg, acc, bfrag_from(NC));
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const T* d3 = dg + c * a.diag_cstride + 2 * a.diag_sstride + 16 * (rb0 + r);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int e = 0; e < 4; ++e) at(c, cb, r, e) = d3[M::row(lg, e)] * acc[r][c * CB + cb][e];
        }
    zero<T, RB, NC * CB>(acc);
    __syncthreads();

    // ---- U+ = V + tau P e ----
    gemm<M, RB, NC * CB>(P, NP, rb0, li, lg, acc, bfrag_from(0));
    T* __restrict__ out = static_cast<T*>(a.out);
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const long line = line0 + li + 16 * cb;
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                T* o = out + c * a.sc + line * NP + 16 * (rb0 + r);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    o[M::row(lg, e)] = V[r][c * CB + cb][e] + tau * acc[r][c * CB + cb][e];
            }
    }
}

template <typename M, int NC, int RB, int CB>
__device__ __forceinline__ void x_tile(const XArgs& a, long tile) {
    XRegs<M, NC, RB, CB> g;
    x_load<M, NC, RB, CB>(a, tile, g);
    x_store<M, NC, RB, CB>(a, g);
    __syncthreads();
    x_compute<M, NC, RB, CB>(a, tile);
}

template <typename M, int NC, int RB, int CB, int MAXT>
__global__ __launch_bounds__(MAXT) void x_stage(XArgs a) {
    x_tile<M, NC, RB, CB>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Product-parallel path for 2-D problems.  A fused stage runs one workgroup
// per 16 columns (or lines) over the whole contracted direction, so a 511^2
// grid has only 32 tiles per stage.  Here every mode product is a launch of
// its own over (row group) x (16-column tile) blocks, and the scalings, the
// reaction and the increment-form residuals move into the epilogues; the
// intermediates stay in L2/MALL (2 MB per field at 511^2).  Every output is
// computed with the same operations in the same order as in the fused
// stages.  The y stage takes two launches, the x stage four:
//   YF: WC = dy .* (P U), WD = dy .* (P f(U))          (dy = Q1y - 1)
//   YB: WA = U + P WC (= w3), WB = f(U) + P WD (= w4)
//   X1: WC = d1 .* (P w3) + d2 .* (P w4)                (= c)
//   X2: W = w3 + tau w4 + P c; WD = f(W) - w4 (= d); U = W + tau d / 2 (= V)
//   X3: WC = d3 .* (P d)                                (= e)
//   X4: U = V + tau P e
// ---------------------------------------------------------------------------

enum SplitKind { kSplitYF = 0, kSplitYB = 1, kSplitX1 = 2, kSplitX2 = 3, kSplitX3 = 4, kSplitX4 = 5 };

struct SplitArgs {
    void* U;              // padded fields, component stride sc
    void* WA;
    void* WB;
    void* WC;
    void* WD;
    const void* P;        // NP x NP of the contracted direction
    const void* diag;     // slot kDiagY (y kinds) or kDiagX1 (x kinds) of component 0
    long diag_sstride, diag_cstride;
    int NP;               // contracted (padded) extent
    int npx;              // padded x extent (field row stride)
    long sc;
    double tau;
    RxnArgs rxn;          // at t_n (y kinds) or t_{n+1} (x kinds)
};

// QP arrays are staged per pass (as many as the LDS holds), so each P
// fragment feeds QP MFMAs per step.
template <typename M, int NC, int KIND, int NW, int QP>
__global__ __launch_bounds__(64 * NW) void split_product(SplitArgs a) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    constexpr bool YK = KIND <= kSplitYB;   // contracted direction y, columns are x
    constexpr int NARR = (KIND <= kSplitX1) ? 2 * NC : NC;
    static_assert(NARR % QP == 0, "passes must cover the arrays");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* X = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const int rb0 = int(blockIdx.x) * NW + w;   // this wave's 16-row block
    const int col0 = int(blockIdx.y) * 16;
    const long sc = a.sc;
    T* U = static_cast<T*>(a.U);
    T* WA = static_cast<T*>(a.WA);
    T* WB = static_cast<T*>(a.WB);
    T* WC = static_cast<T*>(a.WC);
    T* WD = static_cast<T*>(a.WD);
    // element (contracted or output index k, column c of the tile)
    auto at = [&](int k, int c) -> long {
        return YK ? long(k) * a.npx + col0 + c : long(col0 + c) * a.npx + k;
    };
    auto coords = [&](int k, int c, int& x, int& y) {
        x = YK ? col0 + c : k;
        y = YK ? k : col0 + c;
    };

    const int AST = 16 * RS;
    T4 acc[NARR / QP][1][QP];
#pragma unroll
    for (int q0 = 0; q0 < NARR; q0 += QP) {
      // stage arrays q0 .. q0+QP-1 of the tile: X[array][column][k]
#pragma unroll
      for (int q = q0; q < q0 + QP; ++q) {
        for (int v = tid; v < 16 * NP; v += blockDim.x) {
            const int k = YK ? v / 16 : v % NP;
            const int c = YK ? v % 16 : v / NP;
            const long gi = at(k, c);
            T val;
            if constexpr (KIND == kSplitYF) {
                if (q < NC) {
                    val = U[gi + q * sc];
                } else {
                    T u[NC], f[NC];
#pragma unroll
                    for (int cc = 0; cc < NC; ++cc) u[cc] = U[gi + cc * sc];
                    int x, y;
                    coords(k, c, x, y);
                    react<T, NC>(a.rxn, u, f, x, y, 0);
                    val = f[q - NC];
                }
            } else if constexpr (KIND == kSplitYB) {
                val = q < NC ? WC[gi + q * sc] : WD[gi + (q - NC) * sc];
            } else if constexpr (KIND == kSplitX1) {
                val = q < NC ? WA[gi + q * sc] : WB[gi + (q - NC) * sc];
            } else if constexpr (KIND == kSplitX2 || KIND == kSplitX4) {
                val = WC[gi + q * sc];
            } else {
                val = WD[gi + q * sc];
            }
            X[(q - q0) * AST + c * RS + k] = val;
        }
      }
        __syncthreads();
        zero<T, 1, QP>(acc[q0 / QP]);
        gemm<M, 1, QP>(a.P, NP, rb0, li, lg, acc[q0 / QP],
                       [&](int qq, int k0) { return lds_vec<T, M::KL>(X + qq * AST + li * RS + k0); });
        __syncthreads();
    }
    // result of array q at register e
    auto res = [&](int q, int e) { return acc[q / QP][0][q % QP][e]; };

    const T* __restrict__ dg = static_cast<const T*>(a.diag);
    const T tau = T(a.tau);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int k = 16 * rb0 + M::row(lg, e);
        const long gi = at(k, li);
        int x, y;
        coords(k, li, x, y);
        if constexpr (KIND == kSplitYF) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const T d = dg[c * a.diag_cstride + k];
                WC[gi + c * sc] = res(c, e) * d;
                WD[gi + c * sc] = res(NC + c, e) * d;
            }
        } else if constexpr (KIND == kSplitYB) {
            T u[NC], f[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) u[c] = U[gi + c * sc];
            react<T, NC>(a.rxn, u, f, x, y, 0);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                WA[gi + c * sc] = u[c] + res(c, e);
                WB[gi + c * sc] = f[c] + res(NC + c, e);
            }
        } else if constexpr (KIND == kSplitX1) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const T* d1 = dg + c * a.diag_cstride;
                const T* d2 = d1 + a.diag_sstride;
                WC[gi + c * sc] = d1[k] * res(c, e) + d2[k] * res(NC + c, e);
            }
        } else if constexpr (KIND == kSplitX2) {
            T Wv[NC], F[NC], w4[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                w4[c] = WB[gi + c * sc];
                Wv[c] = WA[gi + c * sc] + tau * w4[c] + res(c, e);
            }
            react<T, NC>(a.rxn, Wv, F, x, y, 0);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const T d = F[c] - w4[c];
                WD[gi + c * sc] = d;
                U[gi + c * sc] = Wv[c] + T(0.5) * tau * d;
            }
        } else if constexpr (KIND == kSplitX3) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
                WC[gi + c * sc] = dg[c * a.diag_cstride + 2 * a.diag_sstride + k] * res(c, e);
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) U[gi + c * sc] = U[gi + c * sc] + tau * res(c, e);
        }
    }
}

// ---------------------------------------------------------------------------
// Grouped (batched) launches: one persistent launch runs a stage for every
// instance of a shape class.  Instance i owns tiles start[i] .. start[i+1]-1
// of the launch; workgroups stride over the tiles, find their instance by
// binary search and run the same tile body with that instance's arguments.
// ---------------------------------------------------------------------------

template <typename A>
struct Group {
    const A* args;       // per-instance stage arguments (device memory)
    const long* start;   // [n + 1] first tile of each instance
    int n;
    long ntiles;
    double t0;           // time of the call's first step
    int k;               // the stage's time is t0 + k tau_i
};

template <typename A>
__device__ __forceinline__ int group_instance(const Group<A>& g, long tile) {
    int lo = 0, hi = g.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.start[mid] <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ void group_time(RxnArgs& r, double t0, int k) {
    if (r.kind == ETD_RXN_AC_MMS) r.exp_lt = exp(-r.p[0] * (t0 + k * r.tau));
}

template <typename M, int NC, bool FIRST, int RB, int CB, int MAXT>
__global__ __launch_bounds__(MAXT) void outer_group(Group<OuterArgs> g) {
    for (long t = blockIdx.x; t < g.ntiles; t += gridDim.x) {
        const int i = group_instance(g, t);
        OuterArgs a = g.args[i];
        group_time(a.rxn, g.t0, g.k);
        outer_tile<M, NC, FIRST, RB, CB>(a, t - g.start[i]);
        __syncthreads();   // the next tile restages the LDS
    }
}

template <typename M, int NC, int RB, int CB, int MAXT>
__global__ __launch_bounds__(MAXT) void x_group(Group<XArgs> g) {
    for (long t = blockIdx.x; t < g.ntiles; t += gridDim.x) {
        const int i = group_instance(g, t);
        XArgs a = g.args[i];
        group_time(a.rxn, g.t0, g.k);
        x_tile<M, NC, RB, CB>(a, t - g.start[i]);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// x stage of a two-component system whose joint tile exceeds the LDS: one
// component at a time, in two kernels around W (written to memory), because
// the reaction at W couples the components pointwise.
// ---------------------------------------------------------------------------

struct XSplitArgs {
    const void* w3;       // this component (a) / unused (b)
    const void* w4;       // this component
    const void* W;        // (b) W of component 0; component 1 at +sc
    void* out;            // (a) W of this component; (b) U+ of this component
    const void* P;
    const void* diag;     // slot X1 of this component
    long diag_sstride;
    int NP;
    long sc;
    int comp;
    int npy;
    double tau;
    RxnArgs rxn;          // at t_{n+1}
};

// (a) W = w3 + tau w4 + P ((q1 - 1) .* (P w3) + tau (q2 - 1) .* (P w4)).
// LDS: [2][16 lines][NP + pad] (w3 then c, w4).
template <typename M, int RB, int MAXT>
__global__ __launch_bounds__(MAXT) void x_stage_w(XSplitArgs a) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* R = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = 16 * RS;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const long line0 = long(blockIdx.x) * 16;
    const T* __restrict__ w3 = static_cast<const T*>(a.w3);
    const T* __restrict__ w4 = static_cast<const T*>(a.w4);
    const void* __restrict__ P = a.P;
    const T tau = T(a.tau);
    const int vpl = NP / VN;
#pragma unroll 4
    for (int v = tid; v < 16 * vpl; v += blockDim.x) {
        const int j = v / vpl, x = (v - j * vpl) * VN;
        const long gi = line0 * NP + long(v) * VN;
        *reinterpret_cast<TV*>(R + j * RS + x) = *reinterpret_cast<const TV*>(w3 + gi);
        *reinterpret_cast<TV*>(R + AST + j * RS + x) = *reinterpret_cast<const TV*>(w4 + gi);
    }
    __syncthreads();
    const int rb0 = RB * w;
    auto bfrag_from = [&](int q0) {
        return [&, q0](int q, int k0) { return lds_vec<T, M::KL>(R + (q0 + q) * AST + li * RS + k0); };
    };
    auto at = [&](int q, int r, int e) -> T& { return R[q * AST + li * RS + 16 * (rb0 + r) + M::row(lg, e)]; };
    const T* __restrict__ d1 = static_cast<const T*>(a.diag);
    const T* __restrict__ d2 = d1 + a.diag_sstride;
    T4 res[RB][2];
    {
        T4 acc[RB][2];
        zero<T, RB, 2>(acc);
        gemm<M, RB, 2>(P, NP, rb0, li, lg, acc, bfrag_from(0));
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) res[r][q][e] = at(q, r, e);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = 16 * (rb0 + r) + M::row(lg, e);
                at(0, r, e) = d1[k] * acc[r][0][e] + d2[k] * acc[r][1][e];
            }
        __syncthreads();
    }
    T4 acc[RB][1];
    zero<T, RB, 1>(acc);
    gemm<M, RB, 1>(P, NP, rb0, li, lg, acc, bfrag_from(0));
    T* __restrict__ o = static_cast<T*>(a.out) + (line0 + li) * NP;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            o[16 * (rb0 + r) + M::row(lg, e)] = res[r][0][e] + tau * res[r][1][e] + acc[r][0][e];
}

// (b) d = f_comp(W_u, W_v) - w4; U+ = W + tau d/2 + tau P ((q3 - 1/2) .* (P d)).
// LDS: [2][16 lines][NP + pad] (d, then e).
template <typename M, int RB, int MAXT>
__global__ __launch_bounds__(MAXT) void x_stage_u(XSplitArgs a) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* R = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = 16 * RS;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const long line0 = long(blockIdx.x) * 16;
    const T* __restrict__ W0 = static_cast<const T*>(a.W);
    const T* __restrict__ w4 = static_cast<const T*>(a.w4);
    const void* __restrict__ P = a.P;
    const T tau = T(a.tau);
    const int vpl = NP / VN;
#pragma unroll 4
    for (int v = tid; v < 16 * vpl; v += blockDim.x) {
        const int j = v / vpl, x = (v - j * vpl) * VN;
        const long gi = line0 * NP + long(v) * VN;
        const TV wu = *reinterpret_cast<const TV*>(W0 + gi);
        const TV wv = *reinterpret_cast<const TV*>(W0 + a.sc + gi);
        const TV b4 = *reinterpret_cast<const TV*>(w4 + gi);
        TV d;
#pragma unroll
        for (int t = 0; t < VN; ++t) {
            T fu, fv;
            react2<T>(a.rxn, wu[t], wv[t], fu, fv);
            d[t] = (a.comp == 0 ? fu : fv) - b4[t];
        }
        *reinterpret_cast<TV*>(R + j * RS + x) = d;
    }
    __syncthreads();
    const int rb0 = RB * w;
    auto bfrag_from = [&](int q0) {
        return [&, q0](int q, int k0) { return lds_vec<T, M::KL>(R + (q0 + q) * AST + li * RS + k0); };
    };
    auto at = [&](int q, int r, int e) -> T& { return R[q * AST + li * RS + 16 * (rb0 + r) + M::row(lg, e)]; };
    const T* __restrict__ d3 = static_cast<const T*>(a.diag) + 2 * a.diag_sstride;
    T4 acc[RB][1];
    zero<T, RB, 1>(acc);
    gemm<M, RB, 1>(P, NP, rb0, li, lg, acc, bfrag_from(0));
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) at(1, r, e) = d3[16 * (rb0 + r) + M::row(lg, e)] * acc[r][0][e];
    zero<T, RB, 1>(acc);
    __syncthreads();
    gemm<M, RB, 1>(P, NP, rb0, li, lg, acc, bfrag_from(1));
    const T* __restrict__ Wc = W0 + a.comp * a.sc + (line0 + li) * NP;
    T* __restrict__ o = static_cast<T*>(a.out) + (line0 + li) * NP;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int x = 16 * (rb0 + r) + M::row(lg, e);
            o[x] = Wc[x] + T(0.5) * tau * at(0, r, e) + tau * acc[r][0][e];
        }
}

// ---------------------------------------------------------------------------
// Adjoint of one step (reverse mode), for the gradient of a loss of U_N with
// respect to U_0, kappa_c and q.  With every Q symmetric and the directions
// commuting, the transpose of the step of Sec. 3.1 is
//   g  = tau Q3x U+bar,           Wbar = U+bar + J(W)^T g,
//   wbar = Q1x Wbar,              vbar = tau Q2x Wbar - g,
//   Ubar = L wbar + J(U)^T L vbar,   L = Q1y Q1z (3-D) or Q1y (2-D),
// and a parameter p enters through d lambda / d p:
//   dLoss/dp += <Wbar, dQ1x w> + tau <Wbar, dQ2x v> + tau <U+bar, dQ3x d>
//             + <wbar, dL U> + <vbar, dL f(U)>,     d = f(W) - v,
// each <a, dQ b> = sum over lines and modes j of (Pa)_j (Pb)_j Q'(tau
// lambda_j) tau d lambda_j / d p.  The x-direction part and the rest of the
// step are two fused kernels; each workgroup accumulates its FP64 partial
// sums [kappa_0 .. kappa_{NC-1}, q] into its own slot (no atomics, so the
// result is repeatable).
// ---------------------------------------------------------------------------

struct GradArgs {
    const double* table;  // derivative weights, [comp][dir][slot][kMaxPadded]
    double* partial;      // this launch's slots, NC + 1 doubles per workgroup
    int dir;              // contracted direction 0/1/2
    double inv_dim;       // d lambda / d q
};

// Block reduction of the lanes' partial sums; adds them into the slot of this
// workgroup (one writer per slot per launch).
template <int NG>
__device__ __forceinline__ void add_partials(double (&acc)[NG], double* partial) {
    __shared__ double red[16][NG];
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        double v = acc[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        acc[k] = v;
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NG; ++k) red[w][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < NG) {
        double t = 0.0;
        for (int i = 0; i < int(blockDim.x >> 6); ++i) t += red[i][threadIdx.x];
        partial[long(blockIdx.x) * NG + threadIdx.x] += t;
    }
}

struct XAdjArgs {
    const void* ubar;     // U+bar, all components (stride sc)
    const void* W;        // forward W
    const void* w;        // forward w3
    const void* v;        // forward w4
    void* wbar;           // out: Q1x Wbar
    void* vbar;           // out: tau Q2x Wbar - g
    const void* P;
    const void* diag;     // slot X1 of component 0
    long diag_sstride, diag_cstride;
    int NP;
    long sc;
    int npy;
    double tau;
    RxnArgs rxn;          // at t_{n+1}
    GradArgs grad;
};

// x-direction adjoint over 16 lines.  LDS: 8*NC fields [16 lines][NP + pad]:
// ubar, w, v, W (staged), S1 = P ubar, Sw = P w, Sv = P v (own rows), and the
// scaled coefficients; later slots are reused as noted.
template <typename M, int NC, int RB, int MAXT>
__global__ __launch_bounds__(MAXT) void x_adjoint(XAdjArgs a) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    constexpr int UB = 0, WW = NC, VV = 2 * NC, FW = 3 * NC, S1 = 4 * NC, SW = 5 * NC, SV = 6 * NC, GS = 7 * NC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* R = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = 16 * RS;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const long line0 = long(blockIdx.x) * 16;
    const void* __restrict__ P = a.P;
    const T tau = T(a.tau);
    const int vpl = NP / VN;
    const T* src[4] = {static_cast<const T*>(a.ubar), static_cast<const T*>(a.w), static_cast<const T*>(a.v),
                       static_cast<const T*>(a.W)};
#pragma unroll 2
    for (int v = tid; v < 16 * vpl; v += blockDim.x) {
        const int j = v / vpl, x = (v - j * vpl) * VN;
        const long gi = line0 * NP + long(v) * VN;
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int c = 0; c < NC; ++c)
                *reinterpret_cast<TV*>(R + (f * NC + c) * AST + j * RS + x) =
                    *reinterpret_cast<const TV*>(src[f] + c * a.sc + gi);
    }
    __syncthreads();
    const int rb0 = RB * w;
    auto bfrag_from = [&](int q0) {
        return [&, q0](int q, int k0) { return lds_vec<T, M::KL>(R + (q0 + q) * AST + li * RS + k0); };
    };
    auto at = [&](int q, int r, int e) -> T& { return R[q * AST + li * RS + 16 * (rb0 + r) + M::row(lg, e)]; };
    const T* __restrict__ dg = static_cast<const T*>(a.diag);
    const double* gt = a.grad.table;
    const long gcs = 3L * kGradSlots * kMaxPadded;   // component stride of the weight table

    // ---- S1 = P ubar, Sw = P w, Sv = P v ----
    T4 ub[RB][NC];
    {
        T4 acc[RB][3 * NC];
        zero<T, RB, 3 * NC>(acc);
        gemm<M, RB, 3 * NC>(P, NP, rb0, li, lg, acc, bfrag_from(0));
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const T* d3 = dg + c * a.diag_cstride + 2 * a.diag_sstride + 16 * (rb0 + r);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    ub[r][c][e] = at(UB + c, r, e);
                    at(S1 + c, r, e) = acc[r][c][e];
                    at(SW + c, r, e) = acc[r][NC + c][e];
                    at(SV + c, r, e) = acc[r][2 * NC + c][e];
                    at(GS + c, r, e) = d3[M::row(lg, e)] * acc[r][c][e];   // (q3 - 1/2) S1
                }
            }
    }
    __syncthreads();

    // ---- g = tau (ubar/2 + P ((q3 - 1/2) S1)); d = f(W) - v; Wbar = ubar + J(W)^T g ----
    double gacc[NC + 1];
#pragma unroll
    for (int k = 0; k <= NC; ++k) gacc[k] = 0.0;
    T4 g[RB][NC], wb[RB][NC];
    {
        T4 acc[RB][NC];
        zero<T, RB, NC>(acc);
        gemm<M, RB, NC>(P, NP, rb0, li, lg, acc, bfrag_from(GS));
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                T Wv[NC], F[NC], gg[NC], jt[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    gg[c] = tau * (T(0.5) * ub[r][c][e] + acc[r][c][e]);
                    g[r][c][e] = gg[c];
                    Wv[c] = at(FW + c, r, e);
                }
                const long line = line0 + li;
                const int x = 16 * (rb0 + r) + M::row(lg, e), y = int(line % a.npy), z = int(line / a.npy);
                react<T, NC>(a.rxn, Wv, F, x, y, z);
                react_jt<T, NC>(a.rxn, Wv, gg, jt);
                if (a.rxn.kind == ETD_RXN_AC_MMS) {   // psi(t_{n+1}) depends on kappa and q
                    const double ue = ac_ue(a.rxn, x, y, z) * double(gg[0]);
                    gacc[0] += a.rxn.ac_mu * ue;
                    gacc[NC] += ue;
                }
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    wb[r][c][e] = ub[r][c][e] + jt[c];
                    at(UB + c, r, e) = F[c] - at(VV + c, r, e);   // d, over ubar
                    at(WW + c, r, e) = wb[r][c][e];               // Wbar, over w
                }
            }
    }
    __syncthreads();

    // ---- Sd = P d, S2 = P Wbar; gradient terms; scaled coefficients of S2 ----
    {
        T4 acc[RB][2 * NC];
        zero<T, RB, 2 * NC>(acc);
        gemm<M, RB, 2 * NC>(P, NP, rb0, li, lg, acc, bfrag_from(UB));
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const T* d1 = dg + c * a.diag_cstride + 16 * (rb0 + r);
                const T* d2 = d1 + a.diag_sstride;
                const double* wt = gt + c * gcs + (long(a.grad.dir) * kGradSlots) * kMaxPadded + 16 * (rb0 + r);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = M::row(lg, e);
                    const double sd = acc[r][c][e], s2 = acc[r][NC + c][e];
                    const double t = s2 * double(at(SW + c, r, e)) * wt[kGradRho1 * kMaxPadded + k] +
                                     s2 * double(at(SV + c, r, e)) * wt[kGradRho2 * kMaxPadded + k] +
                                     double(at(S1 + c, r, e)) * sd * wt[kGradRho3 * kMaxPadded + k];
                    gacc[c] += t * wt[kGradMu * kMaxPadded + k];
                    gacc[NC] += t * a.grad.inv_dim;
                    at(VV + c, r, e) = d1[k] * T(s2);   // (q1 - 1) S2, over v
                    at(FW + c, r, e) = d2[k] * T(s2);   // tau (q2 - 1) S2, over W
                }
            }
    }
    __syncthreads();

    // ---- wbar = Wbar + P ((q1 - 1) S2); vbar = -g + tau Wbar + P (tau (q2 - 1) S2) ----
    {
        T4 acc[RB][2 * NC];
        zero<T, RB, 2 * NC>(acc);
        gemm<M, RB, 2 * NC>(P, NP, rb0, li, lg, acc, bfrag_from(VV));
        T* __restrict__ ow = static_cast<T*>(a.wbar);
        T* __restrict__ ov = static_cast<T*>(a.vbar);
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const long o = c * a.sc + (line0 + li) * NP + 16 * (rb0 + r);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int x = M::row(lg, e);
                    ow[o + x] = wb[r][c][e] + acc[r][c][e];
                    ov[o + x] = -g[r][c][e] + tau * wb[r][c][e] + acc[r][NC + c][e];
                }
            }
    }
    __syncthreads();
    add_partials<NC + 1>(gacc, a.grad.partial);
}

struct OuterAdjArgs {
    const void* a0;       // adjoint inputs (two fields)
    const void* a1;
    const void* f0;       // forward partners: middle: w1, v1; first: U (f(U) formed here)
    const void* f1;
    void* out0;           // Q1 a0, Q1 a1
    void* out1;
    const void* P;
    const void* diag;     // q1 - 1 of this direction, component 0
    long diag_cstride;
    int NP, ncb;
    long sk, sb, sc;
    int npx, npy, dim;
    RxnArgs rxn;          // first: f at t_n
    GradArgs grad;
};

// Adjoint of an outer stage (z or y): the forward stage applied to the two
// adjoint fields, plus the gradient terms <a, dQ1 f> against the forward
// partners.  LDS: 4*NC fields [16 columns][NP + pad]: a0, a1, f0, f1.
template <typename M, int NC, bool FIRST, int RB, int MAXT>
__global__ __launch_bounds__(MAXT) void outer_adjoint(OuterAdjArgs a) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    constexpr int VPR = 16 / VN;
    constexpr int NA = 2 * NC, NF = 4 * NC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* X = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = 16 * RS;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const int cb = blockIdx.x % a.ncb;
    const long bt = blockIdx.x / a.ncb;
    const long gbase = bt * a.sb + long(cb) * 16;
    const void* __restrict__ P = a.P;
    const T* a0 = static_cast<const T*>(a.a0);
    const T* a1 = static_cast<const T*>(a.a1);
    const T* f0 = static_cast<const T*>(a.f0);
    const T* f1 = static_cast<const T*>(a.f1);
#pragma unroll 2
    for (int v = tid; v < NP * VPR; v += blockDim.x) {
        const int k = v / VPR, j0 = (v - k * VPR) * VN;
        const long gi = gbase + long(k) * a.sk + j0;
        TV fa[NC], fb[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const TV x0 = *reinterpret_cast<const TV*>(a0 + gi + c * a.sc);
            const TV x1 = *reinterpret_cast<const TV*>(a1 + gi + c * a.sc);
            fa[c] = *reinterpret_cast<const TV*>(f0 + gi + c * a.sc);
            if constexpr (!FIRST) fb[c] = *reinterpret_cast<const TV*>(f1 + gi + c * a.sc);
#pragma unroll
            for (int t = 0; t < VN; ++t) {
                X[c * AST + (j0 + t) * RS + k] = x0[t];
                X[(NC + c) * AST + (j0 + t) * RS + k] = x1[t];
            }
        }
        if constexpr (FIRST) {
#pragma unroll
            for (int t = 0; t < VN; ++t) {
                const int col = cb * 16 + j0 + t;
                int x, y, z;
                if (a.dim == 3) {
                    z = k;
                    y = col / a.npx;
                    x = col - y * a.npx;
                } else {
                    z = 0;
                    y = k;
                    x = col;
                }
                T uu[NC], ff[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) uu[c] = fa[c][t];
                react<T, NC>(a.rxn, uu, ff, x, y, z);
#pragma unroll
                for (int c = 0; c < NC; ++c) fb[c][t] = ff[c];
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int t = 0; t < VN; ++t) {
                X[(NA + c) * AST + (j0 + t) * RS + k] = fa[c][t];
                X[(NA + NC + c) * AST + (j0 + t) * RS + k] = fb[c][t];
            }
    }
    __syncthreads();
    const int rb0 = RB * w;
    auto bfrag = [&](int q, int k0) { return lds_vec<T, M::KL>(X + q * AST + li * RS + k0); };
    auto at = [&](int q, int r, int e) -> T& { return X[q * AST + li * RS + 16 * (rb0 + r) + M::row(lg, e)]; };
    const T* __restrict__ dg = static_cast<const T*>(a.diag);
    const double* gt = a.grad.table;
    const long gcs = 3L * kGradSlots * kMaxPadded;
    double gacc[NC + 1];
#pragma unroll
    for (int k = 0; k <= NC; ++k) gacc[k] = 0.0;
    T4 acc[RB][NF];
    T4 res[RB][NA];
    zero<T, RB, NF>(acc);
    gemm<M, RB, NF>(P, NP, rb0, li, lg, acc, bfrag);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double* wt = gt + c * gcs + (long(a.grad.dir) * kGradSlots) * kMaxPadded + 16 * (rb0 + r);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = M::row(lg, e);
                const double t = (double(acc[r][c][e]) * acc[r][NA + c][e] +
                                  double(acc[r][NC + c][e]) * acc[r][NA + NC + c][e]) *
                                 wt[kGradRho1 * kMaxPadded + k];
                gacc[c] += t * wt[kGradMu * kMaxPadded + k];
                gacc[NC] += t * a.grad.inv_dim;
            }
        }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < NA; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) res[r][q][e] = at(q, r, e);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const T* dc = dg + (q % NC) * a.diag_cstride + 16 * (rb0 + r);
#pragma unroll
            for (int e = 0; e < 4; ++e) at(q, r, e) = acc[r][q][e] * dc[M::row(lg, e)];
        }
    __syncthreads();
    T4 acc2[RB][NA];
    zero<T, RB, NA>(acc2);
    gemm<M, RB, NA>(P, NP, rb0, li, lg, acc2, bfrag);
    T* __restrict__ out0 = static_cast<T*>(a.out0);
    T* __restrict__ out1 = static_cast<T*>(a.out1);
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            T* o = (q < NC ? out0 : out1) + (q % NC) * a.sc + gbase + li;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[long(16 * (rb0 + r) + M::row(lg, e)) * a.sk] = res[r][q][e] + acc2[r][q][e];
        }
    __syncthreads();
    add_partials<NC + 1>(gacc, a.grad.partial);
}

// Ubar = A + J(U)^T B over a padded field (all components at each node).
// B is the adjoint of f(t_n, U); where f depends on kappa or q explicitly
// (AC_MMS) the block adds <B, d f / d p> to its gradient slot.
template <typename T, int NC>
__global__ __launch_bounds__(256) void add_jt_field(const T* __restrict__ U, const T* __restrict__ A,
                                                    const T* __restrict__ B, T* __restrict__ out, long npts,
                                                    RxnArgs r, int px, int py, double* partial) {
    if (r.kind == ETD_RXN_AC_MMS) {
        double gacc[NC + 1];
#pragma unroll
        for (int k = 0; k <= NC; ++k) gacc[k] = 0.0;
        for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < npts; i += long(gridDim.x) * blockDim.x) {
            const long yz = i / px;
            const double ue = ac_ue(r, int(i - yz * px), int(yz % py), int(yz / py)) * double(B[i]);
            gacc[0] += r.ac_mu * ue;
            gacc[NC] += ue;
        }
        add_partials<NC + 1>(gacc, partial);
    }
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < npts; i += long(gridDim.x) * blockDim.x) {
        T u[NC], b[NC], jt[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            u[c] = U[c * npts + i];
            b[c] = B[c * npts + i];
        }
        react_jt<T, NC>(r, u, b, jt);
#pragma unroll
        for (int c = 0; c < NC; ++c) out[c * npts + i] = A[c * npts + i] + jt[c];
    }
}

template <typename T>
__global__ void copy_field(const T* __restrict__ src, T* __restrict__ dst, long n) {
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x) dst[i] = src[i];
}

__global__ void fill_zero(double* __restrict__ p, long n) {
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < n; i += long(gridDim.x) * blockDim.x) p[i] = 0.0;
}

// Sum the workgroup slots (fixed order) into out[NG].
__global__ void sum_partials(const double* __restrict__ part, long nslots, int ng, double* __restrict__ out) {
    __shared__ double sh[256];
    for (int k = 0; k < ng; ++k) {
        double t = 0.0;
        for (long i = threadIdx.x; i < nslots; i += blockDim.x) t += part[i * ng + k];
        sh[threadIdx.x] = t;
        __syncthreads();
        for (int st = blockDim.x / 2; st > 0; st >>= 1) {
            if (int(threadIdx.x) < st) sh[threadIdx.x] += sh[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = sh[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Layout conversion and validation reductions
// ---------------------------------------------------------------------------

struct Dims {
    int nc, nx, ny, nz;       // interior
    int px, py, pz;           // padded
};

// user layout (interior, contiguous) -> padded field (zeros on the padding)
template <typename T>
__global__ void pack_field(const T* __restrict__ src, T* __restrict__ dst, Dims d) {
    const long total = long(d.nc) * d.pz * d.py * d.px;
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < total; i += long(gridDim.x) * blockDim.x) {
        long t = i;
        const int x = int(t % d.px); t /= d.px;
        const int y = int(t % d.py); t /= d.py;
        const int z = int(t % d.pz);
        const int c = int(t / d.pz);
        T v = T(0);
        if (x < d.nx && y < d.ny && z < d.nz) v = src[((long(c) * d.nz + z) * d.ny + y) * d.nx + x];
        dst[i] = v;
    }
}

template <typename T>
__global__ void unpack_field(const T* __restrict__ src, T* __restrict__ dst, Dims d) {
    const long total = long(d.nc) * d.nz * d.ny * d.nx;
    for (long i = blockIdx.x * long(blockDim.x) + threadIdx.x; i < total; i += long(gridDim.x) * blockDim.x) {
        long t = i;
        const int x = int(t % d.nx); t /= d.nx;
        const int y = int(t % d.ny); t /= d.ny;
        const int z = int(t % d.nz);
        const int c = int(t / d.nz);
        dst[i] = src[((long(c) * d.pz + z) * d.py + y) * d.px + x];
    }
}

constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

// Per-block partial sums in a fixed order: [sum (a-b)^2, sum b^2, max|a-b|, #nonfinite(a)].
template <typename T>
__global__ __launch_bounds__(kRedThreads) void compare_partial(const T* __restrict__ a, const T* __restrict__ b,
                                                               long n, double* __restrict__ part) {
    __shared__ double sh[4][kRedThreads];
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (long i = blockIdx.x * long(kRedThreads) + threadIdx.x; i < n; i += long(gridDim.x) * kRedThreads) {
        const double av = double(a[i]), bv = double(b[i]);
        if (!isfinite(av)) {
            s3 += 1.0;
            continue;
        }
        const double df = av - bv;
        s0 += df * df;
        s1 += bv * bv;
        s2 = fmax(s2, fabs(df));
    }
    sh[0][threadIdx.x] = s0;
    sh[1][threadIdx.x] = s1;
    sh[2][threadIdx.x] = s2;
    sh[3][threadIdx.x] = s3;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
            sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + s]);
            sh[3][threadIdx.x] += sh[3][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(kRedThreads) void compare_final(double* __restrict__ part, int nblocks) {
    __shared__ double sh[4][kRedThreads];
    double s[4] = {0, 0, 0, 0};
    for (int i = threadIdx.x; i < nblocks; i += kRedThreads) {
        s[0] += part[i * 4 + 0];
        s[1] += part[i * 4 + 1];
        s[2] = fmax(s[2], part[i * 4 + 2]);
        s[3] += part[i * 4 + 3];
    }
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int st = kRedThreads / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + st];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + st];
            sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + st]);
            sh[3][threadIdx.x] += sh[3][threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[nblocks * 4 + 0] = sqrt(sh[0][0]);
        part[nblocks * 4 + 1] = sqrt(sh[1][0]);
        part[nblocks * 4 + 2] = sh[2][0];
        part[nblocks * 4 + 3] = sh[3][0];
    }
}

// ---------------------------------------------------------------------------
// Host-side launch plumbing
// ---------------------------------------------------------------------------

Dims dims_of(const Plan& p) {
    Dims d;
    d.nc = p.nc;
    d.nx = p.n[0];
    d.ny = p.n[1];
    d.nz = p.n[2];
    d.px = p.np[0];
    d.py = p.np[1];
    d.pz = p.np[2];
    return d;
}

RxnArgs rxn_args(const Plan& pl, const char* ws, double t) {
    const etd_problem& p = pl.prob;
    RxnArgs r;
    r.kind = p.rxn;
    for (int i = 0; i < 4; ++i) r.p[i] = p.rxn_param[i];
    r.sines = reinterpret_cast<const double*>(ws + pl.lay.sines);
    r.ac_rate = 0.0;
    r.ac_mu = 0.0;
    r.exp_lt = 0.0;
    r.tau = p.tau;
    if (p.rxn == ETD_RXN_AC_MMS) {
        const double lam = p.rxn_param[0];
        double mu = 0.0;
        for (int d = 0; d < p.dim; ++d) {
            const double L = p.hi[d] - p.lo[d];
            if (p.rxn_param[1] != 0.0) {
                const double h = L / (p.n[d] + 1);
                const double s = std::sin(M_PI * h / (2.0 * L));
                mu += 4.0 / (h * h) * s * s;
            } else {
                mu += (M_PI / L) * (M_PI / L);
            }
        }
        r.ac_rate = -lam + p.kappa[0] * mu + p.q;
        r.ac_mu = mu;
        r.exp_lt = std::exp(-lam * t);
    }
    return r;
}

// Raise a kernel's dynamic-LDS limit once per instantiation (the attribute
// persists for the process).
template <typename K>
hipError_t set_lds(K kernel, size_t bytes, size_t& done) {
    if (bytes <= done) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
    if (e == hipSuccess) done = bytes;
    return e;
}

// Tile shape of a stage launch.  Every wave owns `rb` 16-row blocks of each
// product (a tile has NP/(16 rb) waves) and a tile spans `cb` 16-column
// (outer stages) or 16-line (x stage) blocks, so that each P fragment read
// from L2 feeds 2*NC*cb MFMAs and each B fragment rb of them.  Instantiated
// (rb, cb, launch bound): (1,1,1024), (1,2,1024), (2,1,512), (2,1,1024),
// (4,1,1024), (2,2,512); with an FP32 state also (4,1,512) and (4,2,512),
// and for single-component x stages (2,4,512) and (1,4,1024).
//
// The default shape, measured on the 255^3 workload: for single-component
// FP64 systems up to NP = 256, one row block per wave over two column or line
// blocks (16 waves on one 132 KB tile: 2-5% faster than two row blocks per
// wave); otherwise rb = 2 up to NP = 512 and 4 beyond, two column blocks in
// the outer stages with an FP32 state, and x tiles of four line blocks for
// single-component FP32-state systems, two for other FP32 states (a
// two-component FP64 tile would spill).  An autotuned plan times every valid
// shape instead.
struct TileShape {
    int rb = 0, cb = 0;   // rb == 0: use the default
};

int shape_threads(int NP, int rb) { return 64 * (NP / (16 * rb)); }

template <typename T>
bool shape_rows_ok(int NP, int rb) {
    if (rb != 1 && rb != 2 && rb != 4) return false;
    if (NP % (16 * rb) != 0 || NP / (16 * rb) > kMaxWaves) return false;
    return !(rb == 4 && shape_threads(NP, rb) <= 512 && sizeof(T) != 4);
}

template <typename T, int NC>
bool outer_shape_ok(int NP, TileShape t) {
    if (!shape_rows_ok<T>(NP, t.rb)) return false;
    if (t.cb == 2) {
        if (t.rb >= 2 && shape_threads(NP, t.rb) > 512) return false;
        if (t.rb == 4 && sizeof(T) != 4) return false;
    } else if (t.cb != 1) {
        return false;
    }
    return outer_lds_bytes(NP, 2 * NC, t.cb, sizeof(T)) <= kMaxLds;
}

template <typename T, int NC>
bool x_shape_ok(int NP, long nlines, TileShape t) {
    if (!shape_rows_ok<T>(NP, t.rb)) return false;
    if (t.cb == 2 || t.cb == 4) {
        if (t.rb >= 2 && shape_threads(NP, t.rb) > 512) return false;
        if (t.rb == 4 && (t.cb == 4 || sizeof(T) != 4)) return false;
        if (t.cb == 4 && !(sizeof(T) == 4 && NC == 1)) return false;
    } else if (t.cb != 1) {
        return false;
    }
    if (nlines % (16 * t.cb) != 0) return false;
    return x_lds_bytes(NP, 2 * NC, t.cb, sizeof(T)) <= kMaxLds;
}

template <typename T, int NC>
TileShape default_outer_shape(int NP) {
    if (sizeof(T) == 8 && NC == 1 && outer_shape_ok<T, NC>(NP, TileShape{1, 2})) return TileShape{1, 2};
    if (sizeof(T) == 4 && outer_shape_ok<T, NC>(NP, TileShape{2, 2})) return TileShape{2, 2};
    return TileShape{rows_per_wave(NP), 1};
}

template <typename T, int NC>
TileShape default_x_shape(int NP, long nlines) {
    if (sizeof(T) == 8 && NC == 1 && x_shape_ok<T, NC>(NP, nlines, TileShape{1, 2})) return TileShape{1, 2};
    if (sizeof(T) == 4 && NC == 1 && x_shape_ok<T, NC>(NP, nlines, TileShape{2, 4})) return TileShape{2, 4};
    if ((sizeof(T) == 4 || NC == 1) && x_shape_ok<T, NC>(NP, nlines, TileShape{2, 2})) return TileShape{2, 2};
    return TileShape{rows_per_wave(NP), 1};
}

// Defaults per matrix-core policy: split-BF16 products add four row blocks per
// wave on two column blocks in the outer stages (each split B fragment then
// feeds 24 MFMAs; 7-9% faster than (2, 2) on the 255^3 workload).
template <typename M, int NC>
TileShape default_outer_for(int NP) {
    typedef typename M::elem T;
    if (M::SPLIT_B && NC == 1 && outer_shape_ok<T, NC>(NP, TileShape{4, 2})) return TileShape{4, 2};
    return default_outer_shape<T, NC>(NP);
}

template <typename M, int NC>
TileShape default_x_for(int NP, long nlines) {
    return default_x_shape<typename M::elem, NC>(NP, nlines);
}

int tile_threads(int NP) { return shape_threads(NP, rows_per_wave(NP)); }

// Launch kern<RB, MAXT> for the padded length NP with the default rows per
// wave: (2, 512) up to 256, (2, 1024) up to 512, (4, 1024) up to 1024.
#define DISPATCH_SHAPE(NP, KERNEL, ...)                                   \
    ((NP) <= 256 ? KERNEL(2, 512, __VA_ARGS__)                            \
                 : ((NP) <= 512 ? KERNEL(2, 1024, __VA_ARGS__) : KERNEL(4, 1024, __VA_ARGS__)))

// Workgroups of a kernel resident on the whole device at once (the grid of a
// persistent launch).  Each launcher caches it per instantiation and LDS size.
template <typename K>
long resident_groups(K kernel, int threads, size_t lds) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), threads, lds) !=
            hipSuccess ||
        per_cu < 1 || cus < 1)
        return 0;
    return long(per_cu) * cus;
}

struct GridCache {
    size_t lds = 0;
    long resident = 0;
    template <typename K>
    long grid(K kernel, int threads, size_t l, long ntiles) {
        if (l != lds || resident == 0) {
            resident = resident_groups(kernel, threads, l);
            lds = l;
        }
        return resident > 0 ? std::max(1L, std::min(ntiles, resident)) : ntiles;
    }
};

template <typename M, int NC, bool FIRST, int RB, int CB, int MAXT>
etd_status launch_outer_k(const OuterArgs& a, long ntiles, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = outer_lds_bytes(a.NP, 2 * NC, CB, sizeof(T));
    auto k = outer_stage<M, NC, FIRST, RB, CB, MAXT>;
    static size_t done = 0;
    HIP_TRY(set_lds(k, lds, done), "outer stage LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(ntiles)), dim3(shape_threads(a.NP, RB)), lds, s, a);
    HIP_TRY(hipGetLastError(), "outer stage launch");
    return ETD_OK;
}

#define OUTER_K(RB, MAXT, M, NC, FIRST, CB, a, nb, s) launch_outer_k<M, NC, FIRST, RB, CB, MAXT>(a, nb, s)

template <typename M, int NC, bool FIRST, int RB, int CB, int MAXT>
etd_status launch_outer_group_k(const Group<OuterArgs>& g, int NP, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = outer_lds_bytes(NP, 2 * NC, CB, sizeof(T));
    auto k = outer_group<M, NC, FIRST, RB, CB, MAXT>;
    static size_t done = 0;
    static GridCache gc;
    HIP_TRY(set_lds(k, lds, done), "grouped outer stage LDS attribute");
    const int thr = shape_threads(NP, RB);
    hipLaunchKernelGGL(k, dim3(unsigned(gc.grid(k, thr, lds, g.ntiles))), dim3(thr), lds, s, g);
    HIP_TRY(hipGetLastError(), "grouped outer stage launch");
    return ETD_OK;
}

// Pick the instantiation of a valid shape: L is launch_outer_k or
// launch_outer_group_k applied through a generic lambda.
template <typename T, int NC, typename L>
etd_status outer_by_shape(int NP, TileShape t, L&& launch) {
    const bool small = shape_threads(NP, t.rb) <= 512;
    if (t.rb == 1)
        return t.cb == 2 ? launch(std::integral_constant<int, 1>{}, std::integral_constant<int, 2>{},
                                  std::integral_constant<int, 1024>{})
                         : launch(std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{},
                                  std::integral_constant<int, 1024>{});
    if (t.cb == 2) {
        if constexpr (sizeof(T) == 4)
            if (t.rb == 4)
                return launch(std::integral_constant<int, 4>{}, std::integral_constant<int, 2>{},
                              std::integral_constant<int, 512>{});
        return launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{},
                      std::integral_constant<int, 512>{});
    }
    if (t.rb == 2)
        return small ? launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{},
                              std::integral_constant<int, 512>{})
                     : launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{},
                              std::integral_constant<int, 1024>{});
    if (!small)
        return launch(std::integral_constant<int, 4>{}, std::integral_constant<int, 1>{},
                      std::integral_constant<int, 1024>{});
    if constexpr (sizeof(T) == 4)
        return launch(std::integral_constant<int, 4>{}, std::integral_constant<int, 1>{},
                      std::integral_constant<int, 512>{});
    return fail(ETD_EUNSUPPORTED, "tile shape not available at this precision");
}

// One outer stage over all components of one instance.  a.ncb and ncols16
// count 16-column blocks.  Systems whose joint tile exceeds the LDS run one
// component per launch with the default rows per wave.
template <typename M, int NC, bool FIRST>
etd_status launch_outer(OuterArgs a, long ncols16, TileShape t, hipStream_t s) {
    typedef typename M::elem T;
    if (NC == 2 && !outer_fused(a.NP, NC, sizeof(T))) {
        for (int c = 0; c < NC; ++c) {
            OuterArgs b = a;
            const long off = c * a.sc;
            b.in0 = static_cast<const T*>(a.in0) + off;
            b.in1 = FIRST ? nullptr : static_cast<const T*>(a.in1) + off;
            b.out0 = static_cast<T*>(a.out0) + off;
            b.out1 = static_cast<T*>(a.out1) + off;
            b.diag = static_cast<const T*>(a.diag) + c * a.diag_cstride;
            b.other = FIRST ? static_cast<const T*>(a.in0) + (1 - c) * a.sc : nullptr;
            b.comp = c;
            const etd_status st = DISPATCH_SHAPE(a.NP, OUTER_K, M, 1, FIRST, 1, b, ncols16, s);
            if (st != ETD_OK) return st;
        }
        return ETD_OK;
    }
    if (t.rb == 0) t = default_outer_for<M, NC>(a.NP);
    a.ncb /= t.cb;
    return outer_by_shape<T, NC>(a.NP, t, [&](auto rb, auto cb, auto mt) {
        return launch_outer_k<M, NC, FIRST, decltype(rb)::value, decltype(cb)::value, decltype(mt)::value>(
            a, ncols16 / decltype(cb)::value, s);
    });
}

template <typename M, int NC, int RB, int CB, int MAXT>
etd_status launch_x_k(const XArgs& a, long nlines, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = x_lds_bytes(a.NP, 2 * NC, CB, sizeof(T));
    auto k = x_stage<M, NC, RB, CB, MAXT>;
    static size_t done = 0;
    HIP_TRY(set_lds(k, lds, done), "x stage LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(nlines / (16 * CB))), dim3(shape_threads(a.NP, RB)), lds, s, a);
    HIP_TRY(hipGetLastError(), "x stage launch");
    return ETD_OK;
}

template <typename M, int NC, int RB, int CB, int MAXT>
etd_status launch_x_group_k(const Group<XArgs>& g, int NP, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = x_lds_bytes(NP, 2 * NC, CB, sizeof(T));
    auto k = x_group<M, NC, RB, CB, MAXT>;
    static size_t done = 0;
    static GridCache gc;
    HIP_TRY(set_lds(k, lds, done), "grouped x stage LDS attribute");
    const int thr = shape_threads(NP, RB);
    hipLaunchKernelGGL(k, dim3(unsigned(gc.grid(k, thr, lds, g.ntiles))), dim3(thr), lds, s, g);
    HIP_TRY(hipGetLastError(), "grouped x stage launch");
    return ETD_OK;
}

template <typename T, int NC, typename L>
etd_status x_by_shape(int NP, TileShape t, L&& launch) {
    const bool small = shape_threads(NP, t.rb) <= 512;
    if (t.rb == 1) {
        if (t.cb == 4) {
            if constexpr (sizeof(T) == 4 && NC == 1)
                return launch(std::integral_constant<int, 1>{}, std::integral_constant<int, 4>{},
                              std::integral_constant<int, 1024>{});
            return fail(ETD_EUNSUPPORTED, "tile shape not available for this system");
        }
        return t.cb == 2 ? launch(std::integral_constant<int, 1>{}, std::integral_constant<int, 2>{},
                                  std::integral_constant<int, 1024>{})
                         : launch(std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{},
                                  std::integral_constant<int, 1024>{});
    }
    if (t.cb == 4) {
        if constexpr (sizeof(T) == 4 && NC == 1)
            return launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 4>{},
                          std::integral_constant<int, 512>{});
        return fail(ETD_EUNSUPPORTED, "tile shape not available for this system");
    }
    if (t.cb == 2) {
        if constexpr (sizeof(T) == 4)
            if (t.rb == 4)
                return launch(std::integral_constant<int, 4>{}, std::integral_constant<int, 2>{},
                              std::integral_constant<int, 512>{});
        return launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 2>{},
                      std::integral_constant<int, 512>{});
    }
    if (t.rb == 2)
        return small ? launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{},
                              std::integral_constant<int, 512>{})
                     : launch(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{},
                              std::integral_constant<int, 1024>{});
    if (!small)
        return launch(std::integral_constant<int, 4>{}, std::integral_constant<int, 1>{},
                      std::integral_constant<int, 1024>{});
    if constexpr (sizeof(T) == 4)
        return launch(std::integral_constant<int, 4>{}, std::integral_constant<int, 1>{},
                      std::integral_constant<int, 512>{});
    return fail(ETD_EUNSUPPORTED, "tile shape not available at this precision");
}

template <typename M, int RB, int MAXT, bool SECOND>
etd_status launch_xsplit_k(const XSplitArgs& a, long nlines, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = x_lds_bytes(a.NP, 2, 1, sizeof(T));
    auto k = SECOND ? x_stage_u<M, RB, MAXT> : x_stage_w<M, RB, MAXT>;
    static size_t done = 0;
    HIP_TRY(set_lds(k, lds, done), "split x stage LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(nlines / 16)), dim3(tile_threads(a.NP)), lds, s, a);
    HIP_TRY(hipGetLastError(), "split x stage launch");
    return ETD_OK;
}

#define XS_K(RB, MAXT, M, SECOND, a, nl, s) launch_xsplit_k<M, RB, MAXT, SECOND>(a, nl, s)

// The x stage over all components of one instance.  `scratch` receives W
// when a system is split (its joint tile exceeds the LDS).
template <typename M, int NC>
etd_status launch_x(const XArgs& a, long nlines, TileShape t, typename M::elem* scratch, hipStream_t s) {
    typedef typename M::elem T;
    if (NC == 2 && !x_fused(a.NP, NC, sizeof(T))) {
        XSplitArgs b{};
        b.P = a.P;
        b.diag_sstride = a.diag_sstride;
        b.NP = a.NP;
        b.sc = a.sc;
        b.npy = a.npy;
        b.tau = a.tau;
        b.rxn = a.rxn;
        b.W = scratch;
        for (int c = 0; c < NC; ++c) {
            b.w3 = static_cast<const T*>(a.w3) + c * a.sc;
            b.w4 = static_cast<const T*>(a.w4) + c * a.sc;
            b.out = scratch + c * a.sc;
            b.diag = static_cast<const T*>(a.diag) + c * a.diag_cstride;
            b.comp = c;
            const etd_status st = DISPATCH_SHAPE(a.NP, XS_K, M, false, b, nlines, s);
            if (st != ETD_OK) return st;
        }
        for (int c = 0; c < NC; ++c) {
            b.w4 = static_cast<const T*>(a.w4) + c * a.sc;
            b.out = static_cast<T*>(a.out) + c * a.sc;
            b.diag = static_cast<const T*>(a.diag) + c * a.diag_cstride;
            b.comp = c;
            const etd_status st = DISPATCH_SHAPE(a.NP, XS_K, M, true, b, nlines, s);
            if (st != ETD_OK) return st;
        }
        return ETD_OK;
    }
    if (t.rb == 0) t = default_x_for<M, NC>(a.NP, nlines);
    return x_by_shape<T, NC>(a.NP, t, [&](auto rb, auto cb, auto mt) {
        return launch_x_k<M, NC, decltype(rb)::value, decltype(cb)::value, decltype(mt)::value>(a, nlines, s);
    });
}

TileShape plan_tile(const Plan& pl, int d) { return TileShape{pl.tile_rb[d], pl.tile_cb[d]}; }

etd_status timer_mark(StageTimer& t, int kind, bool begin, hipStream_t s);

#define TIMED(kind, call)                                           \
    do {                                                            \
        etd_status st_ = timer_mark(tm, kind, true, s);             \
        if (st_ != ETD_OK) return st_;                              \
        st_ = (call);                                               \
        if (st_ != ETD_OK) return st_;                              \
        st_ = timer_mark(tm, kind, false, s);                       \
        if (st_ != ETD_OK) return st_;                              \
    } while (0)

// Arguments of one step's stage launches for one instance whose workspace
// region starts at ws (times are filled in per step).  Pdir[d] is the P table
// the instance uses for direction d (a batch shares one per extent).
// outer[k] / ocols[k]: the k-th outer stage and its 16-column blocks;
// nlines: x lines.  Default tile shapes are applied by the launchers.
struct StepArgs {
    int nouter = 0;
    OuterArgs outer[2];
    long ocols[2] = {0, 0};
    int odir[2] = {0, 0};   // contracted direction of each outer stage
    XArgs x;
    long nlines = 0;
    void* split_scratch = nullptr;   // W of a split x stage
};

StepArgs step_args(const Plan& pl, char* ws, const void* const Pdir[3]) {
    const int px = pl.np[0], py = pl.np[1], pz = pl.np[2];
    const long sc = long(px) * py * pz;
    const size_t e = pl.elem;
    char* U = ws + pl.lay.field[0];
    char* WA = ws + pl.lay.field[1];
    char* WB = ws + pl.lay.field[2];
    char* WC = ws + pl.lay.field[3];
    char* WD = ws + pl.lay.field[4];
    const char* diag = ws + pl.lay.diag;
    const long dstride = long(pl.diag_stride);
    const long dcs = long(kDiagSlots) * dstride;
    StepArgs a;
    OuterArgs o{};
    o.diag_cstride = dcs;
    o.sc = sc;
    o.npx = px;
    o.npy = py;
    o.dim = pl.dim;
    const char* w3;
    const char* w4;
    if (pl.dim == 3) {
        // z stage: contracted index z (stride px*py), columns (y, x)
        o.in0 = U;
        o.in1 = nullptr;
        o.out0 = WA;
        o.out1 = WB;
        o.P = Pdir[2];
        o.diag = diag + long(kDiagZ) * dstride * e;
        o.NP = pz;
        o.ncb = px * py / 16;
        o.sk = long(px) * py;
        o.sb = 0;
        a.outer[0] = o;
        a.ocols[0] = o.ncb;
        a.odir[0] = 2;
        // y stage: contracted index y (stride px), columns x, batches z
        o.in0 = WA;
        o.in1 = WB;
        o.out0 = WC;
        o.out1 = WD;
        o.P = Pdir[1];
        o.diag = diag + long(kDiagY) * dstride * e;
        o.NP = py;
        o.ncb = px / 16;
        o.sk = px;
        o.sb = long(px) * py;
        a.outer[1] = o;
        a.ocols[1] = long(o.ncb) * pz;
        a.odir[1] = 1;
        a.nouter = 2;
        w3 = WC;
        w4 = WD;
        a.split_scratch = WA;
    } else {
        o.in0 = U;
        o.in1 = nullptr;
        o.out0 = WA;
        o.out1 = WB;
        o.P = Pdir[1];
        o.diag = diag + long(kDiagY) * dstride * e;
        o.NP = py;
        o.ncb = px / 16;
        o.sk = px;
        o.sb = 0;
        a.outer[0] = o;
        a.ocols[0] = o.ncb;
        a.odir[0] = 1;
        a.nouter = 1;
        w3 = WA;
        w4 = WB;
        a.split_scratch = WC;
    }
    XArgs& x = a.x;
    x = XArgs{};
    x.w3 = w3;
    x.w4 = w4;
    x.out = U;
    x.P = Pdir[0];
    x.diag = diag + long(kDiagX1) * dstride * e;
    x.diag_sstride = dstride;
    x.diag_cstride = dcs;
    x.NP = px;
    x.sc = sc;
    x.npy = py;
    x.tau = pl.prob.tau;
    x.Wout = nullptr;
    a.nlines = long(py) * pz;
    return a;
}

// One product-parallel launch: row groups of 16*NW rows x 16-column tiles.
template <typename M, int NC, int KIND, int NW, int QP>
etd_status launch_split_k(const SplitArgs& a, long ncols, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = size_t(QP) * 16 * (a.NP + 16 / sizeof(T)) * sizeof(T);
    auto k = split_product<M, NC, KIND, NW, QP>;
    static size_t done = 0;
    HIP_TRY(set_lds(k, lds, done), "2-D product LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(a.NP / (16 * NW)), unsigned(ncols / 16)), dim3(64 * NW), lds, s, a);
    HIP_TRY(hipGetLastError(), "2-D product launch");
    return ETD_OK;
}

template <typename M, int NC, int KIND, int NW>
etd_status launch_split_nw(const SplitArgs& a, long ncols, hipStream_t s) {
    typedef typename M::elem T;
    constexpr int NARR = (KIND <= kSplitX1) ? 2 * NC : NC;
    const size_t per = size_t(16) * (a.NP + 16 / sizeof(T)) * sizeof(T);
    if constexpr (NARR % 4 == 0)
        if (4 * per <= kMaxLds) return launch_split_k<M, NC, KIND, NW, 4>(a, ncols, s);
    if constexpr (NARR % 2 == 0)
        if (2 * per <= kMaxLds) return launch_split_k<M, NC, KIND, NW, 2>(a, ncols, s);
    return launch_split_k<M, NC, KIND, NW, 1>(a, ncols, s);
}

template <typename M, int NC, int KIND>
etd_status launch_split(const SplitArgs& a, long ncols, hipStream_t s) {
    return a.NP % 64 == 0 ? launch_split_nw<M, NC, KIND, 4>(a, ncols, s) : launch_split_nw<M, NC, KIND, 2>(a, ncols, s);
}

// 2-D problems take the product-parallel path when it has at least 128
// blocks per launch (NP_y / 64 row groups x NP_x / 16 column tiles; from
// about 512^2 on), where the fused stages would have only NP_x / 16 tiles.
bool use_split2d(const Plan& pl) { return pl.dim == 2 && long(pl.np[1] / 64) * (pl.np[0] / 16) >= 128; }

template <typename M, int NC>
etd_status run_steps_split2d(const Plan& pl, StageTimer& tm, char* ws, double t0, int nsteps, hipStream_t s) {
    typedef typename M::elem T;
    const long dstride = long(pl.diag_stride);
    const char* diag = ws + pl.lay.diag;
    SplitArgs a{};
    a.U = ws + pl.lay.field[0];
    a.WA = ws + pl.lay.field[1];
    a.WB = ws + pl.lay.field[2];
    a.WC = ws + pl.lay.field[3];
    a.WD = ws + pl.lay.field[4];
    a.diag_sstride = dstride;
    a.diag_cstride = long(kDiagSlots) * dstride;
    a.npx = pl.np[0];
    a.sc = long(pl.np[0]) * pl.np[1];
    a.tau = pl.prob.tau;
    SplitArgs y = a, x = a;
    y.P = ws + pl.lay.P[1];
    y.diag = diag + long(kDiagY) * dstride * pl.elem;
    y.NP = pl.np[1];
    x.P = ws + pl.lay.P[0];
    x.diag = diag + long(kDiagX1) * dstride * pl.elem;
    x.NP = pl.np[0];
    const long nx = pl.np[0], ny = pl.np[1];
    for (int step = 0; step < nsteps; ++step) {
        y.rxn = rxn_args(pl, ws, t0 + step * pl.prob.tau);
        x.rxn = rxn_args(pl, ws, t0 + (step + 1) * pl.prob.tau);
        TIMED(0, (launch_split<M, NC, kSplitYF>(y, nx, s)));
        TIMED(0, (launch_split<M, NC, kSplitYB>(y, nx, s)));
        TIMED(2, (launch_split<M, NC, kSplitX1>(x, ny, s)));
        TIMED(2, (launch_split<M, NC, kSplitX2>(x, ny, s)));
        TIMED(2, (launch_split<M, NC, kSplitX3>(x, ny, s)));
        TIMED(2, (launch_split<M, NC, kSplitX4>(x, ny, s)));
    }
    return ETD_OK;
}

template <typename M, int NC>
etd_status run_steps(const Plan& pl, StageTimer& tm, char* ws, double t0, int nsteps, hipStream_t s,
                     typename M::elem* w_out = nullptr) {
    typedef typename M::elem T;
    if (w_out == nullptr && use_split2d(pl)) return run_steps_split2d<M, NC>(pl, tm, ws, t0, nsteps, s);
    const void* Pdir[3] = {ws + pl.lay.P[0], ws + pl.lay.P[1], ws + pl.lay.P[2]};
    StepArgs a = step_args(pl, ws, Pdir);
    a.x.Wout = w_out;
    const double tau = pl.prob.tau;
    for (int step = 0; step < nsteps; ++step) {
        const double tn = t0 + step * tau;
        const double tn1 = t0 + (step + 1) * tau;
        for (int k = 0; k < a.nouter; ++k) {
            a.outer[k].rxn = rxn_args(pl, ws, tn);
            if (k == 0) TIMED(0, (launch_outer<M, NC, true>(a.outer[0], a.ocols[0], plan_tile(pl, a.odir[0]), s)));
            else TIMED(1, (launch_outer<M, NC, false>(a.outer[1], a.ocols[1], plan_tile(pl, a.odir[1]), s)));
        }
        a.x.rxn = rxn_args(pl, ws, tn1);
        TIMED(2, (launch_x<M, NC>(a.x, a.nlines, plan_tile(pl, 0), static_cast<T*>(a.split_scratch), s)));
    }
    return ETD_OK;
}

// One step from Uin to Uout (padded fields, any buffers) that keeps its stage
// fields: f = [w1, w2, w3, w4, W] in 3-D, [w1, w2, W] in 2-D (w1, w2 the
// first stage's outputs, W the x stage's).  Fused tiles only (the adjoint's
// own limits imply them).
template <typename M, int NC>
etd_status replay_step(const Plan& pl, StageTimer& tm, char* ws, double tn, const void* Uin, void* Uout,
                       char* const* f, hipStream_t s) {
    typedef typename M::elem T;
    const void* Pdir[3] = {ws + pl.lay.P[0], ws + pl.lay.P[1], ws + pl.lay.P[2]};
    StepArgs a = step_args(pl, ws, Pdir);
    a.outer[0].in0 = Uin;
    a.outer[0].out0 = f[0];
    a.outer[0].out1 = f[1];
    if (pl.dim == 3) {
        a.outer[1].in0 = f[0];
        a.outer[1].in1 = f[1];
        a.outer[1].out0 = f[2];
        a.outer[1].out1 = f[3];
        a.x.w3 = f[2];
        a.x.w4 = f[3];
        a.x.Wout = f[4];
    } else {
        a.x.w3 = f[0];
        a.x.w4 = f[1];
        a.x.Wout = f[2];
    }
    a.x.out = Uout;
    for (int k = 0; k < a.nouter; ++k) {
        a.outer[k].rxn = rxn_args(pl, ws, tn);
        if (k == 0) TIMED(0, (launch_outer<M, NC, true>(a.outer[0], a.ocols[0], plan_tile(pl, a.odir[0]), s)));
        else TIMED(1, (launch_outer<M, NC, false>(a.outer[1], a.ocols[1], plan_tile(pl, a.odir[1]), s)));
    }
    a.x.rxn = rxn_args(pl, ws, tn + pl.prob.tau);
    TIMED(2, (launch_x<M, NC>(a.x, a.nlines, plan_tile(pl, 0), reinterpret_cast<T*>(ws + pl.lay.field[4]), s)));
    return ETD_OK;
}

template <typename M>
etd_status advance_m(const Plan& pl, StageTimer& tm, void* u, double t0, int nsteps, char* ws, hipStream_t s) {
    typedef typename M::elem T;
    const Dims d = dims_of(pl);
    T* U = reinterpret_cast<T*>(ws + pl.lay.field[0]);
    hipLaunchKernelGGL(pack_field<T>, dim3(2048), dim3(256), 0, s, static_cast<const T*>(u), U, d);
    HIP_TRY(hipGetLastError(), "pack launch");
    etd_status st = pl.nc == 1 ? run_steps<M, 1>(pl, tm, ws, t0, nsteps, s) : run_steps<M, 2>(pl, tm, ws, t0, nsteps, s);
    if (st != ETD_OK) return st;
    hipLaunchKernelGGL(unpack_field<T>, dim3(2048), dim3(256), 0, s, U, static_cast<T*>(u), d);
    HIP_TRY(hipGetLastError(), "unpack launch");
    return ETD_OK;
}

// ---------------------------------------------------------------------------
// Adjoint driver: sqrt(N) checkpointing
// ---------------------------------------------------------------------------

struct AdjLayout {
    int K = 1, nck = 1;          // segment length and number of checkpoints
    size_t field = 0;            // bytes per padded field
    size_t ck = 0, seg = 0;      // checkpoint and segment states
    // per step of a segment, the stage fields the reverse sweep reads:
    // w1, w2, (3-D: w3, w4,) W, each `field` bytes, kSlotFields per step
    int slot_fields = 0;
    size_t slots = 0;
    size_t Ub = 0, A[4] = {0, 0, 0, 0};
    // gradient slots of the x, y and z adjoint kernels and of the pointwise kernel
    size_t part[4] = {0, 0, 0, 0};
    long nslots[4] = {0, 0, 0, 0};
    size_t gsum = 0;             // reduced gradient sums [4][NC + 1]
    size_t total = 0;
};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr long kPointSlots = 2048;   // workgroups of the pointwise adjoint kernel

AdjLayout adjoint_layout(const Plan& pl, int nsteps) {
    AdjLayout L;
    L.K = std::max(1, int(std::ceil(std::sqrt(double(std::max(nsteps, 1))))));
    L.nck = (std::max(nsteps, 1) + L.K - 1) / L.K;
    L.field = pl.lay.field_bytes;
    const int ng = pl.nc + 1;
    const int px = pl.np[0], py = pl.np[1], pz = pl.np[2];
    L.nslots[0] = long(py) * pz / 16;
    if (pl.dim == 3) {
        L.nslots[1] = long(px) / 16 * pz;
        L.nslots[2] = long(px) * py / 16;
    } else {
        L.nslots[1] = long(px) / 16;
    }
    L.nslots[3] = kPointSlots;
    size_t off = 0;
    L.ck = off;
    off += size_t(L.nck) * L.field;
    L.seg = off;
    off += size_t(L.K) * L.field;
    L.slot_fields = pl.dim == 3 ? 5 : 3;
    L.slots = off;
    off += size_t(L.K) * L.slot_fields * L.field;
    L.Ub = off;
    off += L.field;
    for (int i = 0; i < 4; ++i) {
        L.A[i] = off;
        off += L.field;
    }
    for (int k = 0; k < 4; ++k) {
        L.part[k] = off;
        off = a256(off + size_t(std::max(L.nslots[k], 1L)) * ng * 8);
    }
    L.gsum = off;
    off = a256(off + 4 * size_t(ng) * 8);
    L.total = off;
    return L;
}

size_t x_adjoint_lds(int NP, int nc, size_t elem) { return x_lds_bytes(NP, 8 * nc, 1, elem); }
size_t outer_adjoint_lds(int NP, int nc, size_t elem) { return outer_lds_bytes(NP, 4 * nc, 1, elem); }
constexpr size_t kStaticLds = 1024;   // the reduction scratch of add_partials

etd_status adjoint_supported(const Plan& pl) {
    const size_t e = pl.elem;
    if (!x_fused(pl.np[0], pl.nc, e) || x_adjoint_lds(pl.np[0], pl.nc, e) + kStaticLds > kMaxLds)
        return fail(ETD_EUNSUPPORTED, "the adjoint x tile exceeds the LDS budget at this size, precision and component count");
    for (int d = 1; d < pl.dim; ++d)
        if (outer_adjoint_lds(pl.np[d], pl.nc, e) + kStaticLds > kMaxLds)
            return fail(ETD_EUNSUPPORTED, "the adjoint outer tile exceeds the LDS budget at this size and precision");
    return ETD_OK;
}

template <typename M, int NC, int RB, int MAXT>
etd_status launch_xadj_k(const XAdjArgs& a, long nlines, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = x_adjoint_lds(a.NP, NC, sizeof(T));
    auto k = x_adjoint<M, NC, RB, MAXT>;
    static size_t done = 0;
    HIP_TRY(set_lds(k, lds, done), "adjoint x LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(nlines / 16)), dim3(shape_threads(a.NP, RB)), lds, s, a);
    HIP_TRY(hipGetLastError(), "adjoint x launch");
    return ETD_OK;
}
#define XADJ_K(RB, MAXT, M, NC, a, nl, s) launch_xadj_k<M, NC, RB, MAXT>(a, nl, s)

// Adjoint tiles hold four (outer) or eight (x) fields per component, so at
// small extents few workgroups fit per CU: one row block per wave up to
// NP = 128 doubles their waves (the adjoint kernels of a 127^3 two-component
// FP32 step: 0.335 -> 0.296 ms).
#define ADJ_SHAPE(NP, KERNEL, ...) ((NP) <= 128 ? KERNEL(1, 512, __VA_ARGS__) : DISPATCH_SHAPE(NP, KERNEL, __VA_ARGS__))

template <typename M, int NC, bool FIRST, int RB, int MAXT>
etd_status launch_oadj_k(const OuterAdjArgs& a, long nblocks, hipStream_t s) {
    typedef typename M::elem T;
    const size_t lds = outer_adjoint_lds(a.NP, NC, sizeof(T));
    auto k = outer_adjoint<M, NC, FIRST, RB, MAXT>;
    static size_t done = 0;
    HIP_TRY(set_lds(k, lds, done), "adjoint outer LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(nblocks)), dim3(shape_threads(a.NP, RB)), lds, s, a);
    HIP_TRY(hipGetLastError(), "adjoint outer launch");
    return ETD_OK;
}
#define OADJ_K(RB, MAXT, M, NC, FIRST, a, nb, s) launch_oadj_k<M, NC, FIRST, RB, MAXT>(a, nb, s)

template <typename T>
etd_status copy_f(const T* src, T* dst, long n, hipStream_t s) {
    hipLaunchKernelGGL(copy_field<T>, dim3(2048), dim3(256), 0, s, src, dst, n);
    HIP_TRY(hipGetLastError(), "copy launch");
    return ETD_OK;
}

#define TRY(expr)                          \
    do {                                   \
        const etd_status st_ = (expr);     \
        if (st_ != ETD_OK) return st_;     \
    } while (0)

template <typename M, int NC>
etd_status adjoint_t(const Plan& pl, StageTimer& tm, const void* u0, double t0, int N, const void* ubarN,
                     void* ubar0, double* grad, char* ws, char* aws, const AdjLayout& L, hipStream_t s) {
    typedef typename M::elem T;
    const int px = pl.np[0], py = pl.np[1], pz = pl.np[2];
    const long sc = long(px) * py * pz;
    const long nf = sc * NC;   // elements per field
    const double tau = pl.prob.tau;
    const Dims dm = dims_of(pl);
    const int ng = NC + 1;
    auto F = [&](size_t off) { return reinterpret_cast<T*>(aws + off); };
    T* U = reinterpret_cast<T*>(ws + pl.lay.field[0]);
    T* ck = F(L.ck);
    T* seg = F(L.seg);
    T* Ub = F(L.Ub);
    // stage fields of step i of the segment
    auto slot = [&](int i, int j) { return aws + L.slots + (size_t(i) * L.slot_fields + j) * L.field; };
    T* A[4] = {F(L.A[0]), F(L.A[1]), F(L.A[2]), F(L.A[3])};
    const size_t fe = L.field / sizeof(T);   // elements between consecutive fields
    const T* diag = reinterpret_cast<const T*>(ws + pl.lay.diag);
    const long dstride = long(pl.diag_stride), dcs = long(kDiagSlots) * dstride;
    const double* gtab = reinterpret_cast<const double*>(ws + pl.lay.grad);

    // ---- forward pass: checkpoints every K steps ----
    hipLaunchKernelGGL(pack_field<T>, dim3(2048), dim3(256), 0, s, static_cast<const T*>(u0), U, dm);
    HIP_TRY(hipGetLastError(), "pack launch");
    for (int c = 0; c < L.nck; ++c) {
        TRY(copy_f<T>(U, ck + c * fe, nf, s));
        const int n0 = c * L.K, n1 = std::min(N, n0 + L.K);
        if (c + 1 < L.nck) TRY((run_steps<M, NC>(pl, tm, ws, t0 + n0 * tau, n1 - n0, s)));
    }
    // ---- adjoint state and gradient slots ----
    hipLaunchKernelGGL(pack_field<T>, dim3(2048), dim3(256), 0, s, static_cast<const T*>(ubarN), Ub, dm);
    HIP_TRY(hipGetLastError(), "pack launch");
    for (int k = 0; k < 4; ++k) {
        hipLaunchKernelGGL(fill_zero, dim3(64), dim3(256), 0, s, reinterpret_cast<double*>(aws + L.part[k]),
                           std::max(L.nslots[k], 1L) * ng);
        HIP_TRY(hipGetLastError(), "fill launch");
    }
    const double inv_dim = 1.0 / pl.dim;

    for (int c = L.nck - 1; c >= 0; --c) {
        const int n0 = c * L.K, n1 = std::min(N, n0 + L.K);
        // replay the segment, keeping every state and every step's stage fields
        TRY(copy_f<T>(ck + c * fe, seg, nf, s));
        for (int i = 0; i < n1 - n0; ++i) {
            char* f[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
            for (int j = 0; j < L.slot_fields; ++j) f[j] = slot(i, j);
            void* out = i + 1 < n1 - n0 ? static_cast<void*>(seg + (i + 1) * fe) : static_cast<void*>(U);
            TRY((replay_step<M, NC>(pl, tm, ws, t0 + (n0 + i) * tau, seg + i * fe, out, f, s)));
        }
        for (int i = n1 - n0 - 1; i >= 0; --i) {
            const int n = n0 + i;
            const double tn = t0 + n * tau, tn1 = t0 + (n + 1) * tau;
            T* Un = seg + i * fe;
            T* w1 = reinterpret_cast<T*>(slot(i, 0));
            T* w2 = reinterpret_cast<T*>(slot(i, 1));
            T* w3 = pl.dim == 3 ? reinterpret_cast<T*>(slot(i, 2)) : w1;
            T* w4 = pl.dim == 3 ? reinterpret_cast<T*>(slot(i, 3)) : w2;
            T* Wf = reinterpret_cast<T*>(slot(i, L.slot_fields - 1));
            // x direction
            XAdjArgs xa{};
            xa.ubar = Ub;
            xa.W = Wf;
            xa.w = w3;
            xa.v = w4;
            xa.wbar = A[0];
            xa.vbar = A[1];
            xa.P = ws + pl.lay.P[0];
            xa.diag = diag + long(kDiagX1) * dstride;
            xa.diag_sstride = dstride;
            xa.diag_cstride = dcs;
            xa.NP = px;
            xa.sc = sc;
            xa.npy = py;
            xa.tau = tau;
            xa.rxn = rxn_args(pl, ws, tn1);
            xa.grad = GradArgs{gtab, reinterpret_cast<double*>(aws + L.part[0]), 0, inv_dim};
            TRY(ADJ_SHAPE(px, XADJ_K, M, NC, xa, long(py) * pz, s));
            // outer directions
            OuterAdjArgs oa{};
            oa.diag_cstride = dcs;
            oa.sc = sc;
            oa.npx = px;
            oa.npy = py;
            oa.dim = pl.dim;
            oa.rxn = rxn_args(pl, ws, tn);
            const T *Lw, *Lv;
            if (pl.dim == 3) {
                oa.a0 = A[0]; oa.a1 = A[1]; oa.f0 = w1; oa.f1 = w2; oa.out0 = A[2]; oa.out1 = A[3];
                oa.P = ws + pl.lay.P[1];
                oa.diag = diag + long(kDiagY) * dstride;
                oa.NP = py; oa.ncb = px / 16; oa.sk = px; oa.sb = long(px) * py;
                oa.grad = GradArgs{gtab, reinterpret_cast<double*>(aws + L.part[1]), 1, inv_dim};
                TRY(ADJ_SHAPE(py, OADJ_K, M, NC, false, oa, long(px / 16) * pz, s));
                oa.a0 = A[2]; oa.a1 = A[3]; oa.f0 = Un; oa.f1 = nullptr; oa.out0 = A[0]; oa.out1 = A[1];
                oa.P = ws + pl.lay.P[2];
                oa.diag = diag + long(kDiagZ) * dstride;
                oa.NP = pz; oa.ncb = px * py / 16; oa.sk = long(px) * py; oa.sb = 0;
                oa.grad = GradArgs{gtab, reinterpret_cast<double*>(aws + L.part[2]), 2, inv_dim};
                TRY(ADJ_SHAPE(pz, OADJ_K, M, NC, true, oa, long(px) * py / 16, s));
                Lw = A[0];
                Lv = A[1];
            } else {
                oa.a0 = A[0]; oa.a1 = A[1]; oa.f0 = Un; oa.f1 = nullptr; oa.out0 = A[2]; oa.out1 = A[3];
                oa.P = ws + pl.lay.P[1];
                oa.diag = diag + long(kDiagY) * dstride;
                oa.NP = py; oa.ncb = px / 16; oa.sk = px; oa.sb = 0;
                oa.grad = GradArgs{gtab, reinterpret_cast<double*>(aws + L.part[1]), 1, inv_dim};
                TRY(ADJ_SHAPE(py, OADJ_K, M, NC, true, oa, long(px / 16), s));
                Lw = A[2];
                Lv = A[3];
            }
            hipLaunchKernelGGL((add_jt_field<T, NC>), dim3(unsigned(kPointSlots)), dim3(256), 0, s, Un, Lw, Lv, Ub,
                               sc, rxn_args(pl, ws, tn), px, py, reinterpret_cast<double*>(aws + L.part[3]));
            HIP_TRY(hipGetLastError(), "adjoint pointwise launch");
        }
    }
    hipLaunchKernelGGL(unpack_field<T>, dim3(2048), dim3(256), 0, s, Ub, static_cast<T*>(ubar0), dm);
    HIP_TRY(hipGetLastError(), "unpack launch");
    double* gs = reinterpret_cast<double*>(aws + L.gsum);
    for (int k = 0; k < 4; ++k) {
        hipLaunchKernelGGL(sum_partials, dim3(1), dim3(256), 0, s, reinterpret_cast<const double*>(aws + L.part[k]),
                           std::max(L.nslots[k], 1L), ng, gs + k * ng);
        HIP_TRY(hipGetLastError(), "gradient reduction launch");
    }
    double host[4 * 3];
    HIP_TRY(hipMemcpyAsync(host, gs, 4 * ng * sizeof(double), hipMemcpyDeviceToHost, s), "gradient copy");
    HIP_TRY(hipStreamSynchronize(s), "gradient sync");
    for (int k = 0; k < ng; ++k) grad[k] = host[k] + host[ng + k] + host[2 * ng + k] + host[3 * ng + k];
    return ETD_OK;
}

etd_status check_ws(const Plan& pl, const void* ws) {
    if (!ws) return fail(ETD_EWORKSPACE, "workspace pointer is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(ETD_EWORKSPACE, "workspace must be 256-byte aligned");
    (void)pl;
    return ETD_OK;
}

// Record an event for the start (begin = true) or end of a stage launch.
etd_status timer_mark(StageTimer& t, int kind, bool begin, hipStream_t s) {
    if (!t.on) return ETD_OK;
    if (t.used == t.pool.size()) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e), "timing event create");
        t.pool.push_back(e);
    }
    HIP_TRY(hipEventRecord(t.pool[t.used], s), "timing event record");
    ++t.used;
    if (begin) t.kind.push_back(kind);
    return ETD_OK;
}

// ---------------------------------------------------------------------------
// Autotuning: time every valid tile shape of a stage and keep the fastest.
// All shapes compute every output with the same operations in the same
// order, so the choice changes the speed, never the result.
// ---------------------------------------------------------------------------

template <typename T, int NC>
std::vector<TileShape> outer_candidates(int NP) {
    std::vector<TileShape> v;
    for (int rb : {1, 2, 4})
        for (int cb : {1, 2})
            if (outer_shape_ok<T, NC>(NP, TileShape{rb, cb})) v.push_back(TileShape{rb, cb});
    return v;
}

template <typename T, int NC>
std::vector<TileShape> x_candidates(int NP, long nlines) {
    std::vector<TileShape> v;
    for (int rb : {1, 2, 4})
        for (int cb : {1, 2, 4})
            if (x_shape_ok<T, NC>(NP, nlines, TileShape{rb, cb})) v.push_back(TileShape{rb, cb});
    return v;
}

// Mean milliseconds of `launch` over `reps` launches after one warm-up.
template <typename L>
etd_status time_launches(L&& launch, int reps, hipStream_t s, float& ms) {
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "autotune event");
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(he, "autotune event");
    }
    etd_status st = launch();
    if (st == ETD_OK) {
        he = hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == ETD_OK; ++r) st = launch();
        if (he == hipSuccess) he = hipEventRecord(e1, s);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (st == ETD_OK && he != hipSuccess) st = hip_fail(he, "autotune timing");
        ms /= float(reps);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

constexpr int kTuneReps = 5;
constexpr int kMaxBatch = 4096;   // instances per batch

template <typename M, int NC>
etd_status autotune_plan_t(Plan& pl, char* ws, hipStream_t s) {
    typedef typename M::elem T;
    if (NC == 2 && (!x_fused(pl.np[0], NC, sizeof(T)) ||
                    !outer_fused(pl.np[1], NC, sizeof(T)) || (pl.dim == 3 && !outer_fused(pl.np[2], NC, sizeof(T)))))
        return ETD_OK;   // split systems run one fixed shape
    const void* Pdir[3] = {ws + pl.lay.P[0], ws + pl.lay.P[1], ws + pl.lay.P[2]};
    StepArgs a = step_args(pl, ws, Pdir);
    for (int k = 0; k < a.nouter; ++k) a.outer[k].rxn = rxn_args(pl, ws, 0.0);
    a.x.rxn = rxn_args(pl, ws, pl.prob.tau);
    for (int k = 0; k < a.nouter; ++k) {
        const int d = a.odir[k];
        TileShape best{};
        float best_ms = 0.f;
        for (TileShape t : outer_candidates<T, NC>(pl.np[d])) {
            float ms = 0.f;
            const etd_status st = time_launches([&]() {
                return k == 0 ? launch_outer<M, NC, true>(a.outer[0], a.ocols[0], t, s)
                              : launch_outer<M, NC, false>(a.outer[1], a.ocols[1], t, s);
            }, kTuneReps, s, ms);
            if (st != ETD_OK) return st;
            if (best.rb == 0 || ms < best_ms) {
                best = t;
                best_ms = ms;
            }
        }
        pl.tile_rb[d] = best.rb;
        pl.tile_cb[d] = best.cb;
    }
    TileShape best{};
    float best_ms = 0.f;
    for (TileShape t : x_candidates<T, NC>(pl.np[0], a.nlines)) {
        float ms = 0.f;
        const etd_status st = time_launches(
            [&]() { return launch_x<M, NC>(a.x, a.nlines, t, static_cast<T*>(a.split_scratch), s); }, kTuneReps, s,
            ms);
        if (st != ETD_OK) return st;
        if (best.rb == 0 || ms < best_ms) {
            best = t;
            best_ms = ms;
        }
    }
    pl.tile_rb[0] = best.rb;
    pl.tile_cb[0] = best.cb;
    return ETD_OK;
}

// Validate and resolve a tile request for one direction of a plan: (0, 0)
// selects the default shape.
template <typename M, int NC>
etd_status resolve_tile(const Plan& pl, int d, TileShape t, TileShape& out) {
    typedef typename M::elem T;
    const int NP = pl.np[d];
    const long nlines = long(pl.np[1]) * pl.np[2];
    if (t.rb == 0 && t.cb == 0) {
        out = d == 0 ? default_x_for<M, NC>(NP, nlines) : default_outer_for<M, NC>(NP);
        return ETD_OK;
    }
    const bool ok = d == 0 ? x_shape_ok<T, NC>(NP, nlines, t) : outer_shape_ok<T, NC>(NP, t);
    if (!ok) return fail(ETD_EUNSUPPORTED, "tile shape not valid for this direction");
    out = t;
    return ETD_OK;
}

etd_status resolve_tile_any(const Plan& pl, int d, TileShape t, TileShape& out) {
    switch (pl.prob.precision) {
    case ETD_FP64:
        return pl.nc == 1 ? resolve_tile<NativeMma<double>, 1>(pl, d, t, out)
                          : resolve_tile<NativeMma<double>, 2>(pl, d, t, out);
    case ETD_FP32:
        return pl.nc == 1 ? resolve_tile<NativeMma<float>, 1>(pl, d, t, out)
                          : resolve_tile<NativeMma<float>, 2>(pl, d, t, out);
    default:
        return pl.nc == 1 ? resolve_tile<Bf16x6Mma, 1>(pl, d, t, out) : resolve_tile<Bf16x6Mma, 2>(pl, d, t, out);
    }
}

// ---------------------------------------------------------------------------
// Batches: many independent instances (same dimension, component count and
// precision; any extents, coefficients, step, reaction and Pade order)
// advanced together.  Instances of one padded shape form a group; each group
// runs every stage of every step as ONE persistent grouped launch over all of
// its instances' tiles, on a stream of its own, so groups of different shapes
// overlap on the device.  Instances of equal extent share one P table.
// ---------------------------------------------------------------------------

struct BatchGroup {
    int np[3] = {1, 1, 1};
    std::vector<int> inst;            // instance indices
    TileShape tile[3];                // per direction
    size_t oargs[2] = {0, 0}, ostart[2] = {0, 0};   // descriptor offsets (bytes into the workspace)
    size_t xargs = 0, xstart = 0;
    long otiles[2] = {0, 0}, xtiles = 0;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
};

struct Batch {
    std::vector<Plan> plans;
    std::vector<size_t> base;         // workspace offset of each instance's region
    std::vector<int> powner[3];       // instance whose P table instance i uses, per direction
    std::vector<BatchGroup> groups;
    int dim = 0, nc = 0, precision = 0;
    size_t desc = 0, desc_bytes = 0, total = 0;
    char* uploaded = nullptr;         // the workspace the descriptors point into
    hipEvent_t fork = nullptr;
    // Bumped whenever the descriptors change shape or address; a graph
    // captured before then refuses to launch.  Shared with the graphs so that
    // it outlives the batch (0 = batch destroyed).
    std::shared_ptr<unsigned> generation = std::make_shared<unsigned>(1);
};

size_t desc_bytes_of(const Batch& B) {
    size_t n = 0;
    for (const BatchGroup& G : B.groups) {
        const size_t k = G.inst.size();
        n += size_t(B.dim - 1) * a256(k * sizeof(OuterArgs)) + size_t(B.dim - 1) * a256((k + 1) * sizeof(long));
        n += a256(k * sizeof(XArgs)) + a256((k + 1) * sizeof(long));
    }
    return n;
}

etd_status batch_layout(Batch& B) {
    size_t off = 0;
    B.base.resize(B.plans.size());
    for (size_t i = 0; i < B.plans.size(); ++i) {
        B.base[i] = off;
        off = a256(off + B.plans[i].lay.total);
    }
    for (int d = 0; d < 3; ++d) {
        B.powner[d].assign(B.plans.size(), 0);
        for (size_t i = 0; i < B.plans.size(); ++i) {
            size_t j = 0;
            while (j < i && !(B.plans[j].n[d] == B.plans[i].n[d] && B.plans[j].np[d] == B.plans[i].np[d])) ++j;
            B.powner[d][i] = int(j);
        }
    }
    for (size_t i = 0; i < B.plans.size(); ++i) {
        const Plan& pl = B.plans[i];
        size_t g = 0;
        while (g < B.groups.size() &&
               !(B.groups[g].np[0] == pl.np[0] && B.groups[g].np[1] == pl.np[1] && B.groups[g].np[2] == pl.np[2]))
            ++g;
        if (g == B.groups.size()) {
            BatchGroup G;
            for (int d = 0; d < 3; ++d) G.np[d] = pl.np[d];
            B.groups.push_back(G);
        }
        B.groups[g].inst.push_back(int(i));
    }
    B.desc = off;
    B.desc_bytes = desc_bytes_of(B);
    B.total = a256(off + B.desc_bytes);
    return ETD_OK;
}

// Host image of one group's descriptors for the workspace at ws, with the
// group's current tile shapes.
void group_descriptors(const Batch& B, BatchGroup& G, char* ws, size_t& off, std::vector<uint8_t>& img) {
    const int k = int(G.inst.size());
    std::vector<OuterArgs> oa[2];
    std::vector<long> os[2];
    std::vector<XArgs> xa;
    std::vector<long> xs;
    for (int j = 0; j < 2; ++j) os[j].push_back(0);
    xs.push_back(0);
    for (int i : G.inst) {
        const Plan& pl = B.plans[i];
        const void* Pdir[3];
        for (int d = 0; d < 3; ++d) {
            const int o = B.powner[d][i];
            Pdir[d] = ws + B.base[o] + B.plans[o].lay.P[d];
        }
        StepArgs a = step_args(pl, ws + B.base[i], Pdir);
        for (int j = 0; j < a.nouter; ++j) {
            const TileShape t = G.tile[a.odir[j]];
            a.outer[j].rxn = rxn_args(pl, ws + B.base[i], 0.0);
            a.outer[j].ncb /= t.cb;
            oa[j].push_back(a.outer[j]);
            os[j].push_back(os[j].back() + a.ocols[j] / t.cb);
        }
        a.x.rxn = rxn_args(pl, ws + B.base[i], 0.0);
        xa.push_back(a.x);
        xs.push_back(xs.back() + a.nlines / (16 * G.tile[0].cb));
    }
    auto put_bytes = [&](const void* src, size_t n) {
        const size_t at = off;
        std::memcpy(img.data() + (at - B.desc), src, n);
        off = a256(off + n);
        return at;
    };
    for (int j = 0; j < B.dim - 1; ++j) {
        G.oargs[j] = put_bytes(oa[j].data(), k * sizeof(OuterArgs));
        G.ostart[j] = put_bytes(os[j].data(), (k + 1) * sizeof(long));
        G.otiles[j] = os[j].back();
    }
    G.xargs = put_bytes(xa.data(), k * sizeof(XArgs));
    G.xstart = put_bytes(xs.data(), (k + 1) * sizeof(long));
    G.xtiles = xs.back();
}

// Rebuild and upload every group's descriptors (synchronous on s).
etd_status upload_descriptors(Batch& B, char* ws, hipStream_t s) {
    std::vector<uint8_t> img(B.desc_bytes, 0);
    size_t off = B.desc;
    for (BatchGroup& G : B.groups) group_descriptors(B, G, ws, off, img);
    HIP_TRY(hipMemcpyAsync(ws + B.desc, img.data(), img.size(), hipMemcpyHostToDevice, s), "descriptor upload");
    HIP_TRY(hipStreamSynchronize(s), "descriptor upload sync");
    B.uploaded = ws;
    ++*B.generation;
    return ETD_OK;
}

// One stage of one step for every instance of a group: stage 0 = first outer
// stage, 1 = middle outer stage (3-D), 2 = x stage.
template <typename M, int NC>
etd_status group_stage(const Batch& B, const BatchGroup& G, int stage, char* ws, double t0, int k, hipStream_t s) {
    typedef typename M::elem T;
    const int n = int(G.inst.size());
    if (stage < 2) {
        const int d = B.dim == 3 ? (stage == 0 ? 2 : 1) : 1;
        const int NP = G.np[d];
        Group<OuterArgs> g{reinterpret_cast<const OuterArgs*>(ws + G.oargs[stage]),
                           reinterpret_cast<const long*>(ws + G.ostart[stage]), n, G.otiles[stage], t0, k};
        if (stage == 0)
            return outer_by_shape<T, NC>(NP, G.tile[d], [&](auto rb, auto cb, auto mt) {
                return launch_outer_group_k<M, NC, true, decltype(rb)::value, decltype(cb)::value,
                                            decltype(mt)::value>(g, NP, s);
            });
        return outer_by_shape<T, NC>(NP, G.tile[d], [&](auto rb, auto cb, auto mt) {
            return launch_outer_group_k<M, NC, false, decltype(rb)::value, decltype(cb)::value, decltype(mt)::value>(
                g, NP, s);
        });
    }
    Group<XArgs> g{reinterpret_cast<const XArgs*>(ws + G.xargs), reinterpret_cast<const long*>(ws + G.xstart), n,
                   G.xtiles, t0, k};
    return x_by_shape<T, NC>(G.np[0], G.tile[0], [&](auto rb, auto cb, auto mt) {
        return launch_x_group_k<M, NC, decltype(rb)::value, decltype(cb)::value, decltype(mt)::value>(g, G.np[0], s);
    });
}

template <typename M, int NC>
etd_status batch_advance_t(Batch& B, void* const* u, double t0, int nsteps, char* ws, hipStream_t s) {
    typedef typename M::elem T;
    const bool fork = B.groups.size() > 1;
    if (fork) HIP_TRY(hipEventRecord(B.fork, s), "batch fork record");
    for (BatchGroup& G : B.groups) {
        hipStream_t gs = fork ? G.stream : s;
        if (fork) HIP_TRY(hipStreamWaitEvent(gs, B.fork, 0), "batch fork wait");
        for (int i : G.inst) {
            const Plan& pl = B.plans[i];
            hipLaunchKernelGGL(pack_field<T>, dim3(1024), dim3(256), 0, gs, static_cast<const T*>(u[i]),
                               reinterpret_cast<T*>(ws + B.base[i] + pl.lay.field[0]), dims_of(pl));
        }
        HIP_TRY(hipGetLastError(), "batch pack launch");
        for (int step = 0; step < nsteps; ++step) {
            for (int stage = 0; stage < B.dim - 1; ++stage) TRY((group_stage<M, NC>(B, G, stage, ws, t0, step, gs)));
            TRY((group_stage<M, NC>(B, G, 2, ws, t0, step + 1, gs)));
        }
        for (int i : G.inst) {
            const Plan& pl = B.plans[i];
            hipLaunchKernelGGL(unpack_field<T>, dim3(1024), dim3(256), 0, gs,
                               reinterpret_cast<const T*>(ws + B.base[i] + pl.lay.field[0]), static_cast<T*>(u[i]),
                               dims_of(pl));
        }
        HIP_TRY(hipGetLastError(), "batch unpack launch");
        if (fork) {
            HIP_TRY(hipEventRecord(G.done, gs), "batch join record");
            HIP_TRY(hipStreamWaitEvent(s, G.done, 0), "batch join wait");
        }
    }
    return ETD_OK;
}

template <typename M, int NC>
etd_status batch_autotune_t(Batch& B, char* ws, hipStream_t s) {
    typedef typename M::elem T;
    for (BatchGroup& G : B.groups) {
        const long nlines = long(G.np[1]) * G.np[2];
        for (int stage = 0; stage < B.dim; ++stage) {
            const int d = stage == B.dim - 1 ? 0 : (B.dim == 3 ? (stage == 0 ? 2 : 1) : 1);
            const int st_kind = stage == B.dim - 1 ? 2 : stage;
            const std::vector<TileShape> cand =
                d == 0 ? x_candidates<T, NC>(G.np[0], nlines) : outer_candidates<T, NC>(G.np[d]);
            TileShape best{};
            float best_ms = 0.f;
            for (TileShape t : cand) {
                G.tile[d] = t;
                TRY(upload_descriptors(B, ws, s));
                float ms = 0.f;
                TRY(time_launches([&]() { return group_stage<M, NC>(B, G, st_kind, ws, 0.0, 0, s); }, kTuneReps, s, ms));
                if (best.rb == 0 || ms < best_ms) {
                    best = t;
                    best_ms = ms;
                }
            }
            G.tile[d] = best;
        }
    }
    return upload_descriptors(B, ws, s);
}

// ---------------------------------------------------------------------------
// HIP graphs: the launches of a call captured once and replayed.
// ---------------------------------------------------------------------------

etd_status end_capture(hipStream_t s, etd_status st, hipGraph_t& g) {
    g = nullptr;
    const hipError_t he = hipStreamEndCapture(s, &g);
    if (st != ETD_OK) {
        if (g) (void)hipGraphDestroy(g);
        g = nullptr;
        return st;
    }
    if (he != hipSuccess) return hip_fail(he, "graph capture");
    return ETD_OK;
}

}  // namespace

struct etd_batch {
    Batch b;
};

struct etd_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::shared_ptr<unsigned> generation;   // batch graphs: the batch's token
    unsigned captured = 0;                  // its value at capture
};

namespace {

etd_status batch_dispatch_advance(Batch& B, void* const* u, double t0, int nsteps, char* ws, hipStream_t s) {
    switch (B.precision) {
    case ETD_FP64:
        return B.nc == 1 ? batch_advance_t<NativeMma<double>, 1>(B, u, t0, nsteps, ws, s)
                         : batch_advance_t<NativeMma<double>, 2>(B, u, t0, nsteps, ws, s);
    case ETD_FP32:
        return B.nc == 1 ? batch_advance_t<NativeMma<float>, 1>(B, u, t0, nsteps, ws, s)
                         : batch_advance_t<NativeMma<float>, 2>(B, u, t0, nsteps, ws, s);
    default:
        return B.nc == 1 ? batch_advance_t<Bf16x6Mma, 1>(B, u, t0, nsteps, ws, s)
                         : batch_advance_t<Bf16x6Mma, 2>(B, u, t0, nsteps, ws, s);
    }
}

etd_status batch_check(const Batch& B, void* const* u, int nsteps, const void* ws) {
    if (!u) return fail(ETD_EINVAL, "field pointer array is NULL");
    for (size_t i = 0; i < B.plans.size(); ++i)
        if (!u[i]) return fail(ETD_EINVAL, "a field pointer is NULL");
    if (nsteps < 0) return fail(ETD_EINVAL, "nsteps must be >= 0");
    if (!ws || ws != B.uploaded) return fail(ETD_EWORKSPACE, "workspace is not the one the batch was uploaded to");
    return ETD_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

etd_status etd_plan_create(const etd_problem* prob, etd_plan** out) {
    if (!prob || !out) return fail(ETD_EINVAL, "NULL argument");
    *out = nullptr;
    etd_plan* p = new (std::nothrow) etd_plan;
    if (!p) return fail(ETD_EINVAL, "out of host memory");
    std::string err;
    const etd_status st = build_plan(*prob, p->p, err);
    if (st != ETD_OK) {
        delete p;
        return fail(st, err);
    }
    *out = p;
    return ETD_OK;
}

etd_status etd_plan_workspace_bytes(const etd_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return fail(ETD_EINVAL, "NULL argument");
    *bytes = plan->p.lay.total;
    return ETD_OK;
}

etd_status etd_plan_upload(const etd_plan* plan, void* ws, size_t bytes, void* stream) {
    if (!plan) return fail(ETD_EINVAL, "NULL plan");
    etd_status st = check_ws(plan->p, ws);
    if (st != ETD_OK) return st;
    if (bytes < plan->p.lay.total) return fail(ETD_EWORKSPACE, "workspace smaller than etd_plan_workspace_bytes()");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(ws, plan->p.image.data(), plan->p.table_bytes, hipMemcpyHostToDevice, s), "table upload");
    // The stage buffers start zeroed so that padded lanes are exact zeros
    // before the first pack.
    HIP_TRY(hipMemsetAsync(static_cast<char*>(ws) + plan->p.lay.field[0], 0,
                           plan->p.lay.total - plan->p.lay.field[0], s),
            "workspace clear");
    // The host image must outlive the asynchronous copy.
    HIP_TRY(hipStreamSynchronize(s), "table upload sync");
    return ETD_OK;
}

etd_status etd_advance(const etd_plan* plan, void* u, double t0, int nsteps, void* ws, void* stream) {
    if (!plan) return fail(ETD_EINVAL, "NULL plan");
    if (nsteps < 0) return fail(ETD_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(t0)) return fail(ETD_EINVAL, "t0 must be finite");
    if (!u) return fail(ETD_EINVAL, "field pointer is NULL");
    etd_status st = check_ws(plan->p, ws);
    if (st != ETD_OK) return st;
    if (nsteps == 0) return ETD_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    switch (plan->p.prob.precision) {
    case ETD_FP64: return advance_m<NativeMma<double>>(plan->p, plan->timer, u, t0, nsteps, w, s);
    case ETD_FP32: return advance_m<NativeMma<float>>(plan->p, plan->timer, u, t0, nsteps, w, s);
    default: return advance_m<Bf16x6Mma>(plan->p, plan->timer, u, t0, nsteps, w, s);
    }
}

etd_status etd_adjoint_workspace_bytes(const etd_plan* plan, int nsteps, size_t* bytes) {
    if (!plan || !bytes) return fail(ETD_EINVAL, "NULL argument");
    if (nsteps < 1) return fail(ETD_EINVAL, "nsteps must be >= 1");
    const etd_status st = adjoint_supported(plan->p);
    if (st != ETD_OK) return st;
    *bytes = adjoint_layout(plan->p, nsteps).total;
    return ETD_OK;
}

etd_status etd_adjoint(const etd_plan* plan, const void* u0, double t0, int nsteps, const void* ubar_final,
                       void* ubar0, double* grad, void* ws, void* adj_ws, size_t adj_bytes, void* stream) {
    if (!plan || !u0 || !ubar_final || !ubar0 || !grad) return fail(ETD_EINVAL, "NULL argument");
    if (nsteps < 1) return fail(ETD_EINVAL, "nsteps must be >= 1");
    if (!std::isfinite(t0)) return fail(ETD_EINVAL, "t0 must be finite");
    etd_status st = check_ws(plan->p, ws);
    if (st != ETD_OK) return st;
    st = adjoint_supported(plan->p);
    if (st != ETD_OK) return st;
    const AdjLayout L = adjoint_layout(plan->p, nsteps);
    if (!adj_ws || reinterpret_cast<uintptr_t>(adj_ws) % 256 != 0)
        return fail(ETD_EWORKSPACE, "adjoint workspace must be non-NULL and 256-byte aligned");
    if (adj_bytes < L.total) return fail(ETD_EWORKSPACE, "adjoint workspace smaller than etd_adjoint_workspace_bytes()");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    char* a = static_cast<char*>(adj_ws);
    const Plan& pl = plan->p;
    switch (pl.prob.precision) {
    case ETD_FP64:
        return pl.nc == 1 ? adjoint_t<NativeMma<double>, 1>(pl, plan->timer, u0, t0, nsteps, ubar_final, ubar0, grad, w, a, L, s)
                          : adjoint_t<NativeMma<double>, 2>(pl, plan->timer, u0, t0, nsteps, ubar_final, ubar0, grad, w, a, L, s);
    case ETD_FP32:
        return pl.nc == 1 ? adjoint_t<NativeMma<float>, 1>(pl, plan->timer, u0, t0, nsteps, ubar_final, ubar0, grad, w, a, L, s)
                          : adjoint_t<NativeMma<float>, 2>(pl, plan->timer, u0, t0, nsteps, ubar_final, ubar0, grad, w, a, L, s);
    default:
        return pl.nc == 1 ? adjoint_t<Bf16x6Mma, 1>(pl, plan->timer, u0, t0, nsteps, ubar_final, ubar0, grad, w, a, L, s)
                          : adjoint_t<Bf16x6Mma, 2>(pl, plan->timer, u0, t0, nsteps, ubar_final, ubar0, grad, w, a, L, s);
    }
}

etd_status etd_plan_autotune(etd_plan* plan, void* ws, void* stream) {
    if (!plan) return fail(ETD_EINVAL, "NULL plan");
    etd_status st = check_ws(plan->p, ws);
    if (st != ETD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    Plan& pl = plan->p;
    const bool timing = plan->timer.on;
    plan->timer.on = false;
    switch (pl.prob.precision) {
    case ETD_FP64:
        st = pl.nc == 1 ? autotune_plan_t<NativeMma<double>, 1>(pl, w, s) : autotune_plan_t<NativeMma<double>, 2>(pl, w, s);
        break;
    case ETD_FP32:
        st = pl.nc == 1 ? autotune_plan_t<NativeMma<float>, 1>(pl, w, s) : autotune_plan_t<NativeMma<float>, 2>(pl, w, s);
        break;
    default:
        st = pl.nc == 1 ? autotune_plan_t<Bf16x6Mma, 1>(pl, w, s) : autotune_plan_t<Bf16x6Mma, 2>(pl, w, s);
    }
    plan->timer.on = timing;
    return st;
}

etd_status etd_plan_tiles(const etd_plan* plan, int tiles[6]) {
    if (!plan || !tiles) return fail(ETD_EINVAL, "NULL argument");
    const Plan& pl = plan->p;
    for (int d = 0; d < 3; ++d) {
        TileShape t{};
        if (d < pl.dim) {
            const etd_status st = resolve_tile_any(pl, d, TileShape{pl.tile_rb[d], pl.tile_cb[d]}, t);
            if (st != ETD_OK) return st;
        }
        tiles[2 * d] = t.rb;
        tiles[2 * d + 1] = t.cb;
    }
    return ETD_OK;
}

etd_status etd_plan_set_tiles(etd_plan* plan, const int tiles[6]) {
    if (!plan || !tiles) return fail(ETD_EINVAL, "NULL argument");
    Plan& pl = plan->p;
    TileShape r[3];
    for (int d = 0; d < pl.dim; ++d) {
        const etd_status st = resolve_tile_any(pl, d, TileShape{tiles[2 * d], tiles[2 * d + 1]}, r[d]);
        if (st != ETD_OK) return st;
    }
    for (int d = 0; d < pl.dim; ++d) {
        const bool dflt = tiles[2 * d] == 0 && tiles[2 * d + 1] == 0;
        pl.tile_rb[d] = dflt ? 0 : r[d].rb;
        pl.tile_cb[d] = dflt ? 0 : r[d].cb;
    }
    return ETD_OK;
}

etd_status etd_batch_create(const etd_problem* probs, int count, etd_batch** out) {
    if (!probs || !out) return fail(ETD_EINVAL, "NULL argument");
    *out = nullptr;
    if (count < 1 || count > kMaxBatch) return fail(ETD_EINVAL, "count must be in 1..4096");
    etd_batch* b = new (std::nothrow) etd_batch;
    if (!b) return fail(ETD_EINVAL, "out of host memory");
    Batch& B = b->b;
    B.plans.resize(count);
    for (int i = 0; i < count; ++i) {
        std::string err;
        const etd_status st = build_plan(probs[i], B.plans[i], err);
        if (st != ETD_OK) {
            delete b;
            return fail(st, "instance " + std::to_string(i) + ": " + err);
        }
        const Plan& pl = B.plans[i];
        if (i == 0) {
            B.dim = pl.dim;
            B.nc = pl.nc;
            B.precision = pl.prob.precision;
        } else if (pl.dim != B.dim || pl.nc != B.nc || pl.prob.precision != B.precision) {
            delete b;
            return fail(ETD_EINVAL, "instance " + std::to_string(i) +
                                        ": a batch takes one dimension, component count and precision");
        }
        bool fused = x_fused(pl.np[0], pl.nc, pl.elem);
        for (int d = 1; d < pl.dim; ++d) fused = fused && outer_fused(pl.np[d], pl.nc, pl.elem);
        if (!fused) {
            delete b;
            return fail(ETD_EUNSUPPORTED, "instance " + std::to_string(i) +
                                              ": its two-component tile exceeds the LDS (single plans only)");
        }
    }
    batch_layout(B);
    for (BatchGroup& G : B.groups) {
        const Plan& pl = B.plans[G.inst[0]];
        for (int d = 0; d < pl.dim; ++d) {
            const etd_status st = resolve_tile_any(pl, d, TileShape{}, G.tile[d]);
            if (st != ETD_OK) {
                delete b;
                return st;
            }
        }
    }
    *out = b;
    return ETD_OK;
}

etd_status etd_batch_workspace_bytes(const etd_batch* batch, size_t* bytes) {
    if (!batch || !bytes) return fail(ETD_EINVAL, "NULL argument");
    *bytes = batch->b.total;
    return ETD_OK;
}

etd_status etd_batch_upload(etd_batch* batch, void* ws, size_t bytes, void* stream) {
    if (!batch) return fail(ETD_EINVAL, "NULL batch");
    Batch& B = batch->b;
    if (!ws || reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return fail(ETD_EWORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    if (bytes < B.total) return fail(ETD_EWORKSPACE, "workspace smaller than etd_batch_workspace_bytes()");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    for (size_t i = 0; i < B.plans.size(); ++i) {
        const Plan& pl = B.plans[i];
        HIP_TRY(hipMemcpyAsync(w + B.base[i], pl.image.data(), pl.table_bytes, hipMemcpyHostToDevice, s),
                "table upload");
        HIP_TRY(hipMemsetAsync(w + B.base[i] + pl.lay.field[0], 0, pl.lay.total - pl.lay.field[0], s),
                "workspace clear");
    }
    HIP_TRY(hipStreamSynchronize(s), "table upload sync");
    if (!B.fork) HIP_TRY(hipEventCreateWithFlags(&B.fork, hipEventDisableTiming), "batch event");
    for (BatchGroup& G : B.groups) {
        if (!G.stream) HIP_TRY(hipStreamCreateWithFlags(&G.stream, hipStreamNonBlocking), "batch stream");
        if (!G.done) HIP_TRY(hipEventCreateWithFlags(&G.done, hipEventDisableTiming), "batch event");
    }
    return upload_descriptors(B, w, s);
}

etd_status etd_batch_advance(etd_batch* batch, void* const* u, double t0, int nsteps, void* ws, void* stream) {
    if (!batch) return fail(ETD_EINVAL, "NULL batch");
    if (!std::isfinite(t0)) return fail(ETD_EINVAL, "t0 must be finite");
    Batch& B = batch->b;
    etd_status st = batch_check(B, u, nsteps, ws);
    if (st != ETD_OK) return st;
    if (nsteps == 0) return ETD_OK;
    return batch_dispatch_advance(B, u, t0, nsteps, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
}

etd_status etd_batch_autotune(etd_batch* batch, void* ws, void* stream) {
    if (!batch) return fail(ETD_EINVAL, "NULL batch");
    Batch& B = batch->b;
    if (!ws || ws != B.uploaded) return fail(ETD_EWORKSPACE, "workspace is not the one the batch was uploaded to");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    switch (B.precision) {
    case ETD_FP64:
        return B.nc == 1 ? batch_autotune_t<NativeMma<double>, 1>(B, w, s) : batch_autotune_t<NativeMma<double>, 2>(B, w, s);
    case ETD_FP32:
        return B.nc == 1 ? batch_autotune_t<NativeMma<float>, 1>(B, w, s) : batch_autotune_t<NativeMma<float>, 2>(B, w, s);
    default:
        return B.nc == 1 ? batch_autotune_t<Bf16x6Mma, 1>(B, w, s) : batch_autotune_t<Bf16x6Mma, 2>(B, w, s);
    }
}

etd_status etd_batch_tiles(const etd_batch* batch, int instance, int tiles[6]) {
    if (!batch || !tiles) return fail(ETD_EINVAL, "NULL argument");
    const Batch& B = batch->b;
    if (instance < 0 || instance >= int(B.plans.size())) return fail(ETD_EINVAL, "instance out of range");
    for (const BatchGroup& G : B.groups)
        for (int i : G.inst)
            if (i == instance) {
                for (int d = 0; d < 3; ++d) {
                    tiles[2 * d] = d < B.dim ? G.tile[d].rb : 0;
                    tiles[2 * d + 1] = d < B.dim ? G.tile[d].cb : 0;
                }
                return ETD_OK;
            }
    return fail(ETD_EINVAL, "instance not found");
}

etd_status etd_batch_groups(const etd_batch* batch, int* groups) {
    if (!batch || !groups) return fail(ETD_EINVAL, "NULL argument");
    *groups = int(batch->b.groups.size());
    return ETD_OK;
}

etd_status etd_batch_destroy(etd_batch* batch) {
    if (!batch) return ETD_OK;
    Batch& B = batch->b;
    for (BatchGroup& G : B.groups) {
        if (G.stream) (void)hipStreamDestroy(G.stream);
        if (G.done) (void)hipEventDestroy(G.done);
    }
    if (B.fork) (void)hipEventDestroy(B.fork);
    *B.generation = 0;
    delete batch;
    return ETD_OK;
}

etd_status etd_graph_capture(const etd_plan* plan, void* u, double t0, int nsteps, void* ws, void* stream,
                             etd_graph** out) {
    if (!plan || !out || !u) return fail(ETD_EINVAL, "NULL argument");
    *out = nullptr;
    if (!stream) return fail(ETD_EINVAL, "graph capture needs a stream other than the default stream");
    if (nsteps < 1) return fail(ETD_EINVAL, "nsteps must be >= 1");
    if (!std::isfinite(t0)) return fail(ETD_EINVAL, "t0 must be finite");
    etd_status st = check_ws(plan->p, ws);
    if (st != ETD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool timing = plan->timer.on;
    plan->timer.on = false;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed), "graph capture begin");
    char* w = static_cast<char*>(ws);
    switch (plan->p.prob.precision) {
    case ETD_FP64: st = advance_m<NativeMma<double>>(plan->p, plan->timer, u, t0, nsteps, w, s); break;
    case ETD_FP32: st = advance_m<NativeMma<float>>(plan->p, plan->timer, u, t0, nsteps, w, s); break;
    default: st = advance_m<Bf16x6Mma>(plan->p, plan->timer, u, t0, nsteps, w, s);
    }
    plan->timer.on = timing;
    hipGraph_t g;
    st = end_capture(s, st, g);
    if (st != ETD_OK) return st;
    etd_graph* G = new (std::nothrow) etd_graph;
    if (!G) {
        (void)hipGraphDestroy(g);
        return fail(ETD_EINVAL, "out of host memory");
    }
    G->graph = g;
    const hipError_t he = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
    if (he != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete G;
        return hip_fail(he, "graph instantiate");
    }
    *out = G;
    return ETD_OK;
}

etd_status etd_batch_graph_capture(etd_batch* batch, void* const* u, double t0, int nsteps, void* ws, void* stream,
                                   etd_graph** out) {
    if (!batch || !out) return fail(ETD_EINVAL, "NULL argument");
    *out = nullptr;
    if (!stream) return fail(ETD_EINVAL, "graph capture needs a stream other than the default stream");
    if (nsteps < 1) return fail(ETD_EINVAL, "nsteps must be >= 1");
    if (!std::isfinite(t0)) return fail(ETD_EINVAL, "t0 must be finite");
    Batch& B = batch->b;
    etd_status st = batch_check(B, u, nsteps, ws);
    if (st != ETD_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed), "graph capture begin");
    st = batch_dispatch_advance(B, u, t0, nsteps, static_cast<char*>(ws), s);
    hipGraph_t g;
    st = end_capture(s, st, g);
    if (st != ETD_OK) return st;
    etd_graph* G = new (std::nothrow) etd_graph;
    if (!G) {
        (void)hipGraphDestroy(g);
        return fail(ETD_EINVAL, "out of host memory");
    }
    G->graph = g;
    G->generation = B.generation;
    G->captured = *B.generation;
    const hipError_t he = hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0);
    if (he != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete G;
        return hip_fail(he, "graph instantiate");
    }
    *out = G;
    return ETD_OK;
}

etd_status etd_graph_launch(etd_graph* graph, void* stream) {
    if (!graph || !graph->exec) return fail(ETD_EINVAL, "NULL graph");
    if (graph->generation && *graph->generation != graph->captured)
        return fail(ETD_EINVAL, "graph is stale: its batch was re-tuned, re-uploaded or destroyed since capture");
    HIP_TRY(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)), "graph launch");
    return ETD_OK;
}

etd_status etd_graph_destroy(etd_graph* graph) {
    if (!graph) return ETD_OK;
    if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
    if (graph->graph) (void)hipGraphDestroy(graph->graph);
    delete graph;
    return ETD_OK;
}

etd_status etd_compare(const etd_plan* plan, const void* a, const void* b, double out[4], void* ws, void* stream) {
    if (!plan || !a || !b || !out) return fail(ETD_EINVAL, "NULL argument");
    etd_status st = check_ws(plan->p, ws);
    if (st != ETD_OK) return st;
    const Plan& pl = plan->p;
    const long n = long(pl.nc) * pl.n[0] * pl.n[1] * pl.n[2];
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + pl.lay.reduce);
    if (pl.prob.precision == ETD_FP64)
        hipLaunchKernelGGL(compare_partial<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, s,
                           static_cast<const double*>(a), static_cast<const double*>(b), n, part);
    else
        hipLaunchKernelGGL(compare_partial<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, s,
                           static_cast<const float*>(a), static_cast<const float*>(b), n, part);
    HIP_TRY(hipGetLastError(), "compare launch");
    hipLaunchKernelGGL(compare_final, dim3(1), dim3(kRedThreads), 0, s, part, kRedBlocks);
    HIP_TRY(hipGetLastError(), "compare final launch");
    HIP_TRY(hipMemcpyAsync(out, part + kRedBlocks * 4, 4 * sizeof(double), hipMemcpyDeviceToHost, s), "compare copy");
    HIP_TRY(hipStreamSynchronize(s), "compare sync");
    if (out[3] > 0) return fail(ETD_ENONFINITE, "field holds non-finite values");
    return ETD_OK;
}

etd_status etd_plan_table(const etd_plan* plan, int which, int d, int comp, double* out, size_t count) {
    if (!plan || !out) return fail(ETD_EINVAL, "NULL argument");
    const Plan& pl = plan->p;
    if (d < 0 || d >= pl.dim || comp < 0 || comp >= pl.nc) return fail(ETD_EINVAL, "direction or component out of range");
    const std::vector<double>* src = nullptr;
    if (which == 0) src = &pl.lam[d][comp];
    else if (which == 1) src = &pl.P[d];
    else if (which >= 2 && which <= 4) src = &pl.rat[d][comp][which - 2];
    else if (which >= 5 && which <= 7) src = &pl.inc[d][comp][which - 5];
    else return fail(ETD_EINVAL, "unknown table");
    if (count < src->size()) return fail(ETD_EINVAL, "output buffer too small");
    std::memcpy(out, src->data(), src->size() * sizeof(double));
    return ETD_OK;
}

etd_status etd_timing_enable(etd_plan* plan, int enable) {
    if (!plan) return fail(ETD_EINVAL, "NULL plan");
    plan->timer.on = enable != 0;
    plan->timer.used = 0;
    plan->timer.kind.clear();
    return ETD_OK;
}

etd_status etd_timing_read(etd_plan* plan, double ms[3], long long counts[3]) {
    if (!plan || !ms || !counts) return fail(ETD_EINVAL, "NULL argument");
    StageTimer& t = plan->timer;
    for (int k = 0; k < 3; ++k) {
        ms[k] = 0.0;
        counts[k] = 0;
    }
    if (t.used > 0) HIP_TRY(hipEventSynchronize(t.pool[t.used - 1]), "timing sync");
    for (size_t i = 0; i < t.kind.size(); ++i) {
        float dt = 0.0f;
        HIP_TRY(hipEventElapsedTime(&dt, t.pool[2 * i], t.pool[2 * i + 1]), "timing elapsed");
        ms[t.kind[i]] += dt;
        counts[t.kind[i]] += 1;
    }
    t.used = 0;
    t.kind.clear();
    return ETD_OK;
}

etd_status etd_plan_destroy(etd_plan* plan) {
    if (plan)
        for (hipEvent_t e : plan->timer.pool) (void)hipEventDestroy(e);
    delete plan;
    return ETD_OK;
}

const char* etd_status_string(etd_status s) {
    switch (s) {
    case ETD_OK: return "ok";
    case ETD_EINVAL: return "invalid argument";
    case ETD_EUNSUPPORTED: return "unsupported configuration";
    case ETD_EWORKSPACE: return "bad workspace";
    case ETD_EHIP: return "HIP runtime error";
    case ETD_ENONFINITE: return "non-finite values";
    }
    return "unknown status";
}

const char* etd_last_error(void) { return g_err.c_str(); }

}  // extern "C"

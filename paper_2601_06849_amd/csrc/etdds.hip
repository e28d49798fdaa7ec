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

#include <cmath>
#include <cstdio>
#include <cstring>
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

// ---------------------------------------------------------------------------
// Reactions (pointwise source terms of the examples and workloads)
// ---------------------------------------------------------------------------

struct RxnArgs {
    int kind;
    double p[4];
    double ac_rate;        // -lam + kappa * sum_d mu_d + q (AC_MMS)
    double exp_lt;         // e^{-lam t} at the stage's time (AC_MMS)
    const double* sines;   // [3][kMaxPadded] sin(pi (x_i - lo)/L), 0 on the padding
};

// psi of the manufactured Allen-Cahn problem at node (x, y, z).
__device__ __forceinline__ double ac_psi(const RxnArgs& r, int x, int y, int z) {
    const double ue = r.exp_lt * r.sines[x] * r.sines[kMaxPadded + y] * r.sines[2 * kMaxPadded + z];
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
};

// Workgroup: ceil(NP/64) waves; wave w owns output row blocks 4w..4w+3.
// LDS: [2*NC arrays][NP rows][16 + pad] of T, first the inputs, then the
// scaled spectral coefficients.
template <typename T, int NC, bool FIRST>
__global__ __launch_bounds__(256) void outer_stage(OuterArgs a) {
    typedef typename Vec4<T>::type T4;
    constexpr int NA = 2 * NC;
    constexpr int RS = 16 + kOuterRowPad;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* X = reinterpret_cast<T*>(smem_raw);

    const int NP = a.NP;
    const int nrb = NP >> 4;
    const long AST = long(NP) * RS;
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const int cb = blockIdx.x % a.ncb;
    const long bt = blockIdx.x / a.ncb;
    const long gbase = bt * a.sb + long(cb) * 16;
    const T* __restrict__ in0 = static_cast<const T*>(a.in0);
    const T* __restrict__ in1 = static_cast<const T*>(a.in1);
    const T* __restrict__ P = static_cast<const T*>(a.P);

    // ---- stage the tile (and the reaction, for the first stage) ----
    for (int e = tid; e < NP * 16; e += blockDim.x) {
        const int k = e >> 4, j = e & 15;
        const long gi = gbase + long(k) * a.sk + j;
        if constexpr (FIRST) {
            T u[NC], f[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) u[c] = in0[gi + c * a.sc];
            int x, y, z;
            const int col = cb * 16 + j;
            if (a.dim == 3) {
                z = k;
                y = col / a.npx;
                x = col - y * a.npx;
            } else {
                z = 0;
                y = k;
                x = col;
            }
            react<T, NC>(a.rxn, u, f, x, y, z);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                X[c * AST + k * RS + j] = u[c];
                X[(NC + c) * AST + k * RS + j] = f[c];
            }
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                X[c * AST + k * RS + j] = in0[gi + c * a.sc];
                X[(NC + c) * AST + k * RS + j] = in1[gi + c * a.sc];
            }
        }
    }
    __syncthreads();

    const int rb0 = 4 * w;
    T4 acc[4][NA];
    T4 res[4][NA];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            acc[r][q] = T4{0, 0, 0, 0};
            res[r][q] = T4{0, 0, 0, 0};
        }

    // ---- forward product S = P g (all arrays share the A operand) ----
    for (int kb = 0; kb < nrb; ++kb) {
        T4 av[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (rb0 + r < nrb)
                av[r] = *reinterpret_cast<const T4*>(P + long(16 * (rb0 + r) + li) * NP + 16 * kb + 4 * lg);
        T4 bv[NA];
#pragma unroll
        for (int q = 0; q < NA; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) bv[q][e] = X[q * AST + (16 * kb + 4 * lg + e) * RS + li];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (rb0 + r < nrb)
#pragma unroll
                    for (int q = 0; q < NA; ++q) acc[r][q] = mfma4(av[r][e], bv[q][e], acc[r][q]);
    }
    // the inputs at this wave's output rows, for the increment-form epilogue
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (rb0 + r < nrb)
#pragma unroll
            for (int q = 0; q < NA; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    res[r][q][e] = X[q * AST + (16 * (rb0 + r) + acc_row<T>(lg, e)) * RS + li];
    __syncthreads();

    // ---- Hadamard scaling by q1 - 1, coefficients back to LDS ----
    const T* __restrict__ dg = static_cast<const T*>(a.diag);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (rb0 + r < nrb)
#pragma unroll
            for (int q = 0; q < NA; ++q) {
                const T* dc = dg + (q % NC) * a.diag_cstride;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = 16 * (rb0 + r) + acc_row<T>(lg, e);
                    X[q * AST + row * RS + li] = acc[r][q][e] * dc[row];
                }
                acc[r][q] = T4{0, 0, 0, 0};
            }
    __syncthreads();

    // ---- backward product P S and the increment-form epilogue ----
    for (int kb = 0; kb < nrb; ++kb) {
        T4 av[4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (rb0 + r < nrb)
                av[r] = *reinterpret_cast<const T4*>(P + long(16 * (rb0 + r) + li) * NP + 16 * kb + 4 * lg);
        T4 bv[NA];
#pragma unroll
        for (int q = 0; q < NA; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) bv[q][e] = X[q * AST + (16 * kb + 4 * lg + e) * RS + li];
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (rb0 + r < nrb)
#pragma unroll
                    for (int q = 0; q < NA; ++q) acc[r][q] = mfma4(av[r][e], bv[q][e], acc[r][q]);
    }
    T* __restrict__ out0 = static_cast<T*>(a.out0);
    T* __restrict__ out1 = static_cast<T*>(a.out1);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (rb0 + r < nrb)
#pragma unroll
            for (int q = 0; q < NA; ++q) {
                T* o = (q < NC ? out0 : out1) + (q % NC) * a.sc + gbase + li;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = 16 * (rb0 + r) + acc_row<T>(lg, e);
                    o[long(row) * a.sk] = res[r][q][e] + acc[r][q][e];
                }
            }
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
};

// Workgroup: ceil(NP/64) waves over 16 consecutive x-lines.  Wave w owns the
// spectral/physical x rows 64w..64w+63 of every product.  LDS: [2*NC][16
// lines][NP + pad]; arrays 0..NC-1 hold w3 then c then e, arrays NC..2NC-1
// hold w4 then d.
template <typename T, int NC>
__global__ __launch_bounds__(256) void x_stage(XArgs a) {
    typedef typename Vec4<T>::type T4;
    constexpr int NA = 2 * NC;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* R = reinterpret_cast<T*>(smem_raw);

    const int NP = a.NP;
    const int RS = NP + kInnerRowPad;
    const int AST = 16 * RS;
    const int nrb = NP >> 4;
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const long line0 = long(blockIdx.x) * 16;
    const T* __restrict__ w3 = static_cast<const T*>(a.w3);
    const T* __restrict__ w4 = static_cast<const T*>(a.w4);
    const T* __restrict__ P = static_cast<const T*>(a.P);
    const T tau = T(a.tau);

    for (int e = tid; e < 16 * NP; e += blockDim.x) {
        const int j = e / NP, x = e - j * NP;
        const long gi = (line0 + j) * NP + x;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            R[c * AST + j * RS + x] = w3[c * a.sc + gi];
            R[(NC + c) * AST + j * RS + x] = w4[c * a.sc + gi];
        }
    }
    __syncthreads();

    const int rb0 = 4 * w;
    T4 acc[4][NA];
    T4 res[4][NA];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            acc[r][q] = T4{0, 0, 0, 0};
            res[r][q] = T4{0, 0, 0, 0};
        }

    // One contraction: acc[r][q] += P[rows of block rb0+r][:] . B_q, B_q read
    // from LDS array q (lines x positions).
    auto contract = [&](int q0, int nq) {
        for (int kb = 0; kb < nrb; ++kb) {
            T4 av[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (rb0 + r < nrb)
                    av[r] = *reinterpret_cast<const T4*>(P + long(16 * (rb0 + r) + li) * NP + 16 * kb + 4 * lg);
            T4 bv[NA];
#pragma unroll
            for (int q = 0; q < NA; ++q)
                if (q < nq) bv[q] = *reinterpret_cast<const T4*>(R + (q0 + q) * AST + li * RS + 16 * kb + 4 * lg);
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (rb0 + r < nrb)
#pragma unroll
                        for (int q = 0; q < NA; ++q)
                            if (q < nq) acc[r][q] = mfma4(av[r][e], bv[q][e], acc[r][q]);
        }
    };
    // element (line li, x row of accumulator register e) of LDS array q
    auto at = [&](int q, int r, int e) -> T& { return R[q * AST + li * RS + 16 * (rb0 + r) + acc_row<T>(lg, e)]; };

    // ---- b1 = P w3, b2 = P w4 ----
    contract(0, NA);
    // w3, w4 at this wave's x rows, for the increment-form epilogues
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (rb0 + r < nrb)
#pragma unroll
            for (int q = 0; q < NA; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) res[r][q][e] = at(q, r, e);
    __syncthreads();

    const T* __restrict__ dg = static_cast<const T*>(a.diag);
    // ---- c = (q1 - 1) b1 + tau (q2 - 1) b2 into arrays 0..NC-1 ----
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (rb0 + r < nrb)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const T* d1 = dg + c * a.diag_cstride + 16 * (rb0 + r);
                const T* d2 = d1 + a.diag_sstride;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = acc_row<T>(lg, e);
                    at(c, r, e) = d1[k] * acc[r][c][e] + d2[k] * acc[r][NC + c][e];
                }
            }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < NA; ++q) acc[r][q] = T4{0, 0, 0, 0};
    __syncthreads();

    // ---- W = w3 + tau w4 + P c; d = f(W) - w4; V = W + tau d/2 ----
    contract(0, NC);
    T4 V[4][NC];
    const long line = line0 + li;
    const int ly = int(line % a.npy), lz = int(line / a.npy);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (rb0 + r < nrb) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                T Wv[NC], F[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) Wv[c] = res[r][c][e] + tau * res[r][NC + c][e] + acc[r][c][e];
                react<T, NC>(a.rxn, Wv, F, 16 * (rb0 + r) + acc_row<T>(lg, e), ly, lz);
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const T d = F[c] - res[r][NC + c][e];
                    at(NC + c, r, e) = d;
                    V[r][c][e] = Wv[c] + T(0.5) * tau * d;
                }
            }
        }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < NA; ++q) acc[r][q] = T4{0, 0, 0, 0};
    __syncthreads();

    // ---- e = (q3 - 1/2) .* (P d) into arrays 0..NC-1 ----
    contract(NC, NC);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (rb0 + r < nrb)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const T* d3 = dg + c * a.diag_cstride + 2 * a.diag_sstride + 16 * (rb0 + r);
#pragma unroll
                for (int e = 0; e < 4; ++e) at(c, r, e) = d3[acc_row<T>(lg, e)] * acc[r][c][e];
            }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < NA; ++q) acc[r][q] = T4{0, 0, 0, 0};
    __syncthreads();

    // ---- U+ = V + tau P e ----
    contract(0, NC);
    T* __restrict__ out = static_cast<T*>(a.out);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (rb0 + r < nrb)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                T* o = out + c * a.sc + line * NP + 16 * (rb0 + r);
#pragma unroll
                for (int e = 0; e < 4; ++e) o[acc_row<T>(lg, e)] = V[r][c][e] + tau * acc[r][c][e];
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
    r.exp_lt = 0.0;
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
        r.exp_lt = std::exp(-lam * t);
    }
    return r;
}

int waves_for(int NP) { return (NP + 63) / 64; }

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

template <typename T, int NC, bool FIRST>
etd_status launch_outer(const OuterArgs& a, long nblocks, hipStream_t s) {
    const size_t lds = size_t(2 * NC) * a.NP * (16 + kOuterRowPad) * sizeof(T);
    auto k = outer_stage<T, NC, FIRST>;
    static size_t done = 0;
    HIP_TRY(set_lds(k, lds, done), "outer stage LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(nblocks)), dim3(64 * waves_for(a.NP)), lds, s, a);
    HIP_TRY(hipGetLastError(), "outer stage launch");
    return ETD_OK;
}

template <typename T, int NC>
etd_status launch_x(const XArgs& a, long nblocks, hipStream_t s) {
    const size_t lds = size_t(2 * NC) * 16 * (a.NP + kInnerRowPad) * sizeof(T);
    auto k = x_stage<T, NC>;
    static size_t done = 0;
    HIP_TRY(set_lds(k, lds, done), "x stage LDS attribute");
    hipLaunchKernelGGL(k, dim3(unsigned(nblocks)), dim3(64 * waves_for(a.NP)), lds, s, a);
    HIP_TRY(hipGetLastError(), "x stage launch");
    return ETD_OK;
}

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

template <typename T, int NC>
etd_status run_steps(const Plan& pl, StageTimer& tm, char* ws, double t0, int nsteps, hipStream_t s) {
    const int px = pl.np[0], py = pl.np[1], pz = pl.np[2];
    const long sc = long(px) * py * pz;
    T* U = reinterpret_cast<T*>(ws + pl.lay.field[0]);
    T* WA = reinterpret_cast<T*>(ws + pl.lay.field[1]);
    T* WB = reinterpret_cast<T*>(ws + pl.lay.field[2]);
    T* WC = reinterpret_cast<T*>(ws + pl.lay.field[3]);
    T* WD = reinterpret_cast<T*>(ws + pl.lay.field[4]);
    const T* diag = reinterpret_cast<const T*>(ws + pl.lay.diag);
    const long dstride = long(pl.diag_stride);
    const long dcs = long(kDiagSlots) * dstride;
    const double tau = pl.prob.tau;

    for (int step = 0; step < nsteps; ++step) {
        const double tn = t0 + step * tau;
        const double tn1 = t0 + (step + 1) * tau;
        OuterArgs o{};
        o.diag_cstride = dcs;
        o.sc = sc;
        o.npx = px;
        o.npy = py;
        o.dim = pl.dim;
        o.rxn = rxn_args(pl, ws, tn);
        const T* w3;
        const T* w4;
        if (pl.dim == 3) {
            // z stage: contracted index z (stride px*py), columns (y, x)
            o.in0 = U;
            o.in1 = nullptr;
            o.out0 = WA;
            o.out1 = WB;
            o.P = ws + pl.lay.P[2];
            o.diag = diag + long(kDiagZ) * dstride;
            o.NP = pz;
            o.ncb = px * py / 16;
            o.sk = long(px) * py;
            o.sb = 0;
            TIMED(0, (launch_outer<T, NC, true>(o, o.ncb, s)));
            // y stage: contracted index y (stride px), columns x, batches z
            o.in0 = WA;
            o.in1 = WB;
            o.out0 = WC;
            o.out1 = WD;
            o.P = ws + pl.lay.P[1];
            o.diag = diag + long(kDiagY) * dstride;
            o.NP = py;
            o.ncb = px / 16;
            o.sk = px;
            o.sb = long(px) * py;
            TIMED(1, (launch_outer<T, NC, false>(o, long(o.ncb) * pz, s)));
            w3 = WC;
            w4 = WD;
        } else {
            o.in0 = U;
            o.in1 = nullptr;
            o.out0 = WA;
            o.out1 = WB;
            o.P = ws + pl.lay.P[1];
            o.diag = diag + long(kDiagY) * dstride;
            o.NP = py;
            o.ncb = px / 16;
            o.sk = px;
            o.sb = 0;
            TIMED(0, (launch_outer<T, NC, true>(o, o.ncb, s)));
            w3 = WA;
            w4 = WB;
        }
        XArgs x{};
        x.w3 = w3;
        x.w4 = w4;
        x.out = U;
        x.P = ws + pl.lay.P[0];
        x.diag = diag + long(kDiagX1) * dstride;
        x.diag_sstride = dstride;
        x.diag_cstride = dcs;
        x.NP = px;
        x.sc = sc;
        x.npy = py;
        x.tau = tau;
        x.rxn = rxn_args(pl, ws, tn1);
        TIMED(2, (launch_x<T, NC>(x, long(py) * pz / 16, s)));
    }
    return ETD_OK;
}

template <typename T>
etd_status advance_t(const Plan& pl, StageTimer& tm, void* u, double t0, int nsteps, char* ws, hipStream_t s) {
    const Dims d = dims_of(pl);
    T* U = reinterpret_cast<T*>(ws + pl.lay.field[0]);
    hipLaunchKernelGGL(pack_field<T>, dim3(2048), dim3(256), 0, s, static_cast<const T*>(u), U, d);
    HIP_TRY(hipGetLastError(), "pack launch");
    etd_status st = pl.nc == 1 ? run_steps<T, 1>(pl, tm, ws, t0, nsteps, s) : run_steps<T, 2>(pl, tm, ws, t0, nsteps, s);
    if (st != ETD_OK) return st;
    hipLaunchKernelGGL(unpack_field<T>, dim3(2048), dim3(256), 0, s, U, static_cast<T*>(u), d);
    HIP_TRY(hipGetLastError(), "unpack launch");
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
    if (prob->precision == ETD_BF16X6) {
        delete p;
        return fail(ETD_EUNSUPPORTED, "the split-BF16 mode-product kernels are not built in this version");
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
    if (plan->p.prob.precision == ETD_FP64) return advance_t<double>(plan->p, plan->timer, u, t0, nsteps, w, s);
    return advance_t<float>(plan->p, plan->timer, u, t0, nsteps, w, s);
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

// Forward stage kernels: the fused outer and x stages, the product-parallel
// 2-D path, the grouped (batched) launches and the split two-component x stage.
//
// Part of libetdds: included, in order, by library.hpp (each translation
// unit that includes it holds its own copy); internal linkage throughout.
#pragma once

namespace {

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
// threadIdx.x behind an empty asm statement.  Inside a persistent loop the
// tile functions then recompute their per-thread addressing for every tile
// instead of having it hoisted out of the loop and held in vector registers
// for the whole launch (which makes the 1024-thread tiles spill).
__device__ __forceinline__ int tile_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// One thread's share of an outer tile's global inputs: ITER 16-byte vectors
// of each loaded array (the workgroup has exactly 4 NP / RB threads).
// Stage inputs are read once per stage, so their loads carry the
// non-temporal hint and L2 favours P, which every tile reads again.  (The
// scattered element stores of the outputs keep the default policy: with the
// hint their partial lines reach HBM separately.)
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
    const int tid = tile_tid();
#pragma unroll
    for (int i = 0; i < OuterRegs<M, NC, FIRST, RB, CB>::ITER; ++i) {
        const int v = tid + i * blockDim.x;
        if (v >= nvec) break;
        const int k = v / VPR, j0 = (v - k * VPR) * VN;
        const long gi = gbase + long(k) * a.sk + j0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            g.v[i][c] = __builtin_nontemporal_load(reinterpret_cast<const TV*>(in0 + gi + c * a.sc));
            if constexpr (!FIRST) g.v[i][NC + c] = __builtin_nontemporal_load(reinterpret_cast<const TV*>(in1 + gi + c * a.sc));
        }
        if constexpr (FIRST && NC == 1)
            if (a.other) g.other[i] = __builtin_nontemporal_load(reinterpret_cast<const TV*>(static_cast<const T*>(a.other) + gi));
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
    const int tid = tile_tid();
#pragma unroll
    for (int i = 0; i < OuterRegs<M, NC, FIRST, RB, CB>::ITER; ++i) {
        const int v = tid + i * blockDim.x;
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
    typedef typename M::acc AT;                 // accumulator type of the products
    typedef typename Vec4<AT>::type A4;
    constexpr int NCOL = 16 * CB;         // columns per tile
    constexpr int NA = 2 * NC;
    constexpr int NQ = NA * CB;           // B fragments per K block
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* X = reinterpret_cast<T*>(smem_raw);

    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));     // LDS stride between columns
    const int AST = NCOL * RS;
    const int tid = tile_tid();
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
    A4 acc[RB][NQ];
    T4 res[RB][NQ];
    zero<AT, RB, NQ>(acc);

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
    zero<AT, RB, NQ>(acc);
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
    const int tid = tile_tid();
#pragma unroll
    for (int i = 0; i < XRegs<M, NC, RB, CB>::ITER; ++i) {
        const int v = tid + i * blockDim.x;
        if (v >= nvec) break;
        const long gi = base + long(v) * VN;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            g.v[i][c] = __builtin_nontemporal_load(reinterpret_cast<const TV*>(w3 + c * a.sc + gi));
            g.v[i][NC + c] = __builtin_nontemporal_load(reinterpret_cast<const TV*>(w4 + c * a.sc + gi));
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
    const int tid = tile_tid();
#pragma unroll
    for (int i = 0; i < XRegs<M, NC, RB, CB>::ITER; ++i) {
        const int v = tid + i * blockDim.x;
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
    typedef typename M::acc AT;                 // accumulator type of the products
    typedef typename Vec4<AT>::type A4;
    constexpr int NA = 2 * NC;
    constexpr int NL = 16 * CB;           // lines per tile
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* R = reinterpret_cast<T*>(smem_raw);

    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int AST = NL * RS;
    const int tid = tile_tid();
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
        A4 acc[RB][NA * CB];
        zero<AT, RB, NA * CB>(acc);
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
    A4 acc[RB][NC * CB];
    zero<AT, RB, NC * CB>(acc);
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
    zero<AT, RB, NC * CB>(acc);
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
    zero<AT, RB, NC * CB>(acc);
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

// x stage of one component over long lines whose two-array tile exceeds the
// LDS: ONE array of 16*CB lines, so twice the lines of the two-array tile and
// half the reads of P per line.  The first phase takes P w3 and P w4 in two
// passes (w4 restaged over w3); the epilogue reads w3 and w4 at the wave's
// rows from memory (the lines were just staged, so from L2), and V = W +
// tau d/2 waits in the output lines.  Otherwise the same operations in the
// same order as x_compute.
template <typename M, int RB, int CB>
__device__ __forceinline__ void x_tile_one_array(const XArgs& a, long tile) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    typedef typename M::acc AT;
    typedef typename Vec4<AT>::type A4;
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    constexpr int NL = 16 * CB;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* R = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int RS = NP + 16 / int(sizeof(T));
    const int tid = tile_tid();
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    const long line0 = tile * NL;
    const void* __restrict__ P = a.P;
    const T tau = T(a.tau);
    const int rb0 = RB * w;
    const T* __restrict__ w3 = static_cast<const T*>(a.w3);
    const T* __restrict__ w4 = static_cast<const T*>(a.w4);
    const T* __restrict__ dg = static_cast<const T*>(a.diag);
    auto stage = [&](const T* __restrict__ f) {
        const int vpl = NP / VN;
        for (int v = tid; v < NL * vpl; v += blockDim.x) {
            const int j = v / vpl, x = (v - j * vpl) * VN;
            *reinterpret_cast<TV*>(R + j * RS + x) =
                __builtin_nontemporal_load(reinterpret_cast<const TV*>(f + line0 * NP + long(v) * VN));
        }
    };
    auto bfrag = [&](int qq, int k0) { return lds_vec<T, M::KL>(R + (li + 16 * qq) * RS + k0); };
    auto at = [&](int cb, int r, int e) -> T& { return R[(li + 16 * cb) * RS + 16 * (rb0 + r) + M::row(lg, e)]; };

    // ---- b1 = P w3, b2 = P w4 (two passes over the one array) ----
    stage(w3);
    __syncthreads();
    A4 b1[RB][CB];
    zero<AT, RB, CB>(b1);
    gemm<M, RB, CB>(P, NP, rb0, li, lg, b1, bfrag);
    __syncthreads();
    stage(w4);
    __syncthreads();
    A4 acc[RB][CB];
    zero<AT, RB, CB>(acc);
    gemm<M, RB, CB>(P, NP, rb0, li, lg, acc, bfrag);
    __syncthreads();
    // ---- c = (q1 - 1) b1 + tau (q2 - 1) b2 ----
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const T* d1 = dg + 16 * (rb0 + r);
        const T* d2 = d1 + a.diag_sstride;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = M::row(lg, e);
                at(cb, r, e) = d1[k] * b1[r][cb][e] + d2[k] * acc[r][cb][e];
            }
    }
    __syncthreads();

    // ---- W = w3 + tau w4 + P c; d = f(W) - w4; V = W + tau d/2 ----
    zero<AT, RB, CB>(acc);
    gemm<M, RB, CB>(P, NP, rb0, li, lg, acc, bfrag);
    __syncthreads();   // every wave has read c
    // V = W + tau d/2 goes to the output lines (this tile's own) until the
    // last product adds tau P e to it: registers are what limits this tile
    T* __restrict__ out = static_cast<T*>(a.out);
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const long line = line0 + li + 16 * cb;
        const int ly = int(line % a.npy), lz = int(line / a.npy);
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int x = 16 * (rb0 + r) + M::row(lg, e);
                const T w3v = w3[line * NP + x], w4v = w4[line * NP + x];
                T Wv[1], F[1];
                Wv[0] = w3v + tau * w4v + acc[r][cb][e];
                react<T, 1>(a.rxn, Wv, F, x, ly, lz);
                if (a.Wout) static_cast<T*>(a.Wout)[line * NP + x] = Wv[0];
                const T d = F[0] - w4v;
                at(cb, r, e) = d;
                out[line * NP + x] = Wv[0] + T(0.5) * tau * d;
            }
    }
    zero<AT, RB, CB>(acc);
    __syncthreads();

    // ---- e = (q3 - 1/2) .* (P d) ----
    gemm<M, RB, CB>(P, NP, rb0, li, lg, acc, bfrag);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const T* d3 = dg + 2 * a.diag_sstride + 16 * (rb0 + r);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int e = 0; e < 4; ++e) at(cb, r, e) = d3[M::row(lg, e)] * acc[r][cb][e];
    }
    zero<AT, RB, CB>(acc);
    __syncthreads();

    // ---- U+ = V + tau P e ----
    gemm<M, RB, CB>(P, NP, rb0, li, lg, acc, bfrag);
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const long line = line0 + li + 16 * cb;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            T* o = out + line * NP + 16 * (rb0 + r);
#pragma unroll
            for (int e = 0; e < 4; ++e) o[M::row(lg, e)] = o[M::row(lg, e)] + tau * acc[r][cb][e];
        }
    }
}

// Tiles of eight row blocks per wave over two line blocks (FP32 states, one
// component) hold one array: x_tile_one_array.
template <typename M, int NC, int RB, int CB>
constexpr bool x_one_array() {
    return NC == 1 && RB == 8 && CB == 2 && sizeof(typename M::elem) == 4;
}

template <typename M, int NC, int RB, int CB>
__device__ __forceinline__ void x_tile(const XArgs& a, long tile) {
    if constexpr (x_one_array<M, NC, RB, CB>()) {
        x_tile_one_array<M, RB, CB>(a, tile);
    } else {
        XRegs<M, NC, RB, CB> g;
        x_load<M, NC, RB, CB>(a, tile, g);
        x_store<M, NC, RB, CB>(a, g);
        __syncthreads();
        x_compute<M, NC, RB, CB>(a, tile);
    }
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
// computed with the fused stages' operations in the same order, up to how the
// compiler fuses a few epilogue multiply-adds (FP64 results are bitwise those
// of the fused kernels; two-component FP32 ones differ by ~1e-7 relative).
// The y stage takes two launches, the x stage four:
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

// Row group and column tile of workgroup L of a product-parallel launch
// (nrg row groups x T / nrg column tiles, T workgroups).  The dispatcher deals
// consecutive workgroups to the eight XCDs in turn (XCD = L % 8), and every
// row group of a column tile stages the same B panel, so each XCD takes a
// contiguous run of column tiles with all their row groups: the panel comes
// from HBM once and from that XCD's L2 for the other row groups.
__device__ __forceinline__ void split_block(int nrg, int T, int L, int& rg, int& ct) {
    int t = L;
    if (T % 8 == 0) t = (L % 8) * (T / 8) + L / 8;
    rg = t % nrg;
    ct = t / nrg;
}

// Every array of the launch is staged at once, K chunk by K chunk: the B
// panel (16 columns x NP contracted indices per array) streams through two
// LDS buffers of BK indices, the next chunk's loads in flight (in registers)
// while the matrix cores work on the current one.  Each P fragment feeds
// NARR MFMAs per step.  The contraction is split in KS parts over as many
// wave groups (each its own buffers), so a SIMD holds KS waves whose loads
// and MFMAs interleave; the parts are summed in LDS, in a fixed order, and
// the first group runs the epilogue.
template <int KIND, int NC>
struct SplitShape {
    static constexpr int NARR = (KIND <= kSplitX1) ? 2 * NC : NC;   // B arrays of the product
    // arrays read from memory to form them (YF forms f(U) from U while staging)
    static constexpr int NRAW = (KIND == kSplitYF) ? NC : NARR;
};

// LDS of a launch: KS x two buffers of narr arrays x 16 columns x (bk + pad)
inline size_t split_lds_bytes(int narr, int bk, int ks, size_t elem) {
    return size_t(ks) * 2 * size_t(narr) * 16 * (bk + 16 / elem) * elem;
}

// BK contracted indices per chunk; KS * BK divides the padded extent NP, so
// every chunk is whole and inside the field.
template <typename M, int NC, int KIND, int NW, int BK, int KS>
__global__ __launch_bounds__(64 * NW * KS) void split_product(SplitArgs a) {
    typedef typename M::elem T;
    typedef typename Vec4<T>::type T4;
    typedef typename M::acc AT;                 // accumulator type of the products
    typedef typename Vec4<AT>::type A4;
    constexpr bool YK = KIND <= kSplitYB;   // contracted direction y, columns are x
    constexpr int NARR = SplitShape<KIND, NC>::NARR;
    constexpr int NRAW = SplitShape<KIND, NC>::NRAW;
    static_assert(BK % M::KB == 0, "chunks hold whole K blocks");
    constexpr int RSK = BK + 16 / int(sizeof(T));   // LDS stride between columns
    constexpr int AST = 16 * RSK;                   // between arrays
    constexpr int BST = NARR * AST;                 // between the two buffers of a part
    constexpr int GT = 64 * NW;                     // threads of one part's wave group
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* X = reinterpret_cast<T*>(smem_raw);
    const int NP = a.NP;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int kh = w / NW;                          // contraction part of this wave
    const int ptid = tid - kh * GT;                 // thread index within the part
    const int lane = tid & 63;
    const int li = lane & 15, lg = lane >> 4;
    int rg, ct;
    split_block(a.NP / (16 * NW), int(gridDim.x), int(blockIdx.x), rg, ct);
    const int rb0 = rg * NW + (w - kh * NW);   // this wave's 16-row block
    const int col0 = ct * 16;
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

    // Staging moves 16-byte chunks of VN elements: VN consecutive columns of
    // one contracted index k (y kinds, x contiguous) or VN consecutive k of
    // one line (x kinds).  Every padded extent is a multiple of VN and every
    // field is 256-byte aligned, so each chunk is one aligned vector load.
    typedef typename Vec16<T>::type TV;
    constexpr int VN = Vec16<T>::n;
    constexpr int NV = 16 * BK / VN;                // vectors per array and K chunk
    constexpr int PER = (NV + GT - 1) / GT;         // per thread
    auto vec_at = [&](int v, int& k, int& c) {      // vector v of a chunk -> (k within it, column)
        if constexpr (YK) {
            k = v / (16 / VN);
            c = (v % (16 / VN)) * VN;
        } else {
            c = v / (BK / VN);
            k = (v % (BK / VN)) * VN;
        }
    };
    auto raw_ptr = [&](int q) -> const T* {
        if constexpr (KIND == kSplitYF) return U + q * sc;
        else if constexpr (KIND == kSplitYB) return q < NC ? WC + q * sc : WD + (q - NC) * sc;
        else if constexpr (KIND == kSplitX1) return q < NC ? WA + q * sc : WB + (q - NC) * sc;
        else if constexpr (KIND == kSplitX3) return WD + q * sc;
        else return WC + q * sc;
    };
    const int nch = NP / (BK * KS);                 // chunks per part
    const int kbase = kh * nch * BK;                // first contracted index of this part
    T* const mybuf = X + kh * 2 * BST;
    TV pre[PER][NRAW];
    auto load_chunk = [&](int ch) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int v = ptid + j * GT;
            if (NV % GT == 0 || v < NV) {
                int k, c;
                vec_at(v, k, c);
                const long gi = at(kbase + ch * BK + k, c);
#pragma unroll
                for (int q = 0; q < NRAW; ++q) pre[j][q] = *reinterpret_cast<const TV*>(raw_ptr(q) + gi);
            }
        }
    };
    auto store_chunk = [&](int ch) {
        T* buf = mybuf + (ch & 1) * BST;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int v = ptid + j * GT;
            if (NV % GT == 0 || v < NV) {
                int k, c;
                vec_at(v, k, c);
                TV val[NARR];
#pragma unroll
                for (int q = 0; q < NRAW; ++q) val[q] = pre[j][q];
                if constexpr (KIND == kSplitYF) {
#pragma unroll
                    for (int e = 0; e < VN; ++e) {
                        T uj[NC], f[NC];
#pragma unroll
                        for (int cc = 0; cc < NC; ++cc) uj[cc] = pre[j][cc][e];
                        int x, y;
                        coords(kbase + ch * BK + k, c + e, x, y);
                        react<T, NC>(a.rxn, uj, f, x, y, 0);
#pragma unroll
                        for (int cc = 0; cc < NC; ++cc) val[NC + cc][e] = f[cc];
                    }
                }
#pragma unroll
                for (int q = 0; q < NARR; ++q) {
                    T* dst = buf + q * AST + c * RSK + k;
                    if constexpr (YK) {
#pragma unroll
                        for (int e = 0; e < VN; ++e) dst[e * RSK] = val[q][e];
                    } else {
                        *reinterpret_cast<TV*>(dst) = val[q];
                    }
                }
            }
        }
    };
    load_chunk(0);
    store_chunk(0);
    if (nch > 1) load_chunk(1);
    A4 acc[1][NARR];
    zero<AT, 1, NARR>(acc);
    const int nkbp = nch * (BK / M::KB);            // K blocks per part
    // P fragments are requested four K blocks ahead
    gemm_chunked<M, 1, NARR, 4, BK / M::KB>(
        a.P, NP, kh * nkbp, (kh + 1) * nkbp, rb0, li, lg, acc,
        [&](int q, int k0) {
            const int ch = (k0 - kbase) / BK;
            return lds_vec<T, M::KL>(mybuf + (ch & 1) * BST + q * AST + li * RSK + (k0 - kbase - ch * BK));
        },
        [&](int ch) {
            __syncthreads();   // chunk ch is in LDS; chunk ch - 1's buffer is free
            if (ch + 1 < nch) store_chunk(ch + 1);
            if (ch + 2 < nch) load_chunk(ch + 2);
        });
    if constexpr (KS > 1) {
        // sum the parts in order: part p > 0 leaves its accumulators in LDS
        // (lane-major), part 0 adds them and runs the epilogue
        __syncthreads();
        AT* red = reinterpret_cast<AT*>(smem_raw);
        const int wr = w - kh * NW;
        if (kh > 0) {
#pragma unroll
            for (int q = 0; q < NARR; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    red[(((kh - 1) * NW + wr) * NARR * 4 + q * 4 + e) * 64 + lane] = acc[0][q][e];
        }
        __syncthreads();
        if (kh > 0) return;
#pragma unroll
        for (int p = 1; p < KS; ++p)
#pragma unroll
            for (int q = 0; q < NARR; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[0][q][e] += red[(((p - 1) * NW + wr) * NARR * 4 + q * 4 + e) * 64 + lane];
    }
    // result of array q at register e
    auto res = [&](int q, int e) { return acc[0][q][e]; };

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

// The descriptor table is read-only for the whole launch and every address
// into it is uniform over the workgroup: read through the constant address
// space it is fetched with scalar loads, and an instance's arguments then sit
// in scalar registers, as a plain launch's kernel arguments do, instead of
// taking vector registers from the tile body.
template <typename X>
__device__ __forceinline__ const __attribute__((address_space(4))) X* as_constant(const X* p) {
    return (const __attribute__((address_space(4))) X*)(p);
}

// A trivially copyable struct read word by word through the constant space.
template <typename X>
__device__ __forceinline__ X load_constant(const X* p) {
    static_assert(std::is_trivially_copyable<X>::value && sizeof(X) % 4 == 0, "word-wise copy");
    X out;
    const auto src = as_constant(reinterpret_cast<const unsigned*>(p));
    unsigned* dst = reinterpret_cast<unsigned*>(&out);
#pragma unroll
    for (unsigned k = 0; k < sizeof(X) / 4; ++k) dst[k] = src[k];
    return out;
}

template <typename A>
__device__ __forceinline__ int group_instance(const Group<A>& g, long tile) {
    const auto start = as_constant(g.start);
    int lo = 0, hi = g.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= tile) lo = mid;
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
        OuterArgs a = load_constant(g.args + i);
        group_time(a.rxn, g.t0, g.k);
        outer_tile<M, NC, FIRST, RB, CB>(a, t - as_constant(g.start)[i]);
        __syncthreads();   // the next tile restages the LDS
    }
}

template <typename M, int NC, int RB, int CB, int MAXT>
__global__ __launch_bounds__(MAXT) void x_group(Group<XArgs> g) {
    for (long t = blockIdx.x; t < g.ntiles; t += gridDim.x) {
        const int i = group_instance(g, t);
        XArgs a = load_constant(g.args + i);
        group_time(a.rxn, g.t0, g.k);
        x_tile<M, NC, RB, CB>(a, t - as_constant(g.start)[i]);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Resident schedule for small grids: every step of a run in ONE cooperative
// launch.  Each stage is the same tile body as its own launch (one row block
// per wave, one column or line block per tile), the workgroups take the
// stage's tiles in turn, and a grid-wide barrier separates the stages, whose
// release and acquire make each stage's outputs visible to the next.  A small
// grid spends most of a launched step in launch and drain; here the fields
// stay in the L2 and the MALL between stages.  Co-residency of the grid is
// what the cooperative launch guarantees, so every barrier completes.
// ---------------------------------------------------------------------------

struct ResidentArgs {
    OuterArgs outer[2];   // z then y (3-D), y (2-D)
    long otiles[2];       // tiles of each outer stage
    XArgs x;
    long xtiles;          // tiles of the x stage
    int nouter;
    int nsteps;
    double t0;
};

template <typename M, int NC, int MAXT>
__global__ __launch_bounds__(MAXT) void resident_steps(ResidentArgs a) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    for (int s = 0; s < a.nsteps; ++s) {
        for (int k = 0; k < a.nouter; ++k) {
            OuterArgs o = a.outer[k];
            group_time(o.rxn, a.t0, s);
            for (long t = blockIdx.x; t < a.otiles[k]; t += gridDim.x) {
                if (k == 0) outer_tile<M, NC, true, 1, 1>(o, t);
                else outer_tile<M, NC, false, 1, 1>(o, t);
                __syncthreads();   // the next tile restages the LDS
            }
            grid.sync();
        }
        XArgs x = a.x;
        group_time(x.rxn, a.t0, s + 1);
        for (long t = blockIdx.x; t < a.xtiles; t += gridDim.x) {
            x_tile<M, NC, 1, 1>(x, t);
            __syncthreads();
        }
        grid.sync();
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
    typedef typename M::acc AT;                 // accumulator type of the products
    typedef typename Vec4<AT>::type A4;
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
        A4 acc[RB][2];
        zero<AT, RB, 2>(acc);
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
    A4 acc[RB][1];
    zero<AT, RB, 1>(acc);
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
    typedef typename M::acc AT;                 // accumulator type of the products
    typedef typename Vec4<AT>::type A4;
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
    A4 acc[RB][1];
    zero<AT, RB, 1>(acc);
    gemm<M, RB, 1>(P, NP, rb0, li, lg, acc, bfrag_from(0));
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) at(1, r, e) = d3[16 * (rb0 + r) + M::row(lg, e)] * acc[r][0][e];
    zero<AT, RB, 1>(acc);
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

}  // namespace

// The K-loop of one mode-product tile on the matrix cores.
//
// Part of libetdds: included, in order, by library.hpp (each translation
// unit that includes it holds its own copy); internal linkage throughout.
#pragma once

namespace {

// ---------------------------------------------------------------------------
// Shared pieces of the stage kernels
// ---------------------------------------------------------------------------

// acc[r][q] += P[16(rb0+r) .. +16][:] . B_q over the whole contracted length
// NP (a multiple of M::KB).  The A operand comes straight from P in global
// memory (L2-resident; M::a_off / a_kstep give a lane's first fragment and the
// step to the next K block: row-major P, or a fragment-ordered copy)
// and is held in a ring of PF register buffers, so each K block's fragment is
// requested PF blocks before its use (launches with one wave per SIMD need a
// deeper ring to cover the L2 latency, and there FP64 B fragments are read
// from LDS one K block ahead as well).  With PF = 1 the compiler folds the
// ring into loads at the top of each K block (the generated code waits for a
// block's fragments as the block starts); the other waves on the SIMD cover
// that latency, and keeping the loads a block ahead with a compiler memory
// barrier measured slower in most stages, as the held fragments cost
// registers.  bload(q, k0) returns the KL values of B fragment q for
// contracted indices k0 .. k0+KL of this lane's column.
template <typename M, int RB, int NQ, int PF = 1, typename BL>
__device__ __forceinline__ void gemm(const void* __restrict__ P, int NP, int rb0, int li, int lg,
                                     vec_t<typename M::acc, 4> (&acc)[RB][NQ], BL bload) {
    const int nkb = NP / M::KB;
    const long kstep = M::a_kstep(NP);
    long off[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) off[r] = M::a_off(NP, rb0 + r, li, lg);
    // ring[i] holds K block kb + i (addresses clamp to the last block)
    typename M::A ring[PF][RB];
#pragma unroll
    for (int i = 0; i < PF; ++i)
#pragma unroll
        for (int r = 0; r < RB; ++r) ring[i][r] = M::load_a(P, NP, off[r] + min(i, nkb - 1) * kstep);
    // with a ring (PF > 1) FP64 B fragments are also read one K block ahead
    // (measured: 2% on the FP64 2-D kernels; FP32 fragments gain nothing)
    constexpr bool BNEXT = PF > 1 && !M::SPLIT_B && sizeof(typename M::elem) == 8;
    typename M::B bnext[NQ];
    if constexpr (BNEXT) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) bnext[q] = M::prep(bload(q, M::KL * lg));
    }
    for (int kb0 = 0; kb0 < nkb; kb0 += PF) {
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int kb = kb0 + i;
            if (PF > 1 && kb >= nkb) break;
            typename M::A a_cur[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) a_cur[r] = ring[i][r];
            const long kn = min(kb + PF, nkb - 1) * kstep;
#pragma unroll
            for (int r = 0; r < RB; ++r) ring[i][r] = M::load_a(P, NP, off[r] + kn);
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
                if constexpr (BNEXT) {
                    const int kbn = min(kb + 1, nkb - 1) * M::KB + M::KL * lg;
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        b[q] = bnext[q];
                        bnext[q] = M::prep(bload(q, kbn));
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < NQ; ++q) b[q] = M::prep(bload(q, kb * M::KB + M::KL * lg));
                }
#pragma unroll
                for (int t = 0; t < M::NSUB; ++t)
#pragma unroll
                    for (int r = 0; r < RB; ++r)
#pragma unroll
                        for (int q = 0; q < NQ; ++q) M::step(acc[r][q], a_cur[r], b[q], t);
            }
        }
    }
}

// The same K-loop over K blocks kb_lo .. kb_hi - 1 of a B operand that is
// streamed through LDS in chunks of CKB K blocks: at_chunk(c) runs
// (uniformly across the workgroup) before the first K block of the range's
// chunk c and must leave that chunk readable by bload.  The A ring runs on
// across chunk boundaries, so P keeps arriving PF K blocks ahead while a
// chunk is exchanged.
template <typename M, int RB, int NQ, int PF, int CKB, typename BL, typename CH>
__device__ __forceinline__ void gemm_chunked(const void* __restrict__ P, int NP, int kb_lo, int kb_hi, int rb0,
                                             int li, int lg, vec_t<typename M::acc, 4> (&acc)[RB][NQ], BL bload,
                                             CH at_chunk) {
    const long kstep = M::a_kstep(NP);
    long off[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) off[r] = M::a_off(NP, rb0 + r, li, lg);
    typename M::A ring[PF][RB];
#pragma unroll
    for (int i = 0; i < PF; ++i)
#pragma unroll
        for (int r = 0; r < RB; ++r) ring[i][r] = M::load_a(P, NP, off[r] + min(kb_lo + i, kb_hi - 1) * kstep);
    for (int kb0 = kb_lo; kb0 < kb_hi; kb0 += PF) {
#pragma unroll
        for (int i = 0; i < PF; ++i) {
            const int kb = kb0 + i;
            if (kb >= kb_hi) break;
            if ((kb - kb_lo) % CKB == 0) at_chunk((kb - kb_lo) / CKB);
            typename M::A a_cur[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) a_cur[r] = ring[i][r];
            const long kn = min(kb + PF, kb_hi - 1) * kstep;
#pragma unroll
            for (int r = 0; r < RB; ++r) ring[i][r] = M::load_a(P, NP, off[r] + kn);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const typename M::B b = M::prep(bload(q, kb * M::KB + M::KL * lg));
#pragma unroll
                for (int t = 0; t < M::NSUB; ++t)
#pragma unroll
                    for (int r = 0; r < RB; ++r) M::step(acc[r][q], a_cur[r], b, t);
            }
        }
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

}  // namespace

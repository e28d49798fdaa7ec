// The per-precision entry table: the host drivers of one matrix-core policy,
// dispatched on the component count.
//
// Part of libetdds: included, in order, by library.hpp (each translation
// unit that includes it holds its own copy); internal linkage throughout.
#pragma once

namespace {

template <typename M>
etd_status op_advance(const Plan& pl, StageTimer& tm, void* u, double t0, int nsteps, char* ws, hipStream_t s) {
    return advance_m<M>(pl, tm, u, t0, nsteps, ws, s);
}

template <typename M>
etd_status op_adjoint(const Plan& pl, StageTimer& tm, const void* u0, double t0, int nsteps, int segment,
                      const void* ubarN, void* ubar0, double* grad, char* ws, char* aws, hipStream_t s) {
    const AdjLayout L = adjoint_layout(pl, nsteps, segment);
    return pl.nc == 1 ? adjoint_t<M, 1>(pl, tm, u0, t0, nsteps, ubarN, ubar0, grad, ws, aws, L, s)
                      : adjoint_t<M, 2>(pl, tm, u0, t0, nsteps, ubarN, ubar0, grad, ws, aws, L, s);
}

template <typename M>
etd_status op_autotune(Plan& pl, char* ws, hipStream_t s) {
    return pl.nc == 1 ? autotune_plan_t<M, 1>(pl, ws, s) : autotune_plan_t<M, 2>(pl, ws, s);
}

template <typename M>
etd_status op_resolve_tile(const Plan& pl, int d, TileShape t, TileShape& out, long copies) {
    return pl.nc == 1 ? resolve_tile<M, 1>(pl, d, t, out, copies) : resolve_tile<M, 2>(pl, d, t, out, copies);
}

template <typename M>
etd_status op_batch_advance(Batch& B, void* const* u, double t0, int nsteps, char* ws, hipStream_t s) {
    return B.nc == 1 ? batch_advance_t<M, 1>(B, u, t0, nsteps, ws, s) : batch_advance_t<M, 2>(B, u, t0, nsteps, ws, s);
}

template <typename M>
etd_status op_batch_autotune(Batch& B, char* ws, hipStream_t s) {
    return B.nc == 1 ? batch_autotune_t<M, 1>(B, ws, s) : batch_autotune_t<M, 2>(B, ws, s);
}

template <typename M>
PrecisionOps make_ops() {
    PrecisionOps o;
    o.advance = op_advance<M>;
    o.adjoint = op_adjoint<M>;
    o.autotune = op_autotune<M>;
    o.resolve_tile = op_resolve_tile<M>;
    o.batch_advance = op_batch_advance<M>;
    o.batch_autotune = op_batch_autotune<M>;
    return o;
}

}  // namespace

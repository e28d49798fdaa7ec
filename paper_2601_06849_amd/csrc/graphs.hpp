// HIP graph capture helpers.
//
// Part of libetdds: included, in order, by library.hpp (each translation
// unit that includes it holds its own copy); internal linkage throughout.
#pragma once

namespace {

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

// Types shared by the translation units of libetdds: the per-thread error
// message, the stage timer, tile shapes, batches, and the table of entry
// functions that each precision's translation unit instantiates.
//
// The library is built from one translation unit per mode-product precision
// (kern_<precision>.hip: every kernel and host driver instantiated for that
// matrix-core policy) plus etdds.hip (the C ABI).  Everything else in the
// kernel headers has internal linkage, so each unit holds its own copy.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "etdds.h"
#include "plan.hpp"

namespace etdds {

// Message of the most recent failure on this thread (defined in etdds.hip).
extern thread_local std::string g_err;

// Optional per-stage timing: HIP events recorded on the caller's stream
// around every stage launch (diagnostics; not thread-safe).
struct StageTimer {
    bool on = false;
    std::vector<hipEvent_t> pool;    // reusable events
    size_t used = 0;                 // events recorded since the last read
    std::vector<int> kind;           // stage kind of interval i = (ev[2i], ev[2i+1])
};

// Tile shape of a stage launch: `rb` 16-row blocks of each product per wave
// and `cb` 16-column (outer stages) or 16-line (x stage) blocks per tile.
struct TileShape {
    int rb = 0, cb = 0;   // rb == 0: use the default
};

// Batches: instances of one padded shape form a group.
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
    std::vector<size_t> base;         // workspace offset of each instance's region (its plan layout's 0)
    std::vector<size_t> skip;         // leading table bytes the instance neither holds nor uploads
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

// The precision-specific work of the C ABI, instantiated once per
// mode-product precision (each entry dispatches on the component count).
struct PrecisionOps {
    // etd_advance: pack, nsteps steps, unpack (ws: the uploaded workspace)
    etd_status (*advance)(const Plan& pl, StageTimer& tm, void* u, double t0, int nsteps, char* ws, hipStream_t s);
    // etd_adjoint (aws: the adjoint workspace of adjoint_layout(pl, nsteps, segment))
    etd_status (*adjoint)(const Plan& pl, StageTimer& tm, const void* u0, double t0, int nsteps, int segment,
                          const void* ubar_final, void* ubar0, double* grad, char* ws, char* aws, hipStream_t s);
    etd_status (*autotune)(Plan& pl, char* ws, hipStream_t s);
    // validate a tile request for direction d ((0, 0): the default shape for
    // `copies` instances sharing each launch)
    etd_status (*resolve_tile)(const Plan& pl, int d, TileShape t, TileShape& out, long copies);
    etd_status (*batch_advance)(Batch& B, void* const* u, double t0, int nsteps, char* ws, hipStream_t s);
    etd_status (*batch_autotune)(Batch& B, char* ws, hipStream_t s);
};

const PrecisionOps& ops_fp64();
const PrecisionOps& ops_fp32();
const PrecisionOps& ops_bf16x6();
const PrecisionOps& ops_fp64_fp32();
const PrecisionOps& ops_fp64_bf16x6();

}  // namespace etdds

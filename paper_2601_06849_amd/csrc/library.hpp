// Every kernel header of libetdds, in dependency order: common (errors,
// matrix-core policies), reactions, gemm (the K-loop), stages (forward
// kernels), adjoint_kernels, field_kernels (pack/unpack, reductions), launch
// (tile shapes, launchers, step drivers), adjoint (checkpointed reverse sweep),
// autotune, batch, graphs, and ops (the per-precision entry table).
//
// Included by each translation unit of the library; templates are
// instantiated only where a unit uses them (kern_<precision>.hip).
#pragma once

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "etdds.h"
#include "plan.hpp"
#include "types.hpp"

using namespace etdds;

#include "common.hpp"
#include "reactions.hpp"
#include "gemm.hpp"
#include "stages.hpp"
#include "adjoint_kernels.hpp"
#include "field_kernels.hpp"
#include "launch.hpp"
#include "adjoint.hpp"
#include "autotune.hpp"
#include "batch.hpp"
#include "graphs.hpp"
#include "ops.hpp"

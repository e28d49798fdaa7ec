// Host-side plan of the spectral ETD2RK-DS stepper: closed-form eigenpairs of
// the 1-D operators, rational factors in FP64, and the workspace layout.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "etdds.h"

namespace etdds {

// Granularity of the padded grid: every direction is padded with zeros to a
// multiple of 32 (one BF16 MFMA K-step; two FP64/FP32 16-row tiles), or of 64
// beyond 512 points.
constexpr int kPad = 32;
// Largest padded direction the stage kernels support.
constexpr int kMaxPadded = 1024;
// LDS budget of one stage workgroup (bytes) and its largest wave count.
constexpr size_t kMaxLds = 160 * 1024;
constexpr int kMaxWaves = 16;
// Row padding of the LDS tiles: 16 bytes (2 FP64 or 4 FP32 elements), which
// keeps rows 16-byte aligned and makes the row stride 4 banks modulo 64, so
// neither the 16-byte B-fragment reads of 8 lanes nor the element accesses of
// 16 lanes (one column each) share a bank.
inline int row_pad(size_t elem) { return int(16 / elem); }

// LDS footprint of an outer-stage tile (`arrays` fields of 16*cb columns,
// each a run of NP contracted indices plus padding) and of an x-stage tile
// (`arrays` fields of 16*cb lines x NP, plus padding).
inline size_t outer_lds_bytes(int NP, int arrays, int cb, size_t elem) {
    return size_t(arrays) * 16 * cb * (NP + row_pad(elem)) * elem;
}
inline size_t x_lds_bytes(int NP, int arrays, int cb, size_t elem) {
    return size_t(arrays) * 16 * cb * (NP + row_pad(elem)) * elem;
}
// 16-row blocks per wave: a tile needs NP / (16 * rows_per_wave) waves.
inline int rows_per_wave(int NP) { return NP <= 512 ? 2 : 4; }
// Both components of a system share one tile when it fits in LDS; otherwise
// each component is processed alone (the reaction reads the other one from
// memory) and the x stage is split in two kernels around W.
inline bool outer_fused(int NP, int nc, size_t elem) { return outer_lds_bytes(NP, 2 * nc, 1, elem) <= kMaxLds; }
inline bool x_fused(int NP, int nc, size_t elem) { return x_lds_bytes(NP, 2 * nc, 1, elem) <= kMaxLds; }

// Bytes of a state element (fields, tiles, diagonals) and the format of the
// eigenvector tables, per mode-product precision.
inline size_t state_bytes(int precision) {
    return (precision == ETD_FP32 || precision == ETD_BF16X6) ? 4 : 8;
}
inline bool split_bf16(int precision) { return precision == ETD_BF16X6 || precision == ETD_FP64_BF16X6; }
// bytes per entry of a P table that is not split (FP64 products: 8, FP32: 4)
inline size_t p_bytes(int precision) { return precision == ETD_FP64 ? 8 : 4; }

struct Layout {
    size_t P[3];        // eigenvector matrices (NP x NP, row-major; BF16X6: hi, mid, lo)
    size_t P_bytes[3];
    size_t diag;        // increment-form rational factors, see DiagSlot
    size_t diag_bytes;
    size_t sines;       // FP64 sin(pi (x_i - lo)/L) per direction (AC_MMS forcing)
    size_t grad;        // FP64 derivative weights of the adjoint, see GradSlot
    size_t field[5];    // padded fields: U, WA, WB, WC, WD
    size_t field_bytes;
    size_t reduce;      // FP64 partial sums of etd_compare
    size_t total;
};

// Slots of the per-component diagonal table (each NP[d] long, working type).
enum DiagSlot {
    kDiagZ = 0,   // Q1(tau lambda_z) - 1
    kDiagY = 1,   // Q1(tau lambda_y) - 1
    kDiagX1 = 2,  // Q1(tau lambda_x) - 1
    kDiagX2 = 3,  // tau (Q2(tau lambda_x) - 1)
    kDiagX3 = 4,  // Q3(tau lambda_x) - 1/2
    kDiagSlots = 5
};

// Slots of the FP64 derivative-weight table [component][direction][slot][kMaxPadded]
// used by the adjoint's parameter gradients: d Q_l(tau lambda)/d lambda times
// the factor with which Q_l enters the step, and d lambda / d kappa.
enum GradSlot {
    kGradRho1 = 0,  // tau Q1'(tau lambda)
    kGradRho2 = 1,  // tau * tau Q2'(tau lambda)   (x only)
    kGradRho3 = 2,  // tau * tau Q3'(tau lambda)   (x only)
    kGradMu = 3,    // d lambda / d kappa = (4/h^2) sin^2(...)
    kGradSlots = 4
};

struct Plan {
    etd_problem prob;
    int dim = 0, nc = 0;
    int n[3] = {1, 1, 1};
    int np[3] = {1, 1, 1};
    size_t elem = 8;                        // bytes per state element
    // FP64 host tables
    std::vector<double> lam[3][2];          // eigenvalues of A_d (kappa_c applied)
    std::vector<double> P[3];               // n_d x n_d eigenvector matrix
    std::vector<double> rat[3][2][3];       // Q_l(tau lambda_j), l = 1..3
    std::vector<double> inc[3][2][3];       // Q_1 - 1, Q_2 - 1, Q_3 - 1/2 at tau lambda_j
    Layout lay{};
    std::vector<uint8_t> image;             // host image of the table region
    size_t table_bytes = 0;                 // bytes of image (start of workspace)
    size_t diag_stride = 0;                 // elements between diag slots (max NP)
    // stage tile shape per direction (rows per wave, column/line blocks);
    // 0 = the built-in default, else set by the autotuner or the caller
    int tile_rb[3] = {0, 0, 0};
    int tile_cb[3] = {0, 0, 0};
    int schedule = 0;                       // etd_schedule of etd_advance (0: AUTO)
};

etd_status build_plan(const etd_problem& p, Plan& out, std::string& err);

}  // namespace etdds

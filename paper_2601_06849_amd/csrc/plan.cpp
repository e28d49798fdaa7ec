// Plan construction for the spectral ETD2RK-DS stepper (host, FP64).
//
// Steps 1-2 of Algorithms 1-2 (Sec. 3.4): the eigendecomposition of every
// 1-D operator and the Hadamard factors of the rational functions.  The
// matrices of Sec. 2.1, A_d = h_d^-2 tridiag(-kappa, 2 kappa + q h_d^2/dim,
// -kappa), are the scaled second-difference matrix plus a multiple of I, so
// their eigenvectors are the discrete sine vectors and the eigendecomposition
// is taken in closed form:
//   P_d[i][j] = sqrt(2/(n+1)) sin(pi (i+1)(j+1)/(n+1))   (symmetric, P_d^2 = I)
//   lambda_j  = kappa (4/h^2) sin^2((j+1) pi / (2(n+1))) + q/dim.
// Only the operator P diag(.) P^T is unique; this choice of P (sign, order)
// makes it symmetric and orthogonal, so the forward and backward products use
// the same matrix.
//
// The complex partial fractions of Sec. 3.1 are needed only to form the
// Hadamard factors (Remark 1): 2 Re(r_l/(z - s)) equals the real rational
// function, evaluated here directly.  The stepper uses the increment form
// Q(z) = Q(0) + (Q(z) - Q(0)), so the factors are stored as Q1 - 1,
// tau (Q2 - 1) and Q3 - 1/2, each written with a factor z taken out (rational
// families) or from expm1 and Taylor series (exact exponentials) so that no
// cancellation occurs as tau*lambda -> 0.
#include "plan.hpp"

#include <cmath>
#include <cstring>
#include <sstream>

namespace etdds {

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Exact-exponential family (the fully discrete scheme of Sec. 2.2 before any
// Pade approximation): Q_1 = e^{-z}, Q_2 = phi_1(z) = (1 - e^{-z})/z,
// Q_3 = phi_2(z) = (z - 1 + e^{-z})/z^2.  The closed forms of phi_1 - 1 and
// phi_2 - 1/2 cancel as z -> 0, so below z = 2 they are summed from their
// Taylor series sum_{k>=1} (-z)^k/(k+1)! and sum_{k>=1} (-z)^k/(k+2)!
// (alternating, terms decreasing; 28 terms reach 1e-24 at z = 2), and e^{-z} - 1
// comes from expm1.  Derivatives likewise.
constexpr int kSeriesTerms = 28;

void exact_family(double z, double out[3], double inc[3]) {
    const double em1 = std::expm1(-z);    // e^{-z} - 1
    inc[0] = em1;
    if (z < 2.0) {
        double t = 1.0, f1 = 1.0, f2 = 2.0, s1 = 0.0, s2 = 0.0;   // t = (-z)^k, f1 = (k+1)!, f2 = (k+2)!
        for (int k = 1; k <= kSeriesTerms; ++k) {
            t *= -z;
            f1 *= double(k + 1);
            f2 *= double(k + 2);
            s1 += t / f1;
            s2 += t / f2;
        }
        inc[1] = s1;
        inc[2] = s2;
    } else {
        inc[1] = (-em1 - z) / z;
        inc[2] = (z + em1) / (z * z) - 0.5;
    }
    out[0] = 1.0 + em1;
    out[1] = 1.0 + inc[1];
    out[2] = 0.5 + inc[2];
}

void exact_family_derivative(double z, double dq[3]) {
    const double em1 = std::expm1(-z);
    dq[0] = -(1.0 + em1);
    if (z < 2.0) {
        // d/dz sum (-z)^k/(k+m)! = sum_{k>=1} -k (-z)^(k-1)/(k+m)!
        double t = 1.0, f1 = 1.0, f2 = 2.0, s1 = 0.0, s2 = 0.0;   // t = (-z)^(k-1)
        for (int k = 1; k <= kSeriesTerms; ++k) {
            f1 *= double(k + 1);
            f2 *= double(k + 2);
            s1 -= double(k) * t / f1;
            s2 -= double(k) * t / f2;
            t *= -z;
        }
        dq[1] = s1;
        dq[2] = s2;
    } else {
        dq[1] = (z * (1.0 + em1) + em1) / (z * z);
        dq[2] = -em1 / (z * z) - 2.0 * (z + em1) / (z * z * z);
    }
}

// Derivatives Q_l'(z) of the rational factors (quotient rule on the
// polynomial forms below).
void rational_derivative(int pade, double z, double dq[3]) {
    if (pade == 0) {
        exact_family_derivative(z, dq);
        return;
    }
    if (pade == 4) {
        const double den = (((z + 4.0) * z + 12.0) * z + 24.0) * z + 24.0;
        const double dden = ((4.0 * z + 12.0) * z + 24.0) * z + 24.0;
        const double n2 = ((z + 4.0) * z + 12.0) * z + 24.0, dn2 = (3.0 * z + 8.0) * z + 12.0;
        const double n3 = ((z + 3.0) * z + 8.0) * z + 12.0, dn3 = (3.0 * z + 6.0) * z + 8.0;
        const double d2 = den * den;
        dq[0] = -24.0 * dden / d2;
        dq[1] = (dn2 * den - n2 * dden) / d2;
        dq[2] = (dn3 * den - n3 * dden) / d2;
    } else {
        const double D = (z + 2.0) * z + 2.0, dD = 2.0 * z + 2.0, D2 = D * D;
        dq[0] = -2.0 * dD / D2;
        dq[1] = -((z + 4.0) * z + 2.0) / D2;
        dq[2] = -(z + 2.0) * z / D2;
    }
}

// Factors at z = tau*lambda >= 0 (rational families, or the exact
// exponentials for pade = 0).  out[0..2] = Q_1..Q_3 and inc[0..2] = Q_1 - 1,
// Q_2 - 1, Q_3 - 1/2.
void rational(int pade, double z, double out[3], double inc[3]) {
    if (pade == 0) {
        exact_family(z, out, inc);
        return;
    }
    if (pade == 4) {
        // P_{0,4} family (Sec. 5): R_1 = 24/den, R_2 = (z^3+4z^2+12z+24)/den,
        // R_3 = (z^3+3z^2+8z+12)/den, den = z^4+4z^3+12z^2+24z+24.
        const double den = (((z + 4.0) * z + 12.0) * z + 24.0) * z + 24.0;
        const double n2 = ((z + 4.0) * z + 12.0) * z + 24.0;
        const double n3 = ((z + 3.0) * z + 8.0) * z + 12.0;
        out[0] = 24.0 / den;
        out[1] = n2 / den;
        out[2] = n3 / den;
        inc[0] = -z * n2 / den;
        inc[1] = -z * n3 / den;
        inc[2] = -z * (((z + 2.0) * z + 6.0) * z + 8.0) / (2.0 * den);
    } else {
        // P_{0,2} family (Sec. 3.1): Q_1 = 2/D, Q_2 = (z+2)/D, Q_3 = (z+1)/D,
        // D = z^2 + 2z + 2.
        const double D = (z + 2.0) * z + 2.0;
        out[0] = 2.0 / D;
        out[1] = (z + 2.0) / D;
        out[2] = (z + 1.0) / D;
        inc[0] = -z * (z + 2.0) / D;
        inc[1] = -z * (z + 1.0) / D;
        inc[2] = -z * z / (2.0 * D);
    }
}

// Round-to-nearest-even conversion to bfloat16 (upper 16 bits of binary32).
uint16_t to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return uint16_t(u >> 16);
}

double from_bf16(uint16_t h) {
    const uint32_t u = uint32_t(h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return double(f);
}

template <typename T>
void put(std::vector<uint8_t>& img, size_t off, size_t idx, T v) {
    std::memcpy(img.data() + off + idx * sizeof(T), &v, sizeof(T));
}

}  // namespace

etd_status build_plan(const etd_problem& p, Plan& pl, std::string& err) {
    std::ostringstream msg;
    auto bad = [&](const char* what) {
        err = what;
        return ETD_EINVAL;
    };
    if (p.dim != 2 && p.dim != 3) return bad("dim must be 2 or 3");
    if (p.ncomp != 1 && p.ncomp != 2) return bad("ncomp must be 1 or 2");
    const bool two = p.rxn == ETD_RXN_FHN_CUBIC || p.rxn == ETD_RXN_FHN_CLASSIC;
    if (p.rxn < ETD_RXN_NONE || p.rxn > ETD_RXN_FHN_CLASSIC) return bad("unknown reaction");
    if (two != (p.ncomp == 2)) return bad("ncomp must be 2 exactly for the FitzHugh-Nagumo reactions");
    if (p.pade != 0 && p.pade != 2 && p.pade != 4) return bad("pade must be 0 (exact exponentials), 2 or 4");
    if (p.precision < ETD_FP64 || p.precision > ETD_FP64_BF16X6) return bad("unknown precision");
    if (!(p.tau > 0.0) || !std::isfinite(p.tau)) return bad("tau must be a finite positive number");
    if (!(p.q >= 0.0) || !std::isfinite(p.q)) return bad("q must be finite and >= 0");
    for (int c = 0; c < p.ncomp; ++c)
        if (!(p.kappa[c] >= 0.0) || !std::isfinite(p.kappa[c])) return bad("kappa must be finite and >= 0");
    for (int i = 0; i < 8; ++i)
        if (!std::isfinite(p.rxn_param[i])) return bad("reaction parameters must be finite");
    for (int d = 0; d < p.dim; ++d) {
        if (p.n[d] < 1) return bad("n must be >= 1 in every direction");
        if (!(p.hi[d] > p.lo[d]) || !std::isfinite(p.hi[d] - p.lo[d])) return bad("box must have hi > lo");
    }

    pl.prob = p;
    pl.dim = p.dim;
    pl.nc = p.ncomp;
    for (int d = 0; d < 3; ++d) {
        pl.n[d] = d < p.dim ? p.n[d] : 1;
        // multiples of 32; beyond 512 of 64 (four 16-row blocks per wave)
        pl.np[d] = d < p.dim ? round_up(pl.n[d], kPad) : 1;
        if (pl.np[d] > 512) pl.np[d] = round_up(pl.n[d], 2 * kPad);
    }
    for (int d = 0; d < p.dim; ++d)
        if (pl.np[d] > kMaxPadded) {
            msg << "padded direction " << d << " has " << pl.np[d] << " points; the stage kernels take at most "
                << kMaxPadded;
            err = msg.str();
            return ETD_EUNSUPPORTED;
        }
    pl.elem = state_bytes(p.precision);
    for (int d = 0; d < p.dim; ++d) {
        // one component's tile (the split path) must fit; two waves' rows per 16
        const int NP = pl.np[d];
        const bool fits = d == 0 ? x_lds_bytes(NP, 2, 1, pl.elem) <= kMaxLds
                                 : outer_lds_bytes(NP, 2, 1, pl.elem) <= kMaxLds;
        if (!fits || NP / (16 * rows_per_wave(NP)) > kMaxWaves) {
            msg << "padded direction " << d << " (" << NP << " points) exceeds the on-chip tile limits at this precision";
            err = msg.str();
            return ETD_EUNSUPPORTED;
        }
    }

    // ---- FP64 tables -------------------------------------------------------
    for (int d = 0; d < p.dim; ++d) {
        const int n = pl.n[d];
        const double h = (p.hi[d] - p.lo[d]) / (n + 1);
        pl.P[d].assign(size_t(n) * n, 0.0);
        const double s = std::sqrt(2.0 / (n + 1));
        const long period = 2L * (n + 1);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const long arg = (long(i + 1) * long(j + 1)) % period;  // exact argument reduction
                pl.P[d][size_t(i) * n + j] = s * std::sin(M_PI * double(arg) / double(n + 1));
            }
        for (int c = 0; c < pl.nc; ++c) {
            pl.lam[d][c].resize(n);
            for (int l = 0; l < 3; ++l) {
                pl.rat[d][c][l].resize(n);
                pl.inc[d][c][l].resize(n);
            }
            for (int j = 0; j < n; ++j) {
                const double sn = std::sin((j + 1) * M_PI / (2.0 * (n + 1)));
                const double lam = p.kappa[c] * 4.0 / (h * h) * sn * sn + p.q / p.dim;
                pl.lam[d][c][j] = lam;
                double q[3], inc[3];
                rational(p.pade, p.tau * lam, q, inc);
                for (int l = 0; l < 3; ++l) {
                    pl.rat[d][c][l][j] = q[l];
                    pl.inc[d][c][l][j] = inc[l];
                }
            }
        }
    }

    // ---- workspace layout ----------------------------------------------------
    Layout& L = pl.lay;
    size_t off = 0;
    const bool bf = split_bf16(p.precision);
    for (int d = 0; d < 3; ++d) {
        if (d < p.dim) {
            const size_t nn = size_t(pl.np[d]) * pl.np[d];
            L.P[d] = off;
            L.P_bytes[d] = bf ? 3 * nn * 2 : nn * p_bytes(p.precision);
            off = align256(off + L.P_bytes[d]);
        } else {
            L.P[d] = 0;
            L.P_bytes[d] = 0;
        }
    }
    pl.diag_stride = size_t(kMaxPadded);
    const size_t diag_elem = pl.elem;
    L.diag = off;
    L.diag_bytes = size_t(pl.nc) * kDiagSlots * pl.diag_stride * diag_elem;
    off = align256(off + L.diag_bytes);
    L.sines = off;
    off = align256(off + 3 * size_t(kMaxPadded) * 8);
    L.grad = off;
    off = align256(off + size_t(pl.nc) * 3 * kGradSlots * kMaxPadded * 8);
    pl.table_bytes = off;
    L.field_bytes = align256(size_t(pl.nc) * pl.np[0] * pl.np[1] * pl.np[2] * pl.elem);
    for (int f = 0; f < 5; ++f) {
        L.field[f] = off;
        off += L.field_bytes;
    }
    L.reduce = off;
    off = align256(off + 2048 * 4 * 8);
    L.total = off;

    // ---- host image of the tables -------------------------------------------
    pl.image.assign(pl.table_bytes, 0);
    for (int d = 0; d < p.dim; ++d) {
        const int n = pl.n[d], NP = pl.np[d];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double v = pl.P[d][size_t(i) * n + j];
                const size_t idx = size_t(i) * NP + j;
                if (!bf && p_bytes(p.precision) == 8) {
                    put<double>(pl.image, L.P[d], idx, v);
                } else if (!bf) {
                    put<float>(pl.image, L.P[d], idx, float(v));
                } else {
                    const uint16_t hi = to_bf16(float(v));
                    const double r1 = v - from_bf16(hi);
                    const uint16_t mid = to_bf16(float(r1));
                    const double r2 = r1 - from_bf16(mid);
                    const uint16_t lo = to_bf16(float(r2));
                    // fragment order of the split-BF16 A operand: chunk (row
                    // block i/16, K block j/32) of 3 planes x 64 lanes x 8
                    // values, lane (i%16) + 16 ((j%32)/8), value j%8
                    const size_t chunk = (size_t(i / 16) * (NP / 32) + size_t(j / 32)) * (3 * 64 * 8);
                    const size_t lane = size_t(i % 16) + 16 * size_t((j % 32) / 8);
                    const size_t at = chunk + lane * 8 + size_t(j % 8);
                    put<uint16_t>(pl.image, L.P[d], at, hi);
                    put<uint16_t>(pl.image, L.P[d], at + 512, mid);
                    put<uint16_t>(pl.image, L.P[d], at + 1024, lo);
                }
            }
    }
    // Diagonal slots: outer directions (z, y) use Q1 - 1; x uses all three.
    for (int c = 0; c < pl.nc; ++c) {
        for (int slot = 0; slot < kDiagSlots; ++slot) {
            int d;
            if (slot == kDiagZ) d = 2;
            else if (slot == kDiagY) d = 1;
            else d = 0;
            if (d >= p.dim) continue;
            for (int j = 0; j < pl.n[d]; ++j) {
                double q[3], inc[3];
                rational(p.pade, p.tau * pl.lam[d][c][j], q, inc);
                double v;
                if (slot == kDiagZ || slot == kDiagY || slot == kDiagX1) v = inc[0];
                else if (slot == kDiagX2) v = p.tau * inc[1];
                else v = inc[2];
                const size_t idx = (size_t(c) * kDiagSlots + slot) * pl.diag_stride + j;
                if (pl.elem == 8) put<double>(pl.image, L.diag, idx, v);
                else put<float>(pl.image, L.diag, idx, float(v));
            }
        }
    }
    // Sine factors of the manufactured solution (zero on the padding).
    for (int d = 0; d < p.dim; ++d) {
        const double Ld = p.hi[d] - p.lo[d];
        const double h = Ld / (pl.n[d] + 1);
        for (int i = 0; i < pl.n[d]; ++i)
            put<double>(pl.image, L.sines, size_t(d) * kMaxPadded + i, std::sin(M_PI * (i + 1) * h / Ld));
    }
    if (p.dim == 2)
        for (int i = 0; i < kMaxPadded; ++i) put<double>(pl.image, L.sines, 2 * size_t(kMaxPadded) + i, i == 0 ? 1.0 : 0.0);
    // Derivative weights of the adjoint (zero on the padding).
    for (int c = 0; c < pl.nc; ++c)
        for (int d = 0; d < p.dim; ++d) {
            const double h = (p.hi[d] - p.lo[d]) / (pl.n[d] + 1);
            for (int j = 0; j < pl.n[d]; ++j) {
                double dq[3];
                rational_derivative(p.pade, p.tau * pl.lam[d][c][j], dq);
                const double sn = std::sin((j + 1) * M_PI / (2.0 * (pl.n[d] + 1)));
                const size_t base = ((size_t(c) * 3 + d) * kGradSlots) * kMaxPadded + j;
                put<double>(pl.image, L.grad, base + kGradRho1 * kMaxPadded, p.tau * dq[0]);
                put<double>(pl.image, L.grad, base + kGradRho2 * kMaxPadded, p.tau * p.tau * dq[1]);
                put<double>(pl.image, L.grad, base + kGradRho3 * kMaxPadded, p.tau * p.tau * dq[2]);
                put<double>(pl.image, L.grad, base + kGradMu * kMaxPadded, 4.0 / (h * h) * sn * sn);
            }
        }
    return ETD_OK;
}

}  // namespace etdds

// Layout conversion (pack/unpack) and the validation reductions.
//
// Part of libetdds: included, in order, by library.hpp (each translation
// unit that includes it holds its own copy); internal linkage throughout.
#pragma once

namespace {

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

// Per-block partial sums in a fixed order: [sum (a-b)^2, sum b^2, max|a-b|,
// #nonfinite(a)]; the difference terms skip the entries where a is not
// finite, sum b^2 takes every entry.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void compare_partial(const T* __restrict__ a, const T* __restrict__ b,
                                                               long n, double* __restrict__ part) {
    __shared__ double sh[4][kRedThreads];
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (long i = blockIdx.x * long(kRedThreads) + threadIdx.x; i < n; i += long(gridDim.x) * kRedThreads) {
        const double av = double(a[i]), bv = double(b[i]);
        s1 += bv * bv;   // ||b|| over every entry, whatever a holds
        if (!isfinite(av)) {
            s3 += 1.0;
            continue;
        }
        const double df = av - bv;
        s0 += df * df;
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

// Reduce the nblocks per-block partials (fixed order) into res[0..3] =
// [||a-b||_2, ||b||_2, max|a-b|, #nonfinite(a)].
__global__ __launch_bounds__(kRedThreads) void compare_final(const double* __restrict__ part, int nblocks,
                                                             double* __restrict__ res) {
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
        res[0] = sqrt(sh[0][0]);
        res[1] = sqrt(sh[1][0]);
        res[2] = sh[2][0];
        res[3] = sh[3][0];
    }
}

}  // namespace

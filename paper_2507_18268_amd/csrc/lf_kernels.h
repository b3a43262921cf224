// Device helpers shared by the cell-parallel kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "lf_problem.h"

namespace lf {

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8).  Remap so that XCD x owns the contiguous logical range
// [x*G/8, (x+1)*G/8): neighbouring cells (and on box meshes the +-n and +-n^2
// neighbours) are then read through the same XCD's L2.
__device__ __forceinline__ int32_t logical_block() {
    const int32_t g = static_cast<int32_t>(gridDim.x);
    const int32_t b = static_cast<int32_t>(blockIdx.x);
    if (g >= kNumXcd && (g % kNumXcd) == 0) return (b % kNumXcd) * (g / kNumXcd) + b / kNumXcd;
    return b;
}

struct CellRange {
    int32_t begin, end;
};

__device__ __forceinline__ CellRange cell_range(int32_t n, int32_t chunk, int32_t L) {
    int64_t b = static_cast<int64_t>(L) * chunk;
    int64_t e = b + chunk;
    if (e > n) e = n;
    if (b > n) b = n;
    return {static_cast<int32_t>(b), static_cast<int32_t>(e)};
}

// Sum over a wavefront of 64 lanes by xor butterflies; every lane ends with the
// same value because each pairwise sum is commutative.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of NQ values over the workgroup, result in every thread; fixed order.
template <int NQ>
__device__ __forceinline__ void block_sum(double (&v)[NQ]) {
    constexpr int kWaves = kBlock / 64;
    __shared__ double red[NQ][kWaves];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) v[q] = wave_sum(v[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) red[q][wv] = v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = red[q][0];
#pragma unroll
        for (int j = 1; j < kWaves; ++j) s += red[q][j];
        v[q] = s;
    }
    __syncthreads();
}

// Second stage of a two-stage reduction: every workgroup sums the G per-
// workgroup partials of each slot in the same fixed order.
template <int NQ>
__device__ __forceinline__ void reduce_partials(const double *__restrict__ part, const int (&slot)[NQ],
                                                int32_t G, double (&out)[NQ]) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = 0.0;
        for (int32_t i = threadIdx.x; i < G; i += kBlock) s += part[slot[q] * kMaxGrid + i];
        out[q] = s;
    }
    block_sum<NQ>(out);
}

template <int NQ>
__device__ __forceinline__ void write_partials(double *__restrict__ part, const int (&slot)[NQ],
                                               double (&v)[NQ], int32_t L) {
    block_sum<NQ>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) part[slot[q] * kMaxGrid + L] = v[q];
    }
}

// Snapshot of the solver state taken by one thread and shared through LDS, so
// every thread of a workgroup acts on the same values even while workgroup 0
// of the same kernel updates the state.
struct StateView {
    int32_t done, n_iter, converged;
    double nf, res0, wArA_cur, wArA_prev;
};

__device__ __forceinline__ StateView load_state(const PcgState *st) {
    __shared__ StateView sv;
    if (threadIdx.x == 0) {
        StateView v;
        v.done = st->done;
        v.n_iter = st->n_iter;
        v.converged = st->converged;
        v.nf = st->nf;
        v.res0 = st->res0;
        v.wArA_cur = st->wArA_cur;
        v.wArA_prev = st->wArA_slot[(v.n_iter - 1) & 1];
        sv = v;
    }
    __syncthreads();
    StateView v = sv;
    __syncthreads();
    return v;
}

__device__ __forceinline__ bool check_conv(double res, double res0, double tol, double rel_tol) {
    return (res < tol) || (rel_tol > 1e-20 && res < rel_tol * res0);
}

}  // namespace lf

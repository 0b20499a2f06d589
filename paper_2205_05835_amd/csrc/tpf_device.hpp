// Device-side helpers shared by the stage and pressure kernels: periodic
// indexing on the [z][y][x] cell grid, the pointwise laws of the method and
// the deterministic block reductions.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "tpf_index.hpp"

namespace tpf {

// Physical parameters as the kernels consume them.
struct Phys {
    int model, force, clamp;
    double h, inv_h, sigma, sigma_hat, eps, gamma, rho1, rho2, visc1, visc2, delta2;
};

enum { MODEL_CDI = 0, MODEL_SB = 1, MODEL_ISODI = 2 };
enum { FORCE_EB = 0, FORCE_CSF = 1, FORCE_LCSF = 2 };

__device__ __forceinline__ bool block_tile(int xcd, int gx, int gy, int gz, int& bx, int& by, int& bz) {
    return tile_coords(tile_of_block(xcd, (int)gridDim.x, (int)blockIdx.x), gx, gy, gz, bx, by, bz);
}

// the cell of this thread for a (BX x BY x 1) tiling of the grid; W: with
// the wall bits of d.walls (kernels instantiated for boxes with walls; the
// periodic instantiations carry none, so their wall tests fold away)
template <bool W = false>
__device__ __forceinline__ bool cell_of_thread(const Dims& d, Cell& C) {
    int bx, by, bz;
    if (!block_tile(d.xcd, (d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, d.nz, bx, by, bz)) return false;
    const int i = bx * BX + threadIdx.x;
    const int j = by * BY + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return false;
    C = W ? make_cell_w(d, i, j, bz) : make_cell(d, i, j, bz);
    return true;
}

// z-chunked tiling of the stage kernels: the grid has ceil(nz / kz) tiles in
// z and the block of tile (bx, by, kc) handles its BX x BY cells in planes
// kc kz ... kc kz + kz - 1, bottom to top.  The z neighbours one plane reads
// are read again by the same block in the next plane shortly after, so they
// come from L2 instead of HBM.
template <bool W = false, typename F>
__device__ __forceinline__ void for_cells_zchunk(const Dims& d, int kz, F&& body) {
    int bx, by, bz;
    if (!block_tile(d.xcd, (d.nx + BX - 1) / BX, (d.ny + BY - 1) / BY, (d.nz + kz - 1) / kz, bx, by, bz))
        return;
    const int i = bx * BX + threadIdx.x;
    const int j = by * BY + threadIdx.y;
    if (i >= d.nx || j >= d.ny) return;
    const int k0 = bz * kz, k1 = min(d.nz, k0 + kz);
    for (int k = k0; k < k1; ++k) body(W ? make_cell_w(d, i, j, k) : make_cell(d, i, j, k));
}

// Loads and stores at a 32-bit element index: the byte offset is formed in
// 32 bits (grids below 2^29 cells for FP64 fields, 2^30 for FP32), so the
// access compiles to a scalar base address plus one 32-bit vector offset
// instead of a 64-bit address per lane.
template <typename T>
__device__ __forceinline__ T ld(const T* base, unsigned idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (unsigned)(idx * (unsigned)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void st(T* base, unsigned idx, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (unsigned)(idx * (unsigned)sizeof(T))) = v;
}
// Streaming (nontemporal) store for full-grid outputs that the writing
// launch never reads back.  Measured per kernel: it shortens the fine-level
// solver passes and the phase/momentum update (their outputs no longer
// displace the inputs still to be read from the caches), but slows the
// kernels whose consumer re-reads the output at once from the memory-side
// cache (the prolongation, the normals/chemical-potential pass), which keep st.
template <typename T>
__device__ __forceinline__ void stn(T* base, unsigned idx, T v) {
    __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (unsigned)(idx * (unsigned)sizeof(T))));
}

// median of three: clamp in one instruction
__device__ __forceinline__ float med3(float a, float lo, float hi) { return __builtin_amdgcn_fmed3f(a, lo, hi); }
__device__ __forceinline__ double med3(double a, double lo, double hi) { return fmin(fmax(a, lo), hi); }

// a / b and 1 / sqrt(s): in FP32 the hardware reciprocal and reciprocal
// square root (1 ulp) instead of the correctly rounded sequences, which take
// about ten instructions each; FP64 keeps the correctly rounded forms
__device__ __forceinline__ float quot(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double quot(double a, double b) { return a / b; }
__device__ __forceinline__ float rsqrt_of(float s) { return __builtin_amdgcn_rsqf(s); }
__device__ __forceinline__ double rsqrt_of(double s) { return 1.0 / sqrt(s); }

__device__ __forceinline__ int block_linear() {
    return (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
}
__device__ __forceinline__ int nblocks_linear() { return gridDim.x * gridDim.y * gridDim.z; }
__device__ __forceinline__ int thread_linear() {
    return (threadIdx.z * blockDim.y + threadIdx.y) * blockDim.x + threadIdx.x;
}

// ---------------------------------------------------------------- pointwise laws

// psi'(phi) = phi (1 - phi)(1 - 2 phi)   (Eq. 2)
template <typename T>
__device__ __forceinline__ T dpsi(T f) {
    return f * (T(1) - f) * (T(1) - T(2) * f);
}
template <typename T>
__device__ __forceinline__ T psi(T f) {
    T w = f * (T(1) - f);
    return T(0.5) * w * w;
}
template <typename T>
__device__ __forceinline__ T clamp01(const Phys& P, T f) {
    // wave-uniform bounds: without the clamp the interval is the whole line
    const T lo = P.clamp ? T(0) : T(-INFINITY), hi = P.clamp ? T(1) : T(INFINITY);
    return med3(f, lo, hi);
}
// linear mixture laws, phase 1 = phi 1
template <typename T>
__device__ __forceinline__ T rho_of(const Phys& P, T f) {
    return T(P.rho2) + T(P.rho1 - P.rho2) * clamp01(P, f);
}
template <typename T>
__device__ __forceinline__ T visc_of(const Phys& P, T f) {
    return T(P.visc2) + T(P.visc1 - P.visc2) * clamp01(P, f);
}

// ---------------------------------------------------------------- reductions

// Sum NV values over a 256-thread block (wave64 shuffles, then LDS across the
// four waves).  Result valid in thread 0.  Fixed order: deterministic.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
    __shared__ double red[NV][BLOCK / 64];
    const int t = thread_linear();
    const int lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_down(v[q], o, 64);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) red[q][wave] = v[q];
    __syncthreads();
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
            for (int w = 0; w < BLOCK / 64; ++w) s += red[q][w];
            v[q] = s;
        }
    }
}

template <int NV>
__device__ __forceinline__ void block_max(double (&v)[NV]) {
    __shared__ double red[NV][BLOCK / 64];
    const int t = thread_linear();
    const int lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[q] = fmax(v[q], __shfl_down(v[q], o, 64));
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) red[q][wave] = v[q];
    __syncthreads();
    if (t == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double s = red[q][0];
            for (int w = 1; w < BLOCK / 64; ++w) s = fmax(s, red[q][w]);
            v[q] = s;
        }
    }
}

// Write the block sums of NV values to partials[q * nblocks + block].
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double* partials) {
    block_sum<NV>(v);
    if (thread_linear() == 0) {
        const int nb = nblocks_linear(), b = block_linear();
#pragma unroll
        for (int q = 0; q < NV; ++q) partials[(long)q * nb + b] = v[q];
    }
}

}  // namespace tpf

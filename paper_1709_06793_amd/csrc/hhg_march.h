// hhg_march.h -- device helpers shared by the column-marching kernels of the
// operators (hhg_kernels.hip) and of the learned correction
// (hhg_learned.hip): lattice counts, XCD-aware block order, lane shifts,
// range-checked buffer access to one tet's slot array, and the register
// sets that hold one plane of a wave's columns.
#pragma once
#include <hip/hip_runtime.h>

#include "hhg_internal.h"
#include "hhg_lattice.h"

namespace hhg {

__device__ __forceinline__ int tc32(int m) { return (m + 1) * (m + 2) * (m + 3) / 6; }
__device__ __forceinline__ int tr32(int m) { return (m + 1) * (m + 2) / 2; }
// slot of (i,j,k) in one tet lattice in 32-bit arithmetic (n <= 1024)
__device__ __forceinline__ int slot32(int n, int i, int j, int k)
{
    const int s = i + j;
    return tc32(n) - tc32(n - k) + s * (s + 1) / 2 + i;
}

__device__ __forceinline__ int xcd_remap(int b, int grid)
{
    const int per = grid >> 3;  // grid is a multiple of 8
    return (b & 7) * per + (b >> 3);
}

// Blocks of one tet: nv marching blocks and nb blocks that write the Dirichlet
// zeros.  The zeroing blocks are spread evenly among the marching ones (block
// p zeroes iff floor((p+1) nb / P) > floor(p nb / P), P = nv + nb), so that
// each XCD's contiguous share of the blocks holds its share of the marching
// work even on a single tet.  Returns true for a marching block; idx is the
// block's index among its kind.
__device__ __forceinline__ bool march_block(int p, int nv, int nb, int &idx)
{
    const int P = nv + nb;
    const int c1 = (int)(((int64_t)(p + 1) * nb) / P), c0 = (int)(((int64_t)p * nb) / P);
    if (c1 > c0) {
        idx = c0;
        return false;
    }
    idx = p - c1;
    return true;
}

// lane shifts by one position (DPP wave_shr:1 / wave_shl:1; a lane without a
// source lane gets 0)
__device__ __forceinline__ float dpp_prev(float v)  // value of lane-1
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float dpp_next(float v)  // value of lane+1
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double dpp_prev(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x138, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double dpp_next(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x130, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// buffer loads relative to one tet's slot array: the hardware range check
// returns 0 for any index outside [0, n_records), so lanes whose neighbour
// does not exist read 0 without a branch
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tet_rsrc(const void *p, int64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, int idx);
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, int idx)
{
    const auto q = __builtin_amdgcn_raw_buffer_load_b64(r, idx * 8, 0, 0);
    double v;
    __builtin_memcpy(&v, &q, 8);
    return v;
}
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, int idx)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, idx * 4, 0, 0));
}

// buffer stores relative to one tet's slot array; the whole byte offset is
// in the per-lane offset, which the range check covers: a store at an offset
// at or beyond the range is dropped
__device__ __forceinline__ void bstore(double v, __amdgpu_buffer_rsrc_t r, int voff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v),
                                          r, voff, 0, 0);
}
__device__ __forceinline__ void bstore(float v, __amdgpu_buffer_rsrc_t r, int voff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, 0, 0);
}

// one plane of a wave's columns: anti-diagonals s-1, s, s+1 at the lane's
// position for u and k (and f), plus the lane-shifted copies the rows use
template <typename T>
struct MPlane {
    T u[3], k[3], f, d, id;
    T u_sm_l, u_s_l, u_s_r, u_sp_r;
    T k_sm_l, k_s_l, k_s_r, k_sp_r;
};

// plane starting at slot P: in-plane offsets o[3] (slots).  Every load of a
// slot outside the tet's range (planes past the top included) returns 0.
// (residual and Chebyshev modes: f at the row; Chebyshev mode also the
// direction d and D^{-1} at the row)
template <typename T, int MODE>
__device__ __forceinline__ void mplane_load(MPlane<T> &p, __amdgpu_buffer_rsrc_t ru,
                                            __amdgpu_buffer_rsrc_t rk, __amdgpu_buffer_rsrc_t rf,
                                            __amdgpu_buffer_rsrc_t rd, __amdgpu_buffer_rsrc_t ri,
                                            const int o[3], int P)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) p.u[c] = bload<T>(ru, P + o[c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) p.k[c] = bload<T>(rk, P + o[c]);
    if (MODE != MODE_APPLY) p.f = bload<T>(rf, P + o[1]);
    if (MODE == MODE_CHEB) {
        p.d = bload<T>(rd, P + o[1]);
        p.id = bload<T>(ri, P + o[1]);
    }
}
template <typename T, int MODE>
__device__ __forceinline__ void mplane_load(MPlane<T> &p, __amdgpu_buffer_rsrc_t ru,
                                            __amdgpu_buffer_rsrc_t rk, __amdgpu_buffer_rsrc_t rf,
                                            const int o[3], int P)
{
    static_assert(MODE != MODE_CHEB, "Chebyshev mode needs the d and D^{-1} resources");
    mplane_load<T, MODE>(p, ru, rk, rf, rf, rf, o, P);
}

// shifted copies a plane needs as plane k+1 (and again as plane k) ...
template <typename T>
__device__ __forceinline__ void mplane_shift_up(MPlane<T> &p)
{
    p.u_sm_l = dpp_prev(p.u[0]);
    p.u_s_r = dpp_next(p.u[1]);
    p.k_sm_l = dpp_prev(p.k[0]);
    p.k_s_r = dpp_next(p.k[1]);
}
// ... and those it needs as plane k (and again as plane k-1)
template <typename T>
__device__ __forceinline__ void mplane_shift_mid(MPlane<T> &p)
{
    p.u_s_l = dpp_prev(p.u[1]);
    p.u_sp_r = dpp_next(p.u[2]);
    p.k_s_l = dpp_prev(p.k[1]);
    p.k_sp_r = dpp_next(p.k[2]);
}

}  // namespace hhg

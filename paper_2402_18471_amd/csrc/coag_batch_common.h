// coag_batch_common.h -- pieces shared by the cell-batched kernels (the
// step, coag_batch.hip, and its adjoint, coag_adjoint.hip): batch geometry,
// BF16 limb splits, the fragment mass of a pair, wave reductions, the LDS row
// stride and the XCD-aware batch order.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "coag_batch.h"

namespace coag {
namespace bc {

constexpr int kBC = kBatchCells;
constexpr int kBWaves = 8;
constexpr int kBBlock = 64 * kBWaves;
constexpr int kWin = 16;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// round-to-nearest-even BF16 limbs of x: x = a0 + a1 + a2 + O(2^-25 |x|)
struct Limbs {
    __bf16 a0, a1, a2;
};
__device__ __forceinline__ Limbs split3(float x) {
    Limbs L;
    L.a0 = (__bf16)x;
    const float r1 = x - (float)L.a0;
    L.a1 = (__bf16)r1;
    const float r2 = r1 - (float)L.a1;
    L.a2 = (__bf16)r2;
    return L;
}

// the same for eight values, as the BF16x8 operands of one MFMA, two values
// per conversion instruction
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
struct Limbs8 {
    bf16x8 a0, a1, a2;
};
__device__ __forceinline__ Limbs8 split3x8(const float (&x)[8]) {
    union {
        bf16x2 h[4];
        bf16x8 v;
    } A0, A1, A2;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const f32x2 v = {x[2 * e], x[2 * e + 1]};
        A0.h[e] = __builtin_convertvector(v, bf16x2);
        const f32x2 r1 = v - __builtin_convertvector(A0.h[e], f32x2);
        A1.h[e] = __builtin_convertvector(r1, bf16x2);
        const f32x2 r2 = r1 - __builtin_convertvector(A1.h[e], f32x2);
        A2.h[e] = __builtin_convertvector(r2, bf16x2);
    }
    return Limbs8{A0.v, A1.v, A2.v};
}

// mass of the fragments of pair (i, j), total minus remnant (eq. `fragrem`),
// evaluated exactly as the pair tables are: no contraction into an FMA
__device__ __forceinline__ double frag_mass(double mi, double mj, double chi, bool &crater) {
#pragma clang fp contract(off)
    const double cm = chi * mj;
    crater = cm < mi;
    const double mrem = crater ? mi - cm : 0.0;
    return (mi + mj) - mrem;
}

__device__ __forceinline__ double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_min_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

// Row stride of the per-cell LDS arrays: odd, so that 16 cells' entries of
// one bin fall in 16 different banks (a stride that is a multiple of 2^k
// folds them onto 32 / 2^(k-1) banks: 8-way conflicts at N = 80, 4-way at 200)
__host__ __device__ constexpr int batch_row_stride(int N) { return N | 1; }

// A raw buffer over `bytes` bytes from base (a wave-uniform pointer): loads
// through it take a 32-bit byte offset per lane, with no 64-bit address
// arithmetic in the vector unit, and read zero past the end.  The fourth
// descriptor word is the gfx9 raw-buffer format (32-bit data).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_buffer(const void *base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             0x00020000);
}
// a double / a float at byte offset off; nt: non-temporal (streamed once)
template <bool NT>
__device__ __forceinline__ double buf_f64(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, NT ? 2 : 0));
}
template <bool NT>
__device__ __forceinline__ float buf_f32(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, NT ? 2 : 0));
}
// 16 bytes at byte offset off, as two doubles or four floats (the whole
// vector is cast: the compiler mistranslates element reads of the 128-bit
// load's integer result)
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ f64x2 buf_f64x2(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, NT ? 2 : 0));
}
template <bool NT>
__device__ __forceinline__ f32x4 buf_f32x4(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, NT ? 2 : 0));
}

// The batch a workgroup takes.  Workgroups are dealt to the eight XCDs in
// turn (workgroup w to XCD w mod 8), and each XCD runs its share from its own
// queue, so with the plain mapping XCD x would take every batch b = x mod 8:
// on a disc stored radius by radius with eight batches per radius, always the
// same height above the midplane, and the XCD with the stiffest layer would
// finish last.  Workgroup 8k + x takes batch 8k + (x + k) mod 8 instead (the
// last, incomplete group of eight keeps the plain mapping): each XCD sees
// every layer, and batches still start in about index order.
__device__ __forceinline__ long batch_of(long w, long nb) {
    const long k = w >> 3;
    return 8 * k + 8 > nb ? w : 8 * k + ((w + k) & 7);
}

}  // namespace bc
}  // namespace coag

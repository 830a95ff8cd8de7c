// Shared pieces of the butterfly kernels (Sec. 3.2, App. A.1): the argument
// block every butterfly kernel receives, the wave shapes of the level
// launches, and the 16x16x4 matrix-core product with its lane layout.
#pragma once
#include "internal.h"

namespace sht {


template <typename S>
struct BfArgs {
    const int4 *__restrict__ res_task;
    const int4 *__restrict__ res_sub;
    const int2 *__restrict__ res_lane;
    const double2 *__restrict__ res_val;
    const int16_t *__restrict__ perm;
    const int *__restrict__ node_i;
    const S *__restrict__ T;
    const double *__restrict__ z2;
    const long long *__restrict__ coef_off;
    const double *__restrict__ coef;
    const double2 *__restrict__ alm;
    double2 *__restrict__ q;
    S *__restrict__ ws;  // vector workspace, entries of ES values
    const double2 *__restrict__ ybar;  // adjoint input [ring][m][nmaps]
    double *__restrict__ g;            // adjoint output [nalm][nmaps] complex
    int L, K, nrings, nmaps, map0;
    // A pass transforms G groups of NB maps (maps map0 .. map0 + G NB - 1):
    // every workspace entry holds ES = 2 NB G values (re, im per map) and
    // group g owns values [2 NB g, 2 NB (g + 1)) of each entry.  The
    // interpolation matrices are streamed from HBM once per pass; the level
    // workgroups loop over the groups of their node (the repeated reads of a
    // node's blocks hit the caches).
    int ES, G;
    // level-1 and fold lists of the plan (work-queue batches address them
    // through the argument block)
    const int4 *__restrict__ f1_unit;
    const int *__restrict__ fold_slot;
    int fold_count;
};

// Maps of one pass at most (G <= kBfMaxGroups groups of 8 maps).
constexpr int kBfMaxGroups = 8;

// Shape of the pass that starts with `left` maps still to transform: groups
// of 8 maps while at least 8 remain, else one group of 4, 2 or 1.
inline void bf_pass_shape(int left, int *nb, int *groups) {
    if (left >= 8) {
        *nb = 8;
        *groups = left / 8 < kBfMaxGroups ? left / 8 : kBfMaxGroups;
    } else {
        *nb = left >= 4 ? 4 : left >= 2 ? 2 : 1;
        *groups = 1;
    }
}

// Values per workspace entry for transforms of nmaps maps (the first pass
// is the widest).
inline int bf_entry_values(int nmaps) {
    int nb, g;
    bf_pass_shape(nmaps, &nb, &g);
    return 2 * nb * g;
}

constexpr int kBfThreads = 256;

// Read-only operands that every lane of a wave needs at the same address
// (a_lm rows, recurrence coefficients) are read through the constant
// address space so that they arrive by scalar loads into SGPRs.
typedef const __attribute__((address_space(4))) double c_double;

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
template <typename S>
struct Acc;
template <>
struct Acc<double> {
    typedef d4_t type;
};
template <>
struct Acc<float> {
    typedef f4_t type;
};

// D(16x16) += A(16x4) B(4x16) on the matrix cores.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Element r of the accumulator of
// lane l is D[acc_row(l / 16, r)][l % 16]: row 4 (l / 16) + r for FP32, row
// l / 16 + 4 r for FP64 (measured on gfx950).
__device__ __forceinline__ d4_t mfma_16x16x4(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma_16x16x4(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename S>
__device__ __forceinline__ int acc_row(int k4, int r) {
    return sizeof(S) == 8 ? k4 + 4 * r : 4 * k4 + r;
}

// Waves per child of a pair node: each takes 4 / kBfHalves of a group's
// 16-row tiles; a level workgroup holds one wave per child and half.
constexpr int kBfHalves = 1;
constexpr int kBfLevelThreads = 128 * kBfHalves;

// base[idx] with a 32-bit byte offset, so that the load can take a
// wave-uniform 64-bit base in SGPRs and one 32-bit VGPR per lane (blocks of
// interpolation entries and level vectors stay far below 4 GiB).
template <typename S>
__device__ __forceinline__ S ld32(const S *base, unsigned idx) {
    return *reinterpret_cast<const S *>(reinterpret_cast<const char *>(base) + idx * (unsigned)sizeof(S));
}

// LDS of one pair node with n columns: one vector of n entries of 2 NB
// values per child.
template <int NB, typename S>
inline size_t bf_level_lds(int n) {
    return (size_t)n * 2 * (2 * NB * sizeof(S));
}

// The plan-dependent fields of BfArgs; the caller sets the operands of its
// direction (alm, q or ybar, g) and map0.
template <typename S>
inline BfArgs<S> bf_args(const sht_plan_s *p, int nmaps, const S *T, S *ws) {
    BfArgs<S> a;
    a.res_task = reinterpret_cast<const int4 *>(p->d_bf_res_task);
    a.res_sub = reinterpret_cast<const int4 *>(p->d_bf_res_sub);
    a.res_lane = reinterpret_cast<const int2 *>(p->d_bf_res_lane);
    a.res_val = reinterpret_cast<const double2 *>(p->d_bf_res_val);
    a.perm = p->d_bf_perm;
    a.node_i = p->d_bf_node_i;
    a.T = T;
    a.z2 = p->d_z2_hi;
    a.coef_off = p->d_coef_off;
    a.coef = p->d_coef_hi;
    a.alm = nullptr;
    a.q = nullptr;
    a.ws = ws;
    a.ybar = nullptr;
    a.g = nullptr;
    a.L = p->L;
    a.K = p->bf.K;
    a.nrings = p->nrings;
    a.nmaps = nmaps;
    a.map0 = 0;
    a.ES = 2;
    a.G = 1;
    a.f1_unit = reinterpret_cast<const int4 *>(p->d_bf_f1_unit);
    a.fold_slot = p->d_bf_fold_slot;
    a.fold_count = p->bf.built ? (int)(p->bf.fold_off.back() - p->bf.fold_off.front()) : 0;
    return a;
}

}  // namespace sht

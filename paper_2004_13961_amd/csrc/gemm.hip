// Strided, batched dense contractions on the CDNA4 matrix cores.
//
// Every stage of the sum-factorised operator (forward transforms to the
// Legendre-Gauss nodes, pointwise coefficient multiply, transposed
// transforms back to the compact basis) is one such contraction:
//     C[b](i,j) (+)= E[b](i,j) * sum_k A[b](i,k) B[b](k,j)
// with arbitrary element strides, so a 1D table can be applied along any
// tensor axis without transposing data. The optional E multiplier fuses the
// pointwise step of the paper's step 3 into the epilogue of the forward
// transform.
//
// Tiles: 64x64 outputs per 256-thread workgroup, 4 wave64s in a 2x2 layout,
// each wave owning 32x32 = 2x2 MFMA 16x16 blocks. FP64 and FP32 use
// v_mfma_{f64,f32}_16x16x4 (lane l supplies A(l%16, l/16) and B(l/16, l%16)).
// Accumulator register r of lane l holds C(4*(l/16)+r, l%16) for FP32 and
// C(l/16 + 4*r, l%16) for FP64 (its 16x16 result is row-interleaved). BF16 uses
// v_mfma_f32_16x16x32_bf16 (lane l supplies A(l%16, 8*(l/16)..+7) and
// B(8*(l/16)..+7, l%16)), with FP32 accumulation and FP32 global data.
#include "lgp_internal.h"

namespace lgp {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, NT = 256;

__device__ inline dbl4 mfma16x16x4(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline flt4 mfma16x16x4(float a, float b, flt4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T, typename V4>
__global__ __launch_bounds__(NT) void gemm_k4_kernel(GemmArgs g) {
    if (g.stop && *g.stop) return;
    constexpr int BK = 16;
    __shared__ T As[BK][BM + 1];
    __shared__ T Bs[BK][BN + 1];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t b = blockIdx.z;
    const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
    const T* A = (const T*)g.A + b * g.sAb;
    const T* B = (const T*)g.B + b * g.sBb;
    T* C = (T*)g.C + b * g.sCb;
    const bool a_kc = (g.sAk == 1);
    const bool b_jc = (g.sBj == 1);

    V4 acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
            for (int r = 0; r < 4; ++r) acc[x][y][r] = T(0);

    T ra[4], rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            int i, k;
            if (a_kc) { k = tid & 15; i = (tid >> 4) + 16 * p; }
            else      { i = tid & 63; k = (tid >> 6) + 4 * p; }
            const int gi = i0 + i, gk = k0 + k;
            ra[p] = (gi < g.M && gk < g.K) ? A[(int64_t)gi * g.sAi + (int64_t)gk * g.sAk] : T(0);
            int j, kb;
            if (b_jc) { j = tid & 63; kb = (tid >> 6) + 4 * p; }
            else      { kb = tid & 15; j = (tid >> 4) + 16 * p; }
            const int gj = j0 + j, gkb = k0 + kb;
            rb[p] = (gj < g.N && gkb < g.K) ? B[(int64_t)gkb * g.sBk + (int64_t)gj * g.sBj] : T(0);
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            int i, k;
            if (a_kc) { k = tid & 15; i = (tid >> 4) + 16 * p; }
            else      { i = tid & 63; k = (tid >> 6) + 4 * p; }
            As[k][i] = ra[p];
            int j, kb;
            if (b_jc) { j = tid & 63; kb = (tid >> 6) + 4 * p; }
            else      { kb = tid & 15; j = (tid >> 4) + 16 * p; }
            Bs[kb][j] = rb[p];
        }
    };

    load(0);
    store();
    __syncthreads();
    for (int k0 = 0; k0 < g.K; k0 += BK) {
        const bool more = (k0 + BK) < g.K;
        if (more) load(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + (lane >> 4);
            const T a0 = As[kr][wm * 32 + (lane & 15)];
            const T a1 = As[kr][wm * 32 + 16 + (lane & 15)];
            const T b0 = Bs[kr][wn * 32 + (lane & 15)];
            const T b1 = Bs[kr][wn * 32 + 16 + (lane & 15)];
            acc[0][0] = mfma16x16x4(a0, b0, acc[0][0]);
            acc[0][1] = mfma16x16x4(a0, b1, acc[0][1]);
            acc[1][0] = mfma16x16x4(a1, b0, acc[1][0]);
            acc[1][1] = mfma16x16x4(a1, b1, acc[1][1]);
        }
        __syncthreads();
        if (more) {
            store();
            __syncthreads();
        }
    }

    const T* E = g.E ? (const T*)g.E + b * g.sEb : nullptr;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = (sizeof(T) == 8) ? (lane >> 4) + 4 * r : (lane >> 4) * 4 + r;
                const int i = i0 + wm * 32 + mi * 16 + rr;
                const int j = j0 + wn * 32 + ni * 16 + (lane & 15);
                if (i < g.M && j < g.N) {
                    T v = acc[mi][ni][r];
                    if (E) v *= E[(int64_t)i * g.sEi + (int64_t)j * g.sEj];
                    T* c = C + (int64_t)i * g.sCi + (int64_t)j * g.sCj;
                    if (g.accumulate) *c += v;
                    else *c = v;
                }
            }
}

// BF16 operands, FP32 data and accumulation.
__global__ __launch_bounds__(NT) void gemm_bf16_kernel(GemmArgs g) {
    if (g.stop && *g.stop) return;
    constexpr int BK = 32, PAD = 8;
    __shared__ __attribute__((aligned(16))) __bf16 As[BM][BK + PAD];   // [i][k]
    __shared__ __attribute__((aligned(16))) __bf16 Bs[BN][BK + PAD];   // [j][k]
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t b = blockIdx.z;
    const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
    const float* A = (const float*)g.A + b * g.sAb;
    const float* B = (const float*)g.B + b * g.sBb;
    float* C = (float*)g.C + b * g.sCb;
    const bool a_kc = (g.sAk == 1);
    const bool b_jc = (g.sBj == 1);

    flt4 acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
            for (int r = 0; r < 4; ++r) acc[x][y][r] = 0.f;

    float ra[8], rb[8];
    auto idxA = [&](int p, int& i, int& k) {
        if (a_kc) { k = tid & 31; i = (tid >> 5) + 8 * p; }
        else      { i = tid & 63; k = (tid >> 6) + 4 * p; }
    };
    auto idxB = [&](int p, int& j, int& k) {
        if (b_jc) { j = tid & 63; k = (tid >> 6) + 4 * p; }
        else      { k = tid & 31; j = (tid >> 5) + 8 * p; }
    };
    auto load = [&](int k0) {
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            int i, k;
            idxA(p, i, k);
            const int gi = i0 + i, gk = k0 + k;
            ra[p] = (gi < g.M && gk < g.K) ? A[(int64_t)gi * g.sAi + (int64_t)gk * g.sAk] : 0.f;
            int j, kb;
            idxB(p, j, kb);
            const int gj = j0 + j, gkb = k0 + kb;
            rb[p] = (gj < g.N && gkb < g.K) ? B[(int64_t)gkb * g.sBk + (int64_t)gj * g.sBj] : 0.f;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            int i, k;
            idxA(p, i, k);
            As[i][k] = (__bf16)ra[p];
            int j, kb;
            idxB(p, j, kb);
            Bs[j][kb] = (__bf16)rb[p];
        }
    };

    load(0);
    store();
    __syncthreads();
    for (int k0 = 0; k0 < g.K; k0 += BK) {
        const bool more = (k0 + BK) < g.K;
        if (more) load(k0 + BK);
        const int kq = 8 * (lane >> 4);
        const bf16x8 a0 = *(const bf16x8*)&As[wm * 32 + (lane & 15)][kq];
        const bf16x8 a1 = *(const bf16x8*)&As[wm * 32 + 16 + (lane & 15)][kq];
        const bf16x8 b0 = *(const bf16x8*)&Bs[wn * 32 + (lane & 15)][kq];
        const bf16x8 b1 = *(const bf16x8*)&Bs[wn * 32 + 16 + (lane & 15)][kq];
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1, acc[1][1], 0, 0, 0);
        __syncthreads();
        if (more) {
            store();
            __syncthreads();
        }
    }

    const float* E = g.E ? (const float*)g.E + b * g.sEb : nullptr;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + wm * 32 + mi * 16 + (lane >> 4) * 4 + r;
                const int j = j0 + wn * 32 + ni * 16 + (lane & 15);
                if (i < g.M && j < g.N) {
                    float v = acc[mi][ni][r];
                    if (E) v *= E[(int64_t)i * g.sEi + (int64_t)j * g.sEj];
                    float* c = C + (int64_t)i * g.sCi + (int64_t)j * g.sCj;
                    if (g.accumulate) *c += v;
                    else *c = v;
                }
            }
}

lgp_status gemm(GemmMode mode, const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return LGP_OK;
    if (g.K <= 0) return LGP_E_ARG;
    const int gy = (g.M + BM - 1) / BM;
    if (gy > 65535 || g.batch > 65535) return LGP_E_UNSUPPORTED;
    dim3 grid((g.N + BN - 1) / BN, gy, g.batch);
    switch (mode) {
        case GEMM_F64:
            hipLaunchKernelGGL((gemm_k4_kernel<double, dbl4>), grid, dim3(NT), 0, s, g);
            break;
        case GEMM_F32:
            hipLaunchKernelGGL((gemm_k4_kernel<float, flt4>), grid, dim3(NT), 0, s, g);
            break;
        case GEMM_BF16:
            hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(NT), 0, s, g);
            break;
    }
    LGP_CHECK_LAUNCH();
    return LGP_OK;
}

}  // namespace lgp

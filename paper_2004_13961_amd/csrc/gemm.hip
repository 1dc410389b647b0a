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
// Tiles: (32 MI) x (32 NI) outputs per 256-thread workgroup, 4 wave64s in a
// 2x2 layout, each wave owning MI x NI MFMA 16x16 blocks (variants picked per
// shape by the autotuner; the BF16 kernel is 64x64). FP64 and FP32 use
// v_mfma_{f64,f32}_16x16x4 (lane l supplies A(l%16, l/16) and B(l/16, l%16)).
// Accumulator register r of lane l holds C(4*(l/16)+r, l%16) for FP32 and
// C(l/16 + 4*r, l%16) for FP64 (its 16x16 result is row-interleaved). BF16 uses
// v_mfma_f32_16x16x32_bf16 (lane l supplies A(l%16, 8*(l/16)..+7) and
// B(8*(l/16)..+7, l%16)), with FP32 accumulation and FP32 global data.
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

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

// Tile variants: each of the 2x2 waves owns MI x NI MFMA blocks of 16x16,
// so a workgroup computes (32 MI) x (32 NI) outputs. The sum over k runs in
// the same order in every variant (K steps of 16, MFMA k-groups of 4), so all
// variants give bit-identical results; the autotuner below picks the
// fastest per contraction shape.
template <typename T, typename V4, int MI, int NI>
__global__ __launch_bounds__(NT) void gemm_k4_kernel(GemmArgs g) {
    if (g.stop && *g.stop) return;
    constexpr int BK = 16;
    constexpr int TM = 32 * MI, TN = 32 * NI;
    constexpr int PA = TM * BK / NT, PB = TN * BK / NT;   // elements per thread
    __shared__ T As[BK][TM + 1];
    __shared__ T Bs[BK][TN + 1];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t b = blockIdx.z;
    const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
    const T* A = (const T*)g.A + b * g.sAb;
    const T* B = (const T*)g.B + b * g.sBb;
    T* C = (T*)g.C + b * g.sCb;
    const bool a_kc = (g.sAk == 1);
    const bool b_jc = (g.sBj == 1);

    V4 acc[MI][NI];
    for (int x = 0; x < MI; ++x)
        for (int y = 0; y < NI; ++y)
            for (int r = 0; r < 4; ++r) acc[x][y][r] = T(0);

    T ra[PA], rb[PB];
    // element p of this thread in the A tile (TM x BK) and the B tile (BK x TN):
    // consecutive threads along the contiguous index of the source
    auto idxA = [&](int p, int& i, int& k) {
        const int e = tid + NT * p;
        if (a_kc) { k = e % BK; i = e / BK; }
        else      { i = e % TM; k = e / TM; }
    };
    auto idxB = [&](int p, int& j, int& k) {
        const int e = tid + NT * p;
        if (b_jc) { j = e % TN; k = e / TN; }
        else      { k = e % BK; j = e / BK; }
    };
    auto load = [&](int k0) {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            int i, k;
            idxA(p, i, k);
            const int gi = i0 + i, gk = k0 + k;
            ra[p] = (gi < g.M && gk < g.K) ? A[(int64_t)gi * g.sAi + (int64_t)gk * g.sAk] : T(0);
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            int j, kb;
            idxB(p, j, kb);
            const int gj = j0 + j, gkb = k0 + kb;
            rb[p] = (gj < g.N && gkb < g.K) ? B[(int64_t)gkb * g.sBk + (int64_t)gj * g.sBj] : T(0);
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            int i, k;
            idxA(p, i, k);
            As[k][i] = ra[p];
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            int j, kb;
            idxB(p, j, kb);
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
            T av[MI], bv[NI];
#pragma unroll
            for (int mi = 0; mi < MI; ++mi) av[mi] = As[kr][wm * 16 * MI + mi * 16 + (lane & 15)];
#pragma unroll
            for (int ni = 0; ni < NI; ++ni) bv[ni] = Bs[kr][wn * 16 * NI + ni * 16 + (lane & 15)];
#pragma unroll
            for (int mi = 0; mi < MI; ++mi)
#pragma unroll
                for (int ni = 0; ni < NI; ++ni) acc[mi][ni] = mfma16x16x4(av[mi], bv[ni], acc[mi][ni]);
        }
        __syncthreads();
        if (more) {
            store();
            __syncthreads();
        }
    }

    const T* E = g.E ? (const T*)g.E + b * g.sEb : nullptr;
#pragma unroll
    for (int mi = 0; mi < MI; ++mi)
#pragma unroll
        for (int ni = 0; ni < NI; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = (sizeof(T) == 8) ? (lane >> 4) + 4 * r : (lane >> 4) * 4 + r;
                const int i = i0 + wm * 16 * MI + mi * 16 + rr;
                const int j = j0 + wn * 16 * NI + ni * 16 + (lane & 15);
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

// ------------------------------------------------------- autotuner -----
// Tile variants of the FP64 / FP32 kernel: (MI, NI) = blocks of 16x16 per
// wave. The first time a contraction shape (mode, M, N, K, batch, operand
// layouts) is seen outside a stream capture, every variant runs three times
// on the caller's stream and the fastest (HIP events) is kept for that shape
// for the life of the process. Variants agree bit for bit, so the choice
// never changes a result. LGP_GEMM_TUNE=0 keeps the 64x64 variant.
struct GemmVariant {
    int MI, NI;
};
static const GemmVariant kVariants[] = {{2, 2}, {1, 2}, {2, 1}, {1, 1}, {4, 2}, {2, 4}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <typename T, typename V4>
static void launch_variant(int v, const GemmArgs& g, hipStream_t s) {
    const int TM = 32 * kVariants[v].MI, TN = 32 * kVariants[v].NI;
    dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM, g.batch);
    switch (v) {
        case 0: hipLaunchKernelGGL((gemm_k4_kernel<T, V4, 2, 2>), grid, dim3(NT), 0, s, g); break;
        case 1: hipLaunchKernelGGL((gemm_k4_kernel<T, V4, 1, 2>), grid, dim3(NT), 0, s, g); break;
        case 2: hipLaunchKernelGGL((gemm_k4_kernel<T, V4, 2, 1>), grid, dim3(NT), 0, s, g); break;
        case 3: hipLaunchKernelGGL((gemm_k4_kernel<T, V4, 1, 1>), grid, dim3(NT), 0, s, g); break;
        case 4: hipLaunchKernelGGL((gemm_k4_kernel<T, V4, 4, 2>), grid, dim3(NT), 0, s, g); break;
        case 5: hipLaunchKernelGGL((gemm_k4_kernel<T, V4, 2, 4>), grid, dim3(NT), 0, s, g); break;
    }
}

struct GemmKey {
    int mode, M, N, K, batch, akc, bjc, acc;
    bool operator<(const GemmKey& o) const {
        return std::tie(mode, M, N, K, batch, akc, bjc, acc) < std::tie(o.mode, o.M, o.N, o.K, o.batch, o.akc, o.bjc, o.acc);
    }
};
static std::mutex g_tune_mu;
static std::map<GemmKey, int> g_tune;

int gemm_tuned_variant(GemmMode mode, const GemmArgs& g) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const GemmKey key{(int)mode, g.M, g.N, g.K, g.batch, g.sAk == 1, g.sBj == 1, g.accumulate};
    auto it = g_tune.find(key);
    return it == g_tune.end() ? -1 : it->second;
}

template <typename T, typename V4>
static int tune(GemmMode mode, const GemmArgs& g, hipStream_t s) {
    const GemmKey key{(int)mode, g.M, g.N, g.K, g.batch, g.sAk == 1, g.sBj == 1, g.accumulate};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) return it->second;
    }
    const char* env = std::getenv("LGP_GEMM_TUNE");
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if ((env && env[0] == '0') || hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return 0;
    // timing runs write C: with accumulate set they would change it, so an
    // accumulating contraction is timed on a copy of nothing -- it keeps 64x64
    if (g.accumulate) return 0;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return 0;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return 0;
    }
    int best = 0;
    float best_ms = 1e30f;
    for (int v = 0; v < kNumVariants; ++v) {
        launch_variant<T, V4>(v, g, s);   // warm
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < 3; ++r) launch_variant<T, V4>(v, g, s);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) break;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    return best;
}

lgp_status gemm(GemmMode mode, const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return LGP_OK;
    if (g.K <= 0) return LGP_E_ARG;
    if ((g.M + 31) / 32 > 65535 || g.batch > 65535) return LGP_E_UNSUPPORTED;
    switch (mode) {
        case GEMM_F64: {
            const int v = tune<double, dbl4>(mode, g, s);
            launch_variant<double, dbl4>(v, g, s);
            break;
        }
        case GEMM_F32: {
            const int v = tune<float, flt4>(mode, g, s);
            launch_variant<float, flt4>(v, g, s);
            break;
        }
        case GEMM_BF16: {
            dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, g.batch);
            hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(NT), 0, s, g);
            break;
        }
    }
    LGP_CHECK_LAUNCH();
    return LGP_OK;
}

}  // namespace lgp

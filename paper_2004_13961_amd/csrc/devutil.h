// Device helpers shared by the substitution and factorisation kernels:
// coherent loads and stores, wave reductions, the not-yet-written sentinel.
#pragma once
#include "lgp_internal.h"

namespace lgp {

// Raise a kernel's dynamic LDS limit; skipped while `s` is being captured
// into a graph (the attribute, set by an earlier eager launch, persists).
inline void set_dyn_shmem(const void* kernel, size_t bytes, hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s && hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;
    (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// ------------------------------------------------------ device helpers ---
// Values produced and consumed inside one kernel by different workgroups
// (substitution results, factor rows, pivots, progress flags) travel through
// device-coherent accesses: relaxed device-scope atomic loads and stores,
// which the compiler emits as sc1 global accesses and which need no L2
// write-back or invalidate. A producer waits for its own stores to complete
// (s_waitcnt vmcnt(0)) before it publishes a flag, so a consumer that has
// seen the flag and then loads coherently sees the data. Data written by an
// earlier kernel (the factors, the right-hand side) is read with ordinary
// cached loads.
template <typename T>
__device__ inline T ld_coh(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ inline void st_coh(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void wait_own_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ inline void compiler_fence() { asm volatile("" ::: "memory"); }
__device__ inline void publish(unsigned* flag, unsigned v) {
    wait_own_stores();
    st_coh(flag, v);
}

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline float wave_sum(float v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Wave-wide sum with DPP lane moves inside each row of 16 lanes (pair swap,
// quad swap, half-row mirror, row mirror), then the four row sums combined
// through readlane; every lane returns the same value.
template <int CTRL>
__device__ inline int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ inline double dpp_v(double v) {
    const int lo = dpp_i<CTRL>(__double2loint(v));
    const int hi = dpp_i<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ inline float dpp_v(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
__device__ inline double lane_val(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}
__device__ inline float lane_val(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
template <typename T>
__device__ inline T wave_sum_dpp(T v) {
    v += dpp_v<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_v<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_v<0x141>(v);   // row_half_mirror
    v += dpp_v<0x140>(v);   // row_mirror
    return (lane_val(v, 0) + lane_val(v, 16)) + (lane_val(v, 32) + lane_val(v, 48));
}

// Sentinel marking a substitution result that is not written yet: a NaN
// payload that arithmetic never produces (computed NaNs are stored as the
// canonical quiet NaN instead), so polling the value itself tells a
// consumer whether it is ready.
template <typename T> struct Sentinel;
template <> struct Sentinel<double> {
    static __device__ __host__ inline double value() { return __longlong_as_double(0x7FF40000DEADBEEFll); }
    static __device__ inline bool is(double v) { return __double_as_longlong(v) == 0x7FF40000DEADBEEFll; }
    static __device__ inline double clean(double v) { return isnan(v) ? __longlong_as_double(0x7FF8000000000000ll) : v; }
};
template <> struct Sentinel<float> {
    static __device__ __host__ inline float value() { return __int_as_float(0x7FA0BEEF); }
    static __device__ inline bool is(float v) { return __float_as_int(v) == 0x7FA0BEEF; }
    static __device__ inline float clean(float v) { return isnan(v) ? __int_as_float(0x7FC00000) : v; }
};

template <typename T>
__global__ void fill_sentinel_kernel(int64_t n, T* __restrict__ out, const int* __restrict__ stop) {
    if (stop && *stop) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = Sentinel<T>::value();
}

// Wave total with DPP only: sums inside rows of 16 lanes, row_bcast15 adds
// row 0 into row 1 and row 2 into row 3, row_bcast31 adds lane 31 into rows
// 2 and 3; lane 63 then holds the total, read once into scalar registers.
// The moves carry no old value (no register copies); lanes of the rows a
// broadcast leaves out hold junk afterwards, but no later stage reads them
// on the way to lane 63.
template <int CTRL, int ROWS>
__device__ inline double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ inline double wave_total_bcast(double v) {
    v += dpp_mov<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
    v += dpp_mov<0x141, 0xF>(v);   // row_half_mirror
    v += dpp_mov<0x140, 0xF>(v);   // row_mirror
    v += dpp_mov<0x142, 0xA>(v);   // row_bcast15 into rows 1, 3
    v += dpp_mov<0x143, 0xC>(v);   // row_bcast31 into rows 2, 3
    return lane_val(v, 63);
}

}  // namespace lgp

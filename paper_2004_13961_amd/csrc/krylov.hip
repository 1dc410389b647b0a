// PCG (paper Alg. 1) with device-resident scalars, and the FP64 iterative
// refinement around a low-precision inner PCG.
//
// One iteration enqueues: z = U^{-1} L^{-1} r (two sweeps), rho = r.z,
// p = z + (rho/rho_old) p, w = K p, alpha = rho / p.w, x += alpha p,
// r -= alpha w, ||r||^2. Dot products are two-pass (fixed block partials,
// then one block sums them in a fixed order), so results do not depend on
// scheduling. Every kernel first reads the `done` flag and returns when a
// previous step declared convergence or breakdown, so the host may enqueue
// several iterations before it looks at the flag.
#include <cmath>
#include <cstdlib>
#include <new>

#include "lgp_internal.h"

namespace lgp {

constexpr int NPART = 512;     // partial sums per dot product
constexpr int VBS = 256;

enum {
    SC_RHO = 0, SC_RHO_OLD, SC_PW, SC_RR, SC_ALPHA, SC_BETA, SC_FF, SC_THRESH2,
    SC_K, SC_KMAX, SC_RHO2, SC_COUNT = 16
};
enum { FL_DONE = 0, FL_BREAK = 1, FL_FIRST = 2, FL_XZERO = 3, FL_COUNT = 4 };

struct SolveWS {
    double* r; double* z; double* p; double* w;            // FP64
    float* r32; float* z32; float* p32; float* w32; float* e32; float* y32;
    double* part; double* sc; int* fl;
    size_t bytes;
};

static size_t plan_ws(SolveWS& S, int64_t n, bool mixed, void* buf) {
    Carver c(buf);
    S.r = c.take<double>(n);
    S.z = c.take<double>(n);
    S.p = c.take<double>(n);
    S.w = c.take<double>(n);
    if (mixed) {
        S.r32 = c.take<float>(n);
        S.z32 = c.take<float>(n);
        S.p32 = c.take<float>(n);
        S.w32 = c.take<float>(n);
        S.e32 = c.take<float>(n);
        S.y32 = c.take<float>(n);
    } else {
        S.r32 = S.z32 = S.p32 = S.w32 = S.e32 = S.y32 = nullptr;
    }
    S.part = c.take<double>(2 * NPART);   // two sets: p.w, then r.r in the same kernel
    S.sc = c.take<double>(SC_COUNT);
    S.fl = c.take<int>(FL_COUNT);
    S.bytes = c.off + 256;
    return S.bytes;
}

size_t solve_ws_bytes(int64_t n, bool mixed) {
    SolveWS S;
    return plan_ws(S, n, mixed, nullptr);
}

// ------------------------------------------------------------ kernels ----
__device__ inline double block_sum(double v) {
    __shared__ double red[VBS / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < VBS / 64; ++k) s += red[k];
    __syncthreads();
    return s;
}

template <typename T>
__global__ __launch_bounds__(VBS) void dot_kernel(int64_t n, const T* __restrict__ a, const T* __restrict__ b,
                                                  double* __restrict__ part, const int* __restrict__ fl) {
    if (fl[FL_DONE]) return;
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VBS + threadIdx.x; i < n; i += (int64_t)NPART * VBS)
        s += (double)a[i] * (double)b[i];
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__device__ inline double sum_parts(const double* part) {
    double s = 0.0;
    for (int k = threadIdx.x; k < NPART; k += VBS) s += part[k];
    return block_sum(s);
}

// rho_old = rho; rho = r.z; beta = rho/rho_old (0 on the first iteration)
__global__ __launch_bounds__(VBS) void fin_rho_kernel(const double* part, double* sc, int* fl) {
    if (fl[FL_DONE]) return;
    const double s = sum_parts(part);
    if (threadIdx.x == 0) {
        sc[SC_RHO_OLD] = sc[SC_RHO];
        sc[SC_RHO] = s;
        if (fl[FL_FIRST]) sc[SC_BETA] = 0.0;
        else sc[SC_BETA] = s / sc[SC_RHO_OLD];
        if (!(s > 0.0) || !isfinite(s)) { fl[FL_BREAK] = 1; fl[FL_DONE] = 1; }
    }
}

// alpha = rho / p.w
__global__ __launch_bounds__(VBS) void fin_alpha_kernel(const double* part, double* sc, int* fl) {
    if (fl[FL_DONE]) return;
    const double s = sum_parts(part);
    if (threadIdx.x == 0) {
        sc[SC_PW] = s;
        sc[SC_ALPHA] = sc[SC_RHO] / s;
        if (!(s > 0.0) || !isfinite(s)) { fl[FL_BREAK] = 1; fl[FL_DONE] = 1; }
    }
}

// rr = r.r; k += 1; stop when sqrt(rr) <= eps ||F|| or k >= k_max (Alg. 1)
__global__ __launch_bounds__(VBS) void fin_rr_kernel(const double* part, double* sc, int* fl, int count_iter) {
    if (fl[FL_DONE]) return;
    const double s = sum_parts(part);
    if (threadIdx.x == 0) {
        sc[SC_RR] = s;
        if (count_iter) {
            sc[SC_K] += 1.0;
            fl[FL_FIRST] = 0;
        }
        if (s <= sc[SC_THRESH2] || sc[SC_K] >= sc[SC_KMAX]) fl[FL_DONE] = 1;
        if (!isfinite(s)) { fl[FL_BREAK] = 1; fl[FL_DONE] = 1; }
    }
}

__global__ void fin_ff_kernel(const double* part, double* sc, double eps2) {
    const double s = sum_parts(part);
    if (threadIdx.x == 0) {
        sc[SC_FF] = s;
        sc[SC_THRESH2] = eps2 * s;
    }
}

template <typename T>
__global__ __launch_bounds__(VBS) void update_p_kernel(int64_t n, const T* __restrict__ z, T* __restrict__ p,
                                                       const double* __restrict__ sc, const int* __restrict__ fl) {
    if (fl[FL_DONE]) return;
    const bool first = fl[FL_FIRST] != 0;
    const T beta = (T)sc[SC_BETA];
    for (int64_t i = blockIdx.x * (int64_t)VBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBS)
        p[i] = first ? z[i] : z[i] + beta * p[i];
}

// x += alpha p; r -= alpha w; partial r.r
template <typename T>
__global__ __launch_bounds__(VBS) void update_xr_kernel(int64_t n, T* __restrict__ x, T* __restrict__ r,
                                                        const T* __restrict__ p, const T* __restrict__ w,
                                                        const double* __restrict__ sc, double* __restrict__ part,
                                                        const int* __restrict__ fl) {
    if (fl[FL_DONE]) return;
    const T alpha = (T)sc[SC_ALPHA];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VBS + threadIdx.x; i < n; i += (int64_t)NPART * VBS) {
        x[i] += alpha * p[i];
        const T ri = r[i] - alpha * w[i];
        r[i] = ri;
        s += (double)ri * (double)ri;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// The single solve's iteration fuses the final sums into the vector updates:
// every workgroup adds the same partials in the same order, so all of them
// hold the same scalar, and workgroup 0 records it. rho alternates between
// two slots by the parity of k, so the workgroups that read rho_old never
// race the one that writes rho. The arithmetic is the one of the separate
// kernels above (which the batched iteration keeps), value for value.
__device__ inline int rho_slot(const double* sc, bool current) {
    const bool odd = ((long long)sc[SC_K] & 1) != 0;
    return (odd == current) ? SC_RHO2 : SC_RHO;
}

// rho = r.z (from the partials); beta = rho / rho_old (0 on the first
// iteration); p = z + beta p
template <typename T>
__global__ __launch_bounds__(VBS) void rho_update_p_kernel(int64_t n, const T* __restrict__ z, T* __restrict__ p,
                                                           const double* __restrict__ part, double* __restrict__ sc,
                                                           int* __restrict__ fl) {
    if (fl[FL_DONE]) return;
    const double rho = sum_parts(part);
    __shared__ double s_rho;
    if (threadIdx.x == 0) s_rho = rho;
    __syncthreads();
    const double r0 = s_rho;
    const bool first = fl[FL_FIRST] != 0;
    const double rho_old = sc[rho_slot(sc, false)];
    const double beta = first ? 0.0 : r0 / rho_old;
    const bool bad = !(r0 > 0.0) || !isfinite(r0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[rho_slot(sc, true)] = r0;
        sc[SC_RHO_OLD] = rho_old;
        sc[SC_BETA] = beta;
        if (bad) { fl[FL_BREAK] = 1; fl[FL_DONE] = 1; }
    }
    if (bad) return;
    const T b = (T)beta;
    for (int64_t i = blockIdx.x * (int64_t)VBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBS)
        p[i] = first ? z[i] : z[i] + b * p[i];
}

// alpha = rho / p.w (from the partials); x += alpha p; r -= alpha w; partials of r.r
template <typename T>
__global__ __launch_bounds__(VBS) void alpha_update_xr_kernel(int64_t n, T* __restrict__ x, T* __restrict__ r,
                                                              const T* __restrict__ p, const T* __restrict__ w,
                                                              const double* __restrict__ part_pw,
                                                              double* __restrict__ part_rr, double* __restrict__ sc,
                                                              int* __restrict__ fl) {
    if (fl[FL_DONE]) return;
    const double pw = sum_parts(part_pw);
    __shared__ double s_pw;
    if (threadIdx.x == 0) s_pw = pw;
    __syncthreads();
    const double pw0 = s_pw;
    const double al = sc[rho_slot(sc, true)] / pw0;
    const bool bad = !(pw0 > 0.0) || !isfinite(pw0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[SC_PW] = pw0;
        sc[SC_ALPHA] = al;
        if (bad) { fl[FL_BREAK] = 1; fl[FL_DONE] = 1; }
    }
    if (bad) return;
    const T alpha = (T)al;
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VBS + threadIdx.x; i < n; i += (int64_t)NPART * VBS) {
        x[i] += alpha * p[i];
        const T ri = r[i] - alpha * w[i];
        r[i] = ri;
        s += (double)ri * (double)ri;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = s;
}

// r = F - w
// r = F - w, or r = F when x was all zeros (then the product was skipped and
// w holds nothing)
__global__ void residual_kernel(int64_t n, const double* __restrict__ F, const double* __restrict__ w,
                                double* __restrict__ r, const int* __restrict__ xzero) {
    const bool zero = *xzero != 0;
    for (int64_t i = blockIdx.x * (int64_t)VBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBS)
        r[i] = zero ? F[i] : F[i] - w[i];
}

__global__ void set_flag_kernel(int* f, int v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *f = v;
}

// *f = 0 if any entry of x is nonzero (NaN counts as nonzero); every writer
// stores the same value
__global__ void clear_if_nonzero_kernel(int64_t n, const double* __restrict__ x, int* f) {
    bool nz = false;
    for (int64_t i = blockIdx.x * (int64_t)VBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBS)
        nz = nz || !(x[i] == 0.0);
    if (__any(nz) && (threadIdx.x & 63) == 0) atomicExch(f, 0);
}

// r32 = r * scale ; e32 = 0
__global__ void to_inner_kernel(int64_t n, const double* __restrict__ r, float* __restrict__ r32,
                                float* __restrict__ e32, double scale) {
    for (int64_t i = blockIdx.x * (int64_t)VBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBS) {
        r32[i] = (float)(r[i] * scale);
        e32[i] = 0.f;
    }
}

// x += scale e32
__global__ void refine_kernel(int64_t n, double* __restrict__ x, const float* __restrict__ e32, double scale) {
    for (int64_t i = blockIdx.x * (int64_t)VBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBS)
        x[i] += scale * (double)e32[i];
}

__global__ void init_scalars_kernel(double* sc, int* fl, double kmax, double ff, double thresh2) {
    if (threadIdx.x == 0) {
        for (int k = 0; k < SC_COUNT; ++k) sc[k] = 0.0;
        sc[SC_KMAX] = kmax;
        sc[SC_FF] = ff;
        sc[SC_THRESH2] = thresh2;
        fl[FL_DONE] = 0;
        fl[FL_BREAK] = 0;
        fl[FL_FIRST] = 1;
        fl[3] = 0;
    }
}

// restart: keep k, clear done, mark first iteration
__global__ void restart_kernel(int* fl) {
    if (threadIdx.x == 0) {
        fl[FL_DONE] = 0;
        fl[FL_BREAK] = 0;
        fl[FL_FIRST] = 1;
    }
}

static inline int vgrid(int64_t n) {
    int64_t g = (n + VBS - 1) / VBS;
    return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

// -------------------------------------------------------------- host -----
struct HostState {
    double sc[SC_COUNT];
    int fl[FL_COUNT];
};

static lgp_status read_state(const SolveWS& S, hipStream_t s, HostState& h) {
    LGP_HIP(hipMemcpyAsync(h.sc, S.sc, sizeof(h.sc), hipMemcpyDeviceToHost, s));
    LGP_HIP(hipMemcpyAsync(h.fl, S.fl, sizeof(h.fl), hipMemcpyDeviceToHost, s));
    LGP_HIP(hipStreamSynchronize(s));
    return LGP_OK;
}

// Inner or outer PCG loop on vectors of type T. `mv` computes w = K p.
template <typename T, typename MV, typename PC>
static lgp_status pcg_loop(int64_t n, T* x, T* r, T* z, T* p, T* w, SolveWS& S, int max_iter, int check_every,
                           MV mv, PC pc, hipStream_t s, int* iters_out, double* rr_out) {
    HostState h;
    lgp_status st;
    for (;;) {
        for (int it = 0; it < check_every; ++it) {
            if ((st = pc(r, z)) != LGP_OK) return st;
            // Alg. 1: rho = r.z, beta, p = z + beta p | w = K p | alpha = rho / p.w,
            // x += alpha p, r -= alpha w | ||r||, k += 1, stop test: five
            // vector kernels besides the product and the substitutions
            hipLaunchKernelGGL(dot_kernel<T>, dim3(NPART), dim3(VBS), 0, s, n, (const T*)r, (const T*)z, S.part,
                               (const int*)S.fl);
            hipLaunchKernelGGL(rho_update_p_kernel<T>, dim3(vgrid(n)), dim3(VBS), 0, s, n, (const T*)z, p,
                               (const double*)S.part, S.sc, S.fl);
            if ((st = mv(p, w)) != LGP_OK) return st;   // kernels return early once done
            hipLaunchKernelGGL(dot_kernel<T>, dim3(NPART), dim3(VBS), 0, s, n, (const T*)p, (const T*)w, S.part,
                               (const int*)S.fl);
            hipLaunchKernelGGL(alpha_update_xr_kernel<T>, dim3(NPART), dim3(VBS), 0, s, n, x, r, (const T*)p,
                               (const T*)w, (const double*)S.part, S.part + NPART, S.sc, S.fl);
            hipLaunchKernelGGL(fin_rr_kernel, dim3(1), dim3(VBS), 0, s, (const double*)(S.part + NPART), S.sc, S.fl,
                               1);
            LGP_CHECK_LAUNCH();
        }
        if ((st = read_state(S, s, h)) != LGP_OK) return st;
        if (h.fl[FL_DONE]) break;
        if ((int)h.sc[SC_K] >= max_iter) break;
    }
    *iters_out = (int)h.sc[SC_K];
    *rr_out = h.sc[SC_RR];
    if (h.fl[FL_BREAK]) return LGP_E_BREAKDOWN;
    return LGP_OK;
}

// ||F||^2 into sc[SC_FF], threshold eps^2 ||F||^2
static lgp_status norm2_into(const double* v, int64_t n, SolveWS& S, double eps, hipStream_t s) {
    hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, s, S.sc, S.fl, 0.0, 0.0, 0.0);
    hipLaunchKernelGGL(dot_kernel<double>, dim3(NPART), dim3(VBS), 0, s, n, v, v, S.part, (const int*)S.fl);
    hipLaunchKernelGGL(fin_ff_kernel, dim3(1), dim3(VBS), 0, s, (const double*)S.part, S.sc, eps * eps);
    LGP_CHECK_LAUNCH();
    return LGP_OK;
}

// r = F - K x in FP64 and ||r|| / ||F|| (read back; synchronises)
static lgp_status true_residual_ws(Problem& P, SolveWS& S, const double* F, const double* x, double normF,
                                   hipStream_t s, double* relres) {
    const int64_t n = P.n;
    lgp_status st2;
    // K x is skipped when x is all zeros (the usual x_0): a flag set on
    // the device, read by the contractions and the residual kernel
    int* xzero = S.fl + FL_XZERO;
    hipLaunchKernelGGL(set_flag_kernel, dim3(1), dim3(64), 0, s, xzero, 1);
    hipLaunchKernelGGL(clear_if_nonzero_kernel, dim3(vgrid(n)), dim3(VBS), 0, s, n, x, xzero);
    if ((st2 = matvec_f64(P, x, S.w, s, xzero)) != LGP_OK) return st2;
    hipLaunchKernelGGL(residual_kernel, dim3(vgrid(n)), dim3(VBS), 0, s, n, F, (const double*)S.w, S.r,
                       (const int*)xzero);
    hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, s, S.sc, S.fl, 0.0, 0.0, 0.0);
    hipLaunchKernelGGL(dot_kernel<double>, dim3(NPART), dim3(VBS), 0, s, n, (const double*)S.r,
                       (const double*)S.r, S.part, (const int*)S.fl);
    hipLaunchKernelGGL(fin_ff_kernel, dim3(1), dim3(VBS), 0, s, (const double*)S.part, S.sc, 0.0);
    LGP_CHECK_LAUNCH();
    HostState h2;
    if ((st2 = read_state(S, s, h2)) != LGP_OK) return st2;
    *relres = sqrt(h2.sc[SC_FF]) / normF;
    return LGP_OK;
}

lgp_status pcg_solve_impl(Problem& P, Factor& M, const double* F, double* x, const lgp_solve_opts& o, void* ws,
                          size_t ws_bytes, hipStream_t s, lgp_solve_info* info) {
    const int64_t n = P.n;
    const bool mixed = (o.inner != LGP_F64);
    SolveWS S;
    if (plan_ws(S, n, mixed, ws) > ws_bytes) return LGP_E_NOMEM;
    if (mixed && M.kind != 0) return LGP_E_UNSUPPORTED;
    if (mixed && !M.has32) return LGP_E_ARG;
    if (!mixed && !M.has64) return LGP_E_UNSUPPORTED;   // factor kept in FP32 only
    lgp_status st;
    info->iters = 0;
    info->outer = 0;
    info->relres_true = NAN;
    info->relres_recursive = NAN;
    info->status = LGP_OK;
    HostState h;

    // ||F||
    if ((st = norm2_into(F, n, S, o.rtol, s)) != LGP_OK) return st;
    if ((st = read_state(S, s, h)) != LGP_OK) return st;
    const double normF = sqrt(h.sc[SC_FF]);
    // a NaN or an infinity in F makes ||F|| non-finite: the stop rule of
    // Alg. 1 can never be met, so the request is rejected
    if (!std::isfinite(normF)) {
        info->status = LGP_E_ARG;
        return LGP_E_ARG;
    }
    if (!(normF > 0.0)) {
        // F = 0: x = 0 is the solution
        LGP_HIP(hipMemsetAsync(x, 0, n * 8, s));
        LGP_HIP(hipStreamSynchronize(s));
        info->relres_true = 0.0;
        info->relres_recursive = 0.0;
        return LGP_OK;
    }
    auto true_residual = [&](double* relres) -> lgp_status {
        return true_residual_ws(P, S, F, x, normF, s, relres);
    };

    double relres = 0.0;
    if ((st = true_residual(&relres)) != LGP_OK) return st;
    // a non-finite initial guess gives a non-finite residual
    if (!std::isfinite(relres)) {
        info->relres_true = relres;
        info->status = LGP_E_ARG;
        return LGP_E_ARG;
    }
    const int check_every = o.check_every > 0 ? o.check_every : 4;

    if (!mixed) {
        int restarts = 0;
        int total = 0;
        double rr = 0.0;
        while (relres > o.rtol) {
            if (total >= o.max_iter || restarts > 3) break;
            // fresh scalars; r already = F - K x
            // fresh scalars; the stop rule uses ||F||, not ||r0|| (Alg. 1)
            hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, s, S.sc, S.fl,
                               (double)(o.max_iter - total), normF * normF, o.rtol * o.rtol * normF * normF);
            LGP_CHECK_LAUNCH();
            int it = 0;
            st = pcg_loop<double>(
                n, x, S.r, S.z, S.p, S.w, S, o.max_iter - total, check_every,
                [&](const double* pp, double* ww) { return matvec_f64(P, pp, ww, s, S.fl); },
                [&](const double* rr_, double* zz) {
                    if (M.kind == 1) return const_apply(M, rr_, zz, s);
                    lgp_status a = sweep(M, false, rr_, M.y_tmp, s, S.fl);
                    if (a != LGP_OK) return a;
                    return sweep(M, true, M.y_tmp, zz, s, S.fl);
                },
                s, &it, &rr);
            total += it;
            if (st != LGP_OK) {
                info->iters = total;
                info->status = st;
                return st;
            }
            lgp_status st2 = true_residual(&relres);
            if (st2 != LGP_OK) return st2;
            info->relres_recursive = sqrt(rr) / normF;
            if (relres > o.rtol) ++restarts;
        }
        info->iters = total;
        info->outer = restarts;
        info->relres_true = relres;
        if (!std::isfinite(relres)) {
            info->status = LGP_E_BREAKDOWN;
            return LGP_E_BREAKDOWN;
        }
        if (relres > o.rtol) {
            info->status = LGP_E_NOCONV;
            return LGP_E_NOCONV;
        }
        return LGP_OK;
    }

    // mixed precision: FP64 iterative refinement around an inner PCG
    const GemmMode mode = (o.inner == LGP_BF16) ? GEMM_BF16 : GEMM_F32;
    int outer = 0, total = 0;
    while (relres > o.rtol && outer < o.max_outer && total < o.max_iter) {
        // S.r holds F - K x (from true_residual); its norm^2 is in sc[SC_FF]
        const double rnorm = relres * normF;
        hipLaunchKernelGGL(to_inner_kernel, dim3(vgrid(n)), dim3(VBS), 0, s, n, (const double*)S.r, S.r32, S.e32,
                           1.0 / rnorm);
        // the inner right-hand side has unit norm
        hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, s, S.sc, S.fl, (double)(o.max_iter - total),
                           1.0, o.inner_rtol * o.inner_rtol);
        LGP_CHECK_LAUNCH();
        int it = 0;
        double rr = 0.0;
        st = pcg_loop<float>(
            n, S.e32, S.r32, S.z32, S.p32, S.w32, S, o.max_iter - total, check_every,
            [&](const float* pp, float* ww) { return matvec_lp(P, pp, ww, mode, s, S.fl); },
            [&](const float* rr_, float* zz) {
                lgp_status a = sweep32(M, false, rr_, S.y32, s, S.fl);
                if (a != LGP_OK) return a;
                return sweep32(M, true, S.y32, zz, s, S.fl);
            },
            s, &it, &rr);
        total += it;
        if (st != LGP_OK && st != LGP_E_BREAKDOWN) return st;
        // x += |r| e
        hipLaunchKernelGGL(refine_kernel, dim3(vgrid(n)), dim3(VBS), 0, s, n, x, (const float*)S.e32, rnorm);
        LGP_CHECK_LAUNCH();
        ++outer;
        lgp_status st2 = true_residual(&relres);
        if (st2 != LGP_OK) return st2;
        info->relres_recursive = sqrt(rr);
        if (it == 0) break;   // inner solver made no progress
    }
    info->iters = total;
    info->outer = outer;
    info->relres_true = relres;
    if (!std::isfinite(relres)) {
        info->status = LGP_E_BREAKDOWN;
        return LGP_E_BREAKDOWN;
    }
    if (relres > o.rtol) {
        info->status = LGP_E_NOCONV;
        return LGP_E_NOCONV;
    }
    return LGP_OK;
}


// ------------------------------------------------------------ batches ----
// PCG (Alg. 1) on several requests of one grid shape at once. Each slot has
// its own vectors, partial sums, scalars and flags; one iteration is the
// single-request sequence with every kernel covering all running slots
// (blockIdx.y = slot) and the substitutions of all slots in one launch, so
// each slot computes exactly what lgp_pcg_solve computes for it. The
// iteration is captured once as a HIP graph per set of running slots and
// replayed; slots that have converged skip their work through their flags.

struct VSlot {
    double* x;
    double* r;
    double* z;
    double* p;
    double* w;
    double* part;
    double* sc;
    int* fl;
};

__global__ __launch_bounds__(VBS) void bdot_kernel(int64_t n, const VSlot* __restrict__ vs, int which) {
    const VSlot v = vs[blockIdx.y];
    if (v.fl[FL_DONE]) return;
    const double* a = which == 0 ? v.r : v.p;
    const double* b = which == 0 ? v.z : v.w;
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VBS + threadIdx.x; i < n; i += (int64_t)NPART * VBS) s += a[i] * b[i];
    s = block_sum(s);
    if (threadIdx.x == 0) v.part[blockIdx.x] = s;
}

__global__ __launch_bounds__(VBS) void bfin_rho_kernel(const VSlot* __restrict__ vs) {
    const VSlot v = vs[blockIdx.x];
    double* sc = v.sc;
    int* fl = v.fl;
    if (fl[FL_DONE]) return;
    const double s = sum_parts(v.part);
    if (threadIdx.x == 0) {
        sc[SC_RHO_OLD] = sc[SC_RHO];
        sc[SC_RHO] = s;
        if (fl[FL_FIRST]) sc[SC_BETA] = 0.0;
        else sc[SC_BETA] = s / sc[SC_RHO_OLD];
        if (!(s > 0.0) || !isfinite(s)) { fl[FL_BREAK] = 1; fl[FL_DONE] = 1; }
    }
}

__global__ __launch_bounds__(VBS) void bfin_alpha_kernel(const VSlot* __restrict__ vs) {
    const VSlot v = vs[blockIdx.x];
    double* sc = v.sc;
    int* fl = v.fl;
    if (fl[FL_DONE]) return;
    const double s = sum_parts(v.part);
    if (threadIdx.x == 0) {
        sc[SC_PW] = s;
        sc[SC_ALPHA] = sc[SC_RHO] / s;
        if (!(s > 0.0) || !isfinite(s)) { fl[FL_BREAK] = 1; fl[FL_DONE] = 1; }
    }
}

__global__ __launch_bounds__(VBS) void bfin_rr_kernel(const VSlot* __restrict__ vs) {
    const VSlot v = vs[blockIdx.x];
    double* sc = v.sc;
    int* fl = v.fl;
    if (fl[FL_DONE]) return;
    const double s = sum_parts(v.part);
    if (threadIdx.x == 0) {
        sc[SC_RR] = s;
        sc[SC_K] += 1.0;
        fl[FL_FIRST] = 0;
        if (s <= sc[SC_THRESH2] || sc[SC_K] >= sc[SC_KMAX]) fl[FL_DONE] = 1;
        if (!isfinite(s)) { fl[FL_BREAK] = 1; fl[FL_DONE] = 1; }
    }
}

__global__ __launch_bounds__(VBS) void bupdate_p_kernel(int64_t n, const VSlot* __restrict__ vs) {
    const VSlot v = vs[blockIdx.y];
    if (v.fl[FL_DONE]) return;
    const bool first = v.fl[FL_FIRST] != 0;
    const double beta = v.sc[SC_BETA];
    for (int64_t i = blockIdx.x * (int64_t)VBS + threadIdx.x; i < n; i += (int64_t)gridDim.x * VBS)
        v.p[i] = first ? v.z[i] : v.z[i] + beta * v.p[i];
}

__global__ __launch_bounds__(VBS) void bupdate_xr_kernel(int64_t n, const VSlot* __restrict__ vs) {
    const VSlot v = vs[blockIdx.y];
    if (v.fl[FL_DONE]) return;
    const double alpha = v.sc[SC_ALPHA];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)VBS + threadIdx.x; i < n; i += (int64_t)NPART * VBS) {
        v.x[i] += alpha * v.p[i];
        const double ri = v.r[i] - alpha * v.w[i];
        v.r[i] = ri;
        s += ri * ri;
    }
    s = block_sum(s);
    if (threadIdx.x == 0) v.part[blockIdx.x] = s;
}

struct BatchSlot {
    int state = 0;          // 0 free, 1 running, 2 finished
    Problem* P = nullptr;
    Factor* M = nullptr;
    const double* F = nullptr;
    double* x = nullptr;
    lgp_solve_opts o{};
    double normF = 0.0;
    int total = 0, restarts = 0;
    lgp_solve_info info{};
    SolveWS S{};            // this slot's vectors and scalars in the batch workspace
    double* y = nullptr;    // forward-substitution output
    unsigned* prog = nullptr;
};

struct Batch {
    int d = 0, N = 0, cap = 0;
    int64_t n = 0;
    hipStream_t s = nullptr;
    std::vector<int> offs;  // pattern of the first factor (every slot must match)
    int nlo = 0, ldl = 0, layout = 0;
    std::vector<BatchSlot> slot;
    VSlot* dv = nullptr;               // device: running slots' pointers, in running order
    SweepSlot<double>* dfw = nullptr;  // device: forward / backward substitution tables
    SweepSlot<double>* dbw = nullptr;
    unsigned* tick = nullptr;
    std::vector<int> run;              // running slot ids in the order of the device tables
    hipGraphExec_t gexec = nullptr;
    bool tables_dirty = true;
    bool sweep_batched = true;
    int iters_since_capture = 0;
    std::vector<VSlot> hv;             // host copies of the device tables (kept until copied)
    std::vector<SweepSlot<double>> hfw, hbw;
};

static size_t plan_batch(Batch& B, int64_t n, int nlines, int cap, void* buf) {
    Carver c(buf);
    B.slot.assign(cap, BatchSlot());
    for (int k = 0; k < cap; ++k) {
        BatchSlot& sl = B.slot[k];
        plan_ws(sl.S, n, false, nullptr);   // layout only
        sl.S.r = c.take<double>(n);
        sl.S.z = c.take<double>(n);
        sl.S.p = c.take<double>(n);
        sl.S.w = c.take<double>(n);
        sl.S.part = c.take<double>(NPART);
        sl.S.sc = c.take<double>(SC_COUNT);
        sl.S.fl = c.take<int>(FL_COUNT);
        sl.y = c.take<double>(n);
        sl.prog = c.take<unsigned>(nlines > 0 ? nlines : 1);
    }
    B.dv = c.take<VSlot>(cap);
    B.dfw = c.take<SweepSlot<double>>(cap);
    B.dbw = c.take<SweepSlot<double>>(cap);
    B.tick = c.take<unsigned>(4);
    return c.off + 256;
}

size_t batch_ws_bytes(int64_t n, int nlines, int cap) {
    Batch B;
    return plan_batch(B, n, nlines, cap, nullptr);
}

Batch* batch_create(Problem& shape, int cap, void* ws, size_t ws_bytes, hipStream_t s, lgp_status* st) {
    const int nlines = shape.d == 3 ? shape.n1 * shape.n1 : (shape.d == 2 ? shape.n1 : 1);
    if (batch_ws_bytes(shape.n, nlines, cap) > ws_bytes) {
        *st = LGP_E_NOMEM;
        return nullptr;
    }
    Batch* B = new (std::nothrow) Batch();
    if (!B) {
        *st = LGP_E_NOMEM;
        return nullptr;
    }
    B->d = shape.d;
    B->N = shape.N;
    B->n = shape.n;
    B->cap = cap;
    B->s = s;
    plan_batch(*B, shape.n, nlines, cap, ws);
    *st = LGP_OK;
    return B;
}

void batch_destroy(Batch* B) {
    if (!B) return;
    if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
    (void)hipStreamSynchronize(B->s);
    delete B;
}

// admission: ||F||, the true residual of x_0 and the first scalars, with the
// single-request kernels on the slot's workspace (synchronises)
lgp_status batch_add(Batch* B, Problem& P, Factor& M, const double* F, double* x, const lgp_solve_opts& o, int* out) {
    if (P.d != B->d || P.N != B->N || M.P != &P || M.kind != 0 || !M.has64) return LGP_E_ARG;
    if (!B->offs.empty() && (M.offs != B->offs || M.nlo != B->nlo || M.ldl != B->ldl || M.layout != B->layout))
        return LGP_E_UNSUPPORTED;   // another pattern: another batch
    int k = 0;
    while (k < B->cap && B->slot[k].state == 1) ++k;
    if (k == B->cap) return LGP_E_NOMEM;
    if (B->offs.empty()) {
        B->offs = M.offs;
        B->nlo = M.nlo;
        B->ldl = M.ldl;
        B->layout = M.layout;
    }
    BatchSlot& sl = B->slot[k];
    sl.P = &P;
    sl.M = &M;
    sl.F = F;
    sl.x = x;
    sl.o = o;
    sl.total = 0;
    sl.restarts = 0;
    sl.info = lgp_solve_info{0, 0, NAN, NAN, LGP_OK};
    hipStream_t s = B->s;
    lgp_status st;
    HostState h;
    if ((st = norm2_into(F, P.n, sl.S, o.rtol, s)) != LGP_OK) return st;
    if ((st = read_state(sl.S, s, h)) != LGP_OK) return st;
    sl.normF = sqrt(h.sc[SC_FF]);
    *out = k;
    if (!std::isfinite(sl.normF)) {
        sl.state = 2;
        sl.info.status = LGP_E_ARG;
        return LGP_OK;
    }
    if (!(sl.normF > 0.0)) {   // F = 0: x = 0
        LGP_HIP(hipMemsetAsync(x, 0, P.n * 8, s));
        LGP_HIP(hipStreamSynchronize(s));
        sl.info.relres_true = 0.0;
        sl.info.relres_recursive = 0.0;
        sl.state = 2;
        return LGP_OK;
    }
    double relres = 0.0;
    if ((st = true_residual_ws(P, sl.S, F, x, sl.normF, s, &relres)) != LGP_OK) return st;
    sl.info.relres_true = relres;
    if (!std::isfinite(relres)) {
        sl.state = 2;
        sl.info.status = LGP_E_ARG;
        return LGP_OK;
    }
    if (!(relres > o.rtol)) {
        sl.state = 2;
        return LGP_OK;
    }
    hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, s, sl.S.sc, sl.S.fl, (double)o.max_iter,
                       sl.normF * sl.normF, o.rtol * o.rtol * sl.normF * sl.normF);
    LGP_CHECK_LAUNCH();
    sl.state = 1;
    B->tables_dirty = true;
    return LGP_OK;
}

static lgp_status batch_tables(Batch* B) {
    B->run.clear();
    for (int k = 0; k < B->cap; ++k)
        if (B->slot[k].state == 1) B->run.push_back(k);
    const int S = (int)B->run.size();
    B->hv.resize(S);
    B->hfw.resize(S);
    B->hbw.resize(S);
    for (int t = 0; t < S; ++t) {
        BatchSlot& sl = B->slot[B->run[t]];
        B->hv[t] = VSlot{sl.x, sl.S.r, sl.S.z, sl.S.p, sl.S.w, sl.S.part, sl.S.sc, sl.S.fl};
        const Factor& M = *sl.M;
        const bool lay3 = M.layout == 1;
        B->hfw[t] = SweepSlot<double>{lay3 ? M.A64 : M.L, nullptr, sl.S.r, sl.y, sl.prog, sl.S.fl};
        B->hbw[t] = SweepSlot<double>{lay3 ? M.A64 : M.Ut, M.invD, sl.y, sl.S.z, sl.prog, sl.S.fl};
    }
    if (S > 0) {
        LGP_HIP(hipMemcpyAsync(B->dv, B->hv.data(), S * sizeof(VSlot), hipMemcpyHostToDevice, B->s));
        LGP_HIP(hipMemcpyAsync(B->dfw, B->hfw.data(), S * sizeof(SweepSlot<double>), hipMemcpyHostToDevice, B->s));
        LGP_HIP(hipMemcpyAsync(B->dbw, B->hbw.data(), S * sizeof(SweepSlot<double>), hipMemcpyHostToDevice, B->s));
        LGP_HIP(hipStreamSynchronize(B->s));   // the host tables may change after this
    }
    if (B->gexec) {
        (void)hipGraphExecDestroy(B->gexec);
        B->gexec = nullptr;
    }
    B->tables_dirty = false;
    return LGP_OK;
}

// one PCG iteration of every running slot, enqueued on the batch's stream
static lgp_status batch_iteration(Batch* B) {
    const int S = (int)B->run.size();
    const int64_t n = B->n;
    hipStream_t s = B->s;
    lgp_status st;
    const Factor& ref = *B->slot[B->run[0]].M;
    // z = U^{-1} L^{-1} r
    if (B->sweep_batched) {
        st = sweep_batch(ref, S, B->dfw, false, B->tick, s);
        if (st == LGP_OK) st = sweep_batch(ref, S, B->dbw, true, B->tick + 1, s);
        if (st == LGP_E_UNSUPPORTED) B->sweep_batched = false;
        else if (st != LGP_OK) return st;
    }
    if (!B->sweep_batched) {
        for (int t = 0; t < S; ++t) {
            BatchSlot& sl = B->slot[B->run[t]];
            if ((st = sweep(*sl.M, false, sl.S.r, sl.y, s, sl.S.fl)) != LGP_OK) return st;
            if ((st = sweep(*sl.M, true, sl.y, sl.S.z, s, sl.S.fl)) != LGP_OK) return st;
        }
    }
    hipLaunchKernelGGL(bdot_kernel, dim3(NPART, S), dim3(VBS), 0, s, n, (const VSlot*)B->dv, 0);
    hipLaunchKernelGGL(bfin_rho_kernel, dim3(S), dim3(VBS), 0, s, (const VSlot*)B->dv);
    hipLaunchKernelGGL(bupdate_p_kernel, dim3(vgrid(n), S), dim3(VBS), 0, s, n, (const VSlot*)B->dv);
    for (int t = 0; t < S; ++t) {
        BatchSlot& sl = B->slot[B->run[t]];
        if ((st = matvec_f64(*sl.P, sl.S.p, sl.S.w, s, sl.S.fl)) != LGP_OK) return st;
    }
    hipLaunchKernelGGL(bdot_kernel, dim3(NPART, S), dim3(VBS), 0, s, n, (const VSlot*)B->dv, 1);
    hipLaunchKernelGGL(bfin_alpha_kernel, dim3(S), dim3(VBS), 0, s, (const VSlot*)B->dv);
    hipLaunchKernelGGL(bupdate_xr_kernel, dim3(NPART, S), dim3(VBS), 0, s, n, (const VSlot*)B->dv);
    hipLaunchKernelGGL(bfin_rr_kernel, dim3(S), dim3(VBS), 0, s, (const VSlot*)B->dv);
    LGP_CHECK_LAUNCH();
    return LGP_OK;
}

// `iters` iterations of every running slot (the first after a change of the
// running set eagerly -- it also settles the contraction tile choices -- the
// others as replays of one captured graph), then per slot: a slot whose PCG
// has stopped gets its true residual, and restarts (at most 3) or finishes.
// Synchronises. *running: slots still running afterwards.
lgp_status batch_step(Batch* B, int iters, int* running) {
    lgp_status st;
    if (B->tables_dirty && (st = batch_tables(B)) != LGP_OK) return st;
    if (!B->run.empty()) {
        // graphs need a stream that can be captured (not the null stream)
        const char* g = std::getenv("LGP_BATCH_GRAPH");
        const bool use_graph = !(g && g[0] == '0') && B->s != nullptr;
        for (int it = 0; it < iters; ++it) {
            if (!use_graph || (!B->gexec && B->iters_since_capture == 0)) {
                if ((st = batch_iteration(B)) != LGP_OK) return st;
                ++B->iters_since_capture;
                continue;
            }
            if (!B->gexec) {
                hipGraph_t graph = nullptr;
                LGP_HIP(hipStreamBeginCapture(B->s, hipStreamCaptureModeThreadLocal));
                const lgp_status cst = batch_iteration(B);
                const hipError_t e = hipStreamEndCapture(B->s, &graph);
                if (cst != LGP_OK) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return cst;
                }
                if (e != hipSuccess) {
                    g_last_hip_error = (int)e;
                    return LGP_E_HIP;
                }
                const hipError_t e2 = hipGraphInstantiate(&B->gexec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e2 != hipSuccess) {
                    g_last_hip_error = (int)e2;
                    B->gexec = nullptr;
                    return LGP_E_HIP;
                }
            }
            LGP_HIP(hipGraphLaunch(B->gexec, B->s));
        }
    }
    LGP_HIP(hipStreamSynchronize(B->s));
    int still = 0;
    for (int k = 0; k < B->cap; ++k) {
        BatchSlot& sl = B->slot[k];
        if (sl.state != 1) continue;
        HostState h;
        if ((st = read_state(sl.S, B->s, h)) != LGP_OK) return st;
        if (!h.fl[FL_DONE]) {
            ++still;
            continue;
        }
        // this round of Alg. 1 has stopped
        sl.total += (int)h.sc[SC_K];
        sl.info.iters = sl.total;
        sl.info.relres_recursive = sqrt(h.sc[SC_RR]) / sl.normF;
        if (h.fl[FL_BREAK]) {
            sl.state = 2;
            sl.info.status = LGP_E_BREAKDOWN;
            B->tables_dirty = true;
            continue;
        }
        double relres = 0.0;
        if ((st = true_residual_ws(*sl.P, sl.S, sl.F, sl.x, sl.normF, B->s, &relres)) != LGP_OK) return st;
        sl.info.relres_true = relres;
        if (relres > sl.o.rtol && std::isfinite(relres) && sl.total < sl.o.max_iter && sl.restarts < 3) {
            ++sl.restarts;
            hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, B->s, sl.S.sc, sl.S.fl,
                               (double)(sl.o.max_iter - sl.total), sl.normF * sl.normF,
                               sl.o.rtol * sl.o.rtol * sl.normF * sl.normF);
            LGP_CHECK_LAUNCH();
            ++still;
            continue;   // stays in the running set (its tables are unchanged)
        }
        sl.info.outer = sl.restarts;
        sl.info.status = !std::isfinite(relres) ? LGP_E_BREAKDOWN : (relres > sl.o.rtol ? LGP_E_NOCONV : LGP_OK);
        sl.state = 2;
        B->tables_dirty = true;
    }
    if (B->tables_dirty) B->iters_since_capture = 0;
    *running = still;
    return LGP_OK;
}

lgp_status batch_info(Batch* B, int k, lgp_solve_info* info, int* finished) {
    if (k < 0 || k >= B->cap || B->slot[k].state == 0) return LGP_E_ARG;
    *info = B->slot[k].info;
    *finished = B->slot[k].state == 2;
    return LGP_OK;
}

lgp_status batch_remove(Batch* B, int k) {
    if (k < 0 || k >= B->cap || B->slot[k].state == 0) return LGP_E_ARG;
    if (B->slot[k].state == 1) B->tables_dirty = true;
    B->slot[k].state = 0;
    B->slot[k].P = nullptr;
    B->slot[k].M = nullptr;
    bool any = false;
    for (auto& sl : B->slot) any |= sl.state != 0;
    if (!any) B->offs.clear();   // an empty batch takes the next pattern
    return LGP_OK;
}

}  // namespace lgp

// Preconditioner of Sec. 4.1-4.2 on the GPU: truncated Legendre series of a
// and b, exact 1D band factors (Lemma LegProduct), NZ(M) as an offset
// stencil, ILU(0) (Alg. 2) in FP64, and the two substitutions of the
// one-step method (Alg. 3 and Alg. 4).
//
// Storage. NZ(M) is a symmetric set of offsets (dx,dy,dz), so ILU(0) of the
// symmetric M gives U = diag(U) L^T; only the strictly lower part of L
// (n_lower values per row, row-major, zero outside the grid) and the pivots
// D = diag(U) are kept. For the backward sweep a second array Ut holds, for
// the rows in reversed order, L(i - delta_k, i), so both sweeps stream their
// operator forward in memory with the same access pattern.
//
// Schedule. Row i depends on rows i + delta for lower offsets delta. With
// Hx, Hy the largest |dx|, |dy| of the pattern, the level
// l(i) = ix + (Hx+1) iy + (Hx+1)(Hy+1) iz strictly increases along every
// dependency, so rows of one level are independent (a hyperplane schedule).
//   * Factorisation: one wave per row, rows handed out in level order by an
//     atomic ticket, completion published by a per-row flag. Each row is
//     computed left-looking (offsets in column order), so only its last
//     offsets wait for recently finished rows.
//   * Sweeps: one workgroup per grid line (fixed iy, iz), lines handed out
//     in order of l, rows of a line in increasing ix; a line waits on the
//     progress counter of line (iy-1, iz) and of line (min(iy+Hy, n1-1),
//     iz-1), which by induction covers every other dependency.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>

#include "devutil.h"

namespace lgp {

// -------------------------------------------------- host: 1D factors -----
// int_{-1}^{1} L_t L_m L_n dx. With g = (t+m+n)/2 (nonzero only for t+m+n
// even and |m-n| <= t <= m+n) the product formula gives
//   2/(2g+1) * C_{g-m} C_{g-n} C_{g-t} / C_g,  C_r = (2r-1)!!/(r! 2^r).
// The large-index ratio C_{g-t}/C_g = prod_{r=g-t+1}^{g} 2r/(2r-1) has only
// t factors; C_{g-m}, C_{g-n} have small indices when t is small.
__host__ __device__ static inline double Cr(int r) {
    double c = 1.0;
    for (int i = 1; i <= r; ++i) c *= (2.0 * i - 1.0) / (2.0 * i);
    return c;
}

__host__ __device__ double triple_legendre(int t, int m, int n) {
    if (t < 0 || m < 0 || n < 0) return 0.0;
    if ((t + m + n) & 1) return 0.0;
    if (t > m + n || t < abs(m - n)) return 0.0;
    const int g = (t + m + n) / 2;
    // order so that the two small indices use direct products
    int small1 = g - m, small2 = g - n, big = g - t;
    // if t is the largest of the three, g-t is the smallest: swap roles so
    // that the ratio is taken against the smallest of (t, m, n)
    int lo = min(t, min(m, n));
    if (lo != t) {
        if (lo == m) { small1 = g - t; big = g - m; }
        else         { small2 = g - t; big = g - n; }
    }
    double ratio = 1.0;   // C_big / C_g = prod_{r=big+1}^{g} 2r/(2r-1)
    for (int r = big + 1; r <= g; ++r) ratio *= (2.0 * r) / (2.0 * r - 1.0);
    return 2.0 / (2.0 * g + 1.0) * Cr(small1) * Cr(small2) * ratio;
}

// S^(t)(i, m) = (2i+3)(2m+3) int L_t L_{i+1} L_{m+1}
__host__ __device__ static inline double S1(int t, int i, int m) { return (2.0 * i + 3) * (2.0 * m + 3) * triple_legendre(t, i + 1, m + 1); }
// M^(t)(i, m) = int L_t (L_i - L_{i+2}) (L_m - L_{m+2})
__host__ __device__ static inline double M1(int t, int i, int m) {
    return triple_legendre(t, i, m) - triple_legendre(t, i, m + 2) - triple_legendre(t, i + 2, m) +
           triple_legendre(t, i + 2, m + 2);
}

size_t plan_factor(Factor& F, void* buf, int store) {
    if (F.d == 3) return plan_factor3(F, buf, store);
    const bool with32 = (store != STORE_F64);
    F.has64 = true;
    F.layout = 0;
    Carver c(buf);
    const int64_t n = F.n;
    const int nlo = F.nlo;
    const int T = F.T, h = F.h, d = F.d, n1 = F.n1;
    int64_t tp = 1;
    for (int k = 0; k < d; ++k) tp *= (T + 1);
    F.ldl = ((nlo + 1) + 31) & ~31;
    const size_t ldl = (size_t)F.ldl;
    F.L = c.take<double>((size_t)(n + 1) * ldl);
    // Ut doubles as scratch before the transpose: the row order (n ints)
    // and the folded line coefficients, which on tiny grids outgrow n rows
    {
        const int W = 2 * h + 1, nzW = (d == 3) ? W : 1;
        const size_t scratch = (((size_t)n * 4 + 255) & ~(size_t)255) + (size_t)F.nlines * nzW * W * 2 * (T + 1) * 8;
        F.Ut = c.take<double>(std::max((size_t)n * ldl, (scratch + 7) / 8));
    }
    F.Dg = c.take<double>(n);
    F.invD = c.take<double>(n);
    F.has32 = with32;
    if (with32) {
        F.L32 = c.take<float>((size_t)n * ldl);
        F.Ut32 = c.take<float>((size_t)n * ldl);
        F.invD32 = c.take<float>(n);
    } else {
        F.L32 = F.Ut32 = F.invD32 = nullptr;
    }
    F.d_offs = c.take<int>((size_t)4 * (nlo + 1));
    F.line_order = c.take<int>(F.nlines);
    F.prog = c.take<unsigned>((size_t)2 * F.nlines);
    F.ticket = c.take<unsigned>(4);
    F.flag = c.take<int>(4);
    F.coefA = c.take<double>((size_t)d * tp);
    F.coefB = c.take<double>(tp);
    F.band = c.take<double>((size_t)2 * (T + 1) * n1 * (2 * h + 1));
    F.pair_ptr = c.take<int>(nlo + 2);
    F.pair_j = c.take<int>(F.npairs > 0 ? F.npairs : 1);
    F.pair_l = c.take<int>(F.npairs > 0 ? F.npairs : 1);
    F.steps = c.take<int>((size_t)4 * (nlo + 1));
    F.sdxyz = c.take<int>(nlo + 1);
    F.pairw = c.take<unsigned>(F.npairs > 0 ? F.npairs : 1);
    {
        const int64_t A1 = F.Hx + 1, B1 = (int64_t)(F.Hx + 1) * (F.Hy + 1);
        F.maxlev = (int)((n1 - 1) * (1 + A1 + (d == 3 ? B1 : 0)) + 1);
    }
    F.lev = c.take<int>((size_t)2 * F.maxlev + 2);
    F.runs = c.take<int>((size_t)4 * (nlo + 1));
    F.y_tmp = c.take<double>(n);
    F.bytes = c.off + 256;
    return F.bytes;
}

struct RowGeo {
    int n1, d;
    int64_t n;
};

// ------------------------------------------------- coefficient fold ------
// For line (iy, iz) and every (dy, dz) in [-h, h]^2 (dz = 0 in 2D) and x
// degree t <= T:
//   Fa[t] = sum_{r,s} a_{r s t} M^(r)(iz, iz+dz) M^(s)(iy, iy+dy)
//   Fb[t] = sum_{r,s} a_{r s t} [M^(r)_z S^(s)_y + S^(r)_z M^(s)_y] + b_{r s t} M^(r)_z M^(s)_y
// so that M(i, i+delta) = sum_t S^(t)(ix, ix+dx) Fa[t] + M^(t)(ix, ix+dx) Fb[t]
// (Kronecker form of Sec. 4.2; in 2D the z factors are 1 and r = 0). The
// term with S in direction j carries a_j's series (coefA + j (T+1)^d), so
// the same fold serves the isotropic form (three equal series) and the
// anisotropic one of Example 4.
// Layout: fold[line][(dz+h)*(2h+1) + (dy+h)][2][T+1].
__global__ void fold_kernel(int d, int n1, int T, int h, const double* __restrict__ band,
                            const double* __restrict__ coefA, const double* __restrict__ coefB,
                            double* __restrict__ fold, int nlines) {
    const int W = 2 * h + 1;
    const int T1 = T + 1;
    const int64_t bandT = (int64_t)n1 * W;          // stride between t
    const double* Sb = band;                         // S^(t)(i, i+delta)
    const double* Mb = band + (int64_t)T1 * bandT;   // M^(t)(i, i+delta)
    const int nz = (d == 3) ? W : 1;
    const int64_t tp = (d == 3) ? (int64_t)T1 * T1 * T1 : (int64_t)T1 * T1;
    for (int line = blockIdx.x; line < nlines; line += gridDim.x) {
        const int iy = line % n1, iz = line / n1;
        const int combos = nz * W * T1;
        for (int c = threadIdx.x; c < combos; c += blockDim.x) {
            const int t = c % T1;
            const int dyi = (c / T1) % W;
            const int dzi = c / (T1 * W);
            const int dy = dyi - h;
            const int dz = (d == 3) ? dzi - h : 0;
            double fa = 0.0, fb = 0.0;
            const bool yin = (iy + dy >= 0 && iy + dy < n1);
            const bool zin = (d == 2) || (iz + dz >= 0 && iz + dz < n1);
            if (yin && zin) {
                const int R = (d == 3) ? T1 : 1;
                for (int r = 0; r < R; ++r) {
                    double mz = 1.0, sz = 0.0;
                    if (d == 3) {
                        mz = Mb[r * bandT + (int64_t)iz * W + (dz + h)];
                        sz = Sb[r * bandT + (int64_t)iz * W + (dz + h)];
                    }
                    for (int s = 0; s < T1; ++s) {
                        const double my = Mb[s * bandT + (int64_t)iy * W + (dy + h)];
                        const double sy = Sb[s * bandT + (int64_t)iy * W + (dy + h)];
                        const int64_t ci = ((int64_t)r * T1 + s) * T1 + t;   // x fastest
                        const double ax = coefA[ci], ay = coefA[tp + ci];
                        const double az = (d == 3) ? coefA[2 * tp + ci] : 0.0, b = coefB[ci];
                        fa += ax * mz * my;
                        fb += ay * mz * sy + az * sz * my + b * mz * my;
                    }
                }
            }
            double* o = fold + (int64_t)line * nz * W * 2 * T1 + ((int64_t)(dzi * W + dyi) * 2) * T1;
            o[t] = fa;
            o[T1 + t] = fb;
        }
    }
}

// ---------------------------------------------------- factorisation ------
// One wave per row. LDS: u[0..nlo] (u[nlo] = diagonal), offsets table.
__global__ __launch_bounds__(64) void ilu_factor_kernel(
    int d, int n1, int64_t n, int nlo, int ldl, int T, int h, const int4* __restrict__ offs,
    const int* __restrict__ row_order, const double* __restrict__ band, const double* __restrict__ fold,
    const int* __restrict__ pair_ptr, const int* __restrict__ pair_k, const int* __restrict__ pair_l,
    double* __restrict__ L, double* __restrict__ Dg, double* __restrict__ invD, unsigned* done,
    unsigned* ticket, int* flag) {
    extern __shared__ double u[];   // nlo + 1
    __shared__ int s_row;
    const int lane = threadIdx.x;
    const int W = 2 * h + 1;
    const int T1 = T + 1;
    const int64_t bandT = (int64_t)n1 * W;
    const int nzW = (d == 3) ? W : 1;
    for (;;) {
        if (lane == 0) {
            unsigned tk = atomicAdd(ticket, 1u);
            s_row = (tk < (unsigned)n) ? row_order[tk] : -1;
        }
        __syncthreads();
        const int64_t i = s_row;
        __syncthreads();
        if (i < 0) break;
        const int ix = (int)(i % n1);
        const int iy = (int)((i / n1) % n1);
        const int iz = (d == 3) ? (int)(i / ((int64_t)n1 * n1)) : 0;
        const int64_t line = i / n1;
        const double* fl = fold + line * (int64_t)nzW * W * 2 * T1;
        // M(i, i + delta_k) for lower offsets and the diagonal
        for (int k = lane; k <= nlo; k += 64) {
            const int4 o = offs[k];
            double v = 0.0;
            const int cx = ix + o.x, cy = iy + o.y, cz = iz + o.z;
            if (cx >= 0 && cx < n1 && cy >= 0 && cy < n1 && cz >= 0 && cz < n1) {
                const double* f = fl + ((int64_t)((o.z + h) * (d == 3 ? 1 : 0) * W + (o.y + h)) * 2) * T1;
                for (int t = 0; t < T1; ++t)
                    v += band[t * bandT + (int64_t)ix * W + (o.x + h)] * f[t] +
                         band[(T1 + t) * bandT + (int64_t)ix * W + (o.x + h)] * f[T1 + t];
            }
            u[k] = v;
        }
        __syncthreads();
        // left-looking (Alg. 2 with U = D L^T): u_j = L(i,j) D(i+dj) =
        // M(i,j) - sum_{k<j} u_k L(i+dj, i+dk); L(i,j) = u_j / D(i+dj) later
        for (int j = 0; j < nlo; ++j) {
            const int4 oj = offs[j];
            const int cx = ix + oj.x, cy = iy + oj.y, cz = iz + oj.z;
            const bool in = (cx >= 0 && cx < n1 && cy >= 0 && cy < n1 && cz >= 0 && cz < n1);
            if (!in) continue;   // uniform across the wave
            const int64_t rj = i + oj.w;
            if (lane == 0) {
                while (ld_coh(&done[rj]) == 0u) __builtin_amdgcn_s_sleep(1);
            }
            __syncthreads();
            compiler_fence();
            double acc = 0.0;
            const double* Lj = L + rj * ldl;
            for (int p = pair_ptr[j] + lane; p < pair_ptr[j + 1]; p += 64)
                acc += u[pair_k[p]] * ld_coh(&Lj[pair_l[p]]);
            acc = wave_sum(acc);
            if (lane == 0) u[j] = u[j] - acc;
            __syncthreads();
        }
        // pivot: D(i) = M(i,i) - sum_k u_k L(i,k),  L(i,k) = u_k / D(i+dk)
        double acc = 0.0;
        for (int k = lane; k < nlo; k += 64) {
            const int4 o = offs[k];
            const int cx = ix + o.x, cy = iy + o.y, cz = iz + o.z;
            const bool in = (cx >= 0 && cx < n1 && cy >= 0 && cy < n1 && cz >= 0 && cz < n1);
            double lk = 0.0;
            if (in) {
                lk = u[k] / ld_coh(&Dg[i + o.w]);
                acc += u[k] * lk;
            }
            st_coh(&L[i * ldl + k], lk);
        }
        acc = wave_sum(acc);
        if (lane == 0) {
            const double piv = u[nlo] - acc;
            if (!(piv > 0.0) || !isfinite(piv)) atomicOr(flag, 1);
            st_coh(&Dg[i], piv);
            invD[i] = 1.0 / piv;
            L[i * ldl + nlo] = 1.0 / piv;
        }
        __syncthreads();
        if (lane == 0) publish(&done[i], 1u);
        __syncthreads();
    }
}

// 1D band tables: band[t][i][delta+h] = S^(t)(i, i+delta), band[T+1+t][i][delta+h]
// = M^(t)(i, i+delta) (Lemma LegProduct), zero outside 0 <= i+delta < n1.
__global__ void band_kernel(int T, int n1, int h, double* __restrict__ band) {
    const int W = 2 * h + 1, T1 = T + 1;
    const int64_t total = (int64_t)T1 * n1 * W;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int dl = (int)(e % W) - h;
        const int i = (int)((e / W) % n1);
        const int t = (int)(e / ((int64_t)W * n1));
        const int m = i + dl;
        const bool in = m >= 0 && m < n1;
        band[e] = in ? S1(t, i, m) : 0.0;
        band[e + total] = in ? M1(t, i, m) : 0.0;
    }
}

// Rows in nondecreasing hyperplane level l = ix + A1 iy + B1 iz: row i goes
// to start[l] + (its rank among the rows of level l, taken by an atomic
// counter; rows of one level are independent, so their order is free).
__global__ void level_order_kernel(int d, int n1, int64_t n, int A1, int B1, const int* __restrict__ start,
                                   int* fill, int* __restrict__ order) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int ix = (int)(i % n1), iy = (int)((i / n1) % n1);
        const int iz = (d == 3) ? (int)(i / ((int64_t)n1 * n1)) : 0;
        const int l = ix + A1 * iy + B1 * iz;
        order[start[l] + atomicAdd(&fill[l], 1)] = (int)i;
    }
}

// Row padding of the factor storage: entries [from, ldl) of every row are
// set to zero (the substitution kernels read whole 32-entry groups).
__global__ void zero_pad_kernel(int64_t rows, int ldl, int from, double* __restrict__ M) {
    const int w = ldl - from;
    const int64_t total = rows * w;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        M[(e / w) * ldl + from + (e % w)] = 0.0;
}

// Backward-sweep operator in reversed row order: Ut[i'][k] = L(i - delta_k, i)
// with i = n-1-i'. Tiled: a workgroup takes R consecutive output rows and
// one run of offsets with equal (dy, dz) (consecutive k, dx ascending); the
// source entries then lie in R + span consecutive rows of L and the run's
// columns, staged through LDS so reads and writes are row segments.
__global__ __launch_bounds__(256) void build_ut_tiled_kernel(int d, int n1, int64_t n, int ldl,
                                                             const int4* __restrict__ offs,
                                                             const int4* __restrict__ runs, int R,
                                                             const double* __restrict__ L,
                                                             double* __restrict__ Ut) {
    extern __shared__ double tile[];
    const int4 run = runs[blockIdx.y];   // {kb, ke, dx of kb, dx of ke-1}
    const int kb = run.x, K = run.y - run.x, dxlo = run.z, dxhi = run.w;
    const int span = dxhi - dxlo;
    const int4 o0 = offs[kb];
    const int64_t base = (int64_t)n1 * o0.y + (int64_t)n1 * n1 * o0.z;   // linear offset without dx
    const int64_t p0 = (int64_t)blockIdx.x * R;
    const int64_t rmin = n - 1 - (p0 + R - 1) - base - dxhi;
    const int rows = R + span;
    for (int e = threadIdx.x; e < rows * K; e += blockDim.x) {
        const int rr = e / K, c = e - rr * K;
        const int64_t r = rmin + rr;
        tile[e] = (r >= 0 && r < n) ? L[r * ldl + kb + c] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < R * K; e += blockDim.x) {
        const int pr = e / K, c = e - pr * K;
        const int64_t ip = p0 + pr;
        if (ip >= n) continue;
        const int64_t i = n - 1 - ip;
        const int4 o = offs[kb + c];
        const int ix = (int)(i % n1), iy = (int)((i / n1) % n1);
        const int iz = (d == 3) ? (int)(i / ((int64_t)n1 * n1)) : 0;
        const int cx = ix - o.x, cy = iy - o.y, cz = iz - o.z;
        const bool in = cx >= 0 && cx < n1 && cy >= 0 && cy < n1 && cz >= 0 && cz < n1;
        const int64_t r = i - o.x - base;
        Ut[ip * ldl + kb + c] = in ? tile[(r - rmin) * K + c] : 0.0;
    }
}

// Backward-sweep operator in reversed row order: Ut[i'][k] = L(i - delta_k, i)
// with i = n-1-i' (untiled form, for patterns whose runs do not fit LDS).
__global__ void build_ut_kernel(int d, int n1, int64_t n, int nlo, int ldl, const int4* __restrict__ offs,
                                const double* __restrict__ L, double* __restrict__ Ut) {
    const int64_t total = n * nlo;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ip = e / nlo;
        const int k = (int)(e % nlo);
        const int64_t i = n - 1 - ip;
        const int ix = (int)(i % n1), iy = (int)((i / n1) % n1);
        const int iz = (d == 3) ? (int)(i / ((int64_t)n1 * n1)) : 0;
        const int4 o = offs[k];
        const int cx = ix - o.x, cy = iy - o.y, cz = iz - o.z;
        double v = 0.0;
        if (cx >= 0 && cx < n1 && cy >= 0 && cy < n1 && cz >= 0 && cz < n1) v = L[(i - o.w) * ldl + k];
        Ut[ip * ldl + k] = v;
    }
}

__global__ void to_f32_kernel(int64_t count, const double* __restrict__ a, float* __restrict__ b) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        b[e] = (float)a[e];
}

// ---------------------------------------------------------- sweeps -------
// out[r] = in[r] * s[r] - sum_k A[r'][k] out[r + sign*delta_k]   (r' the
// stream position: r' = r forward, r' = n-1-r backward). Rows of a line run
// in increasing stream order. NT threads per line.
template <typename T, int NT, bool REV, bool SCALE>
__global__ __launch_bounds__(NT) void sweep_kernel(int d, int n1, int64_t n, int nlo, int ldl,
                                                   const int4* __restrict__ offs,
                                                   const int* __restrict__ line_order, int nlines,
                                                   int Hx, int Hy, const T* __restrict__ A,
                                                   const T* __restrict__ scale, const T* __restrict__ in,
                                                   T* __restrict__ out, unsigned* prog, unsigned* ticket,
                                                   const int* __restrict__ stop) {
    __shared__ int s_line;
    __shared__ T s_red[NT / 64];
    __shared__ unsigned s_have[2];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    if (stop && *stop) return;
    for (;;) {
        if (tid == 0) {
            unsigned tk = atomicAdd(ticket, 1u);
            s_line = (tk < (unsigned)nlines) ? line_order[tk] : -1;
            s_have[0] = 0;
            s_have[1] = 0;
        }
        __syncthreads();
        const int line = s_line;
        if (line < 0) break;
        // stream coordinates of the line (reversed grid when REV)
        const int ly = line % n1, lz = line / n1;
        const int dep0 = (ly > 0) ? line - 1 : -1;                        // (iy-1, iz)
        const int dep1 = (d == 3 && lz > 0) ? (lz - 1) * n1 + min(ly + Hy, n1 - 1) : -1;
        for (int ix = 0; ix < n1; ++ix) {
            const unsigned need = (unsigned)min(n1, ix + Hx + 1);
            if (tid == 0) {
                if (dep0 >= 0 && s_have[0] < need) {
                    unsigned v;
                    while ((v = ld_coh(&prog[dep0])) < need) __builtin_amdgcn_s_sleep(1);
                    s_have[0] = v;
                }
                if (dep1 >= 0 && s_have[1] < need) {
                    unsigned v;
                    while ((v = ld_coh(&prog[dep1])) < need) __builtin_amdgcn_s_sleep(1);
                    s_have[1] = v;
                }
            }
            __syncthreads();
            compiler_fence();
            const int64_t rp = (int64_t)line * n1 + ix;         // stream row
            const int64_t rm = REV ? (n - 1 - rp) : rp;          // memory row
            T acc = T(0);
            for (int k = tid; k < nlo; k += NT) {
                const int4 o = offs[k];
                const int cx = ix + o.x, cy = ly + o.y, cz = lz + o.z;
                if (cx >= 0 && cx < n1 && cy >= 0 && cy < n1 && cz >= 0 && cz < n1) {
                    const int64_t nb = REV ? (rm - o.w) : (rm + o.w);
                    acc += A[rp * ldl + k] * ld_coh(&out[nb]);
                }
            }
            acc = wave_sum(acc);
            if (NT > 64) {
                if (lane == 0) s_red[wv] = acc;
                __syncthreads();
                if (tid == 0)
                    for (int w2 = 1; w2 < NT / 64; ++w2) acc += s_red[w2];
            }
            if (tid == 0) {
                T v = in[rm];
                if (SCALE) v *= scale[rm];
                st_coh(&out[rm], v - acc);
                wait_own_stores();
            }
            __syncthreads();
            if (tid == 0 && (ix == n1 - 1 || ((ix + 1) & 7) == 0)) publish(&prog[line], (unsigned)(ix + 1));
        }
        __syncthreads();
    }
}

// 2D substitution, banded. A workgroup owns B consecutive grid lines (one
// wave per line) and walks them as a pipeline; all operands of the row dot
// products come from LDS, which holds full lines: the Hy lines preceding
// the band (written by earlier workgroups) and the band's own B lines.
// Every dependency is carried by the value itself: the LDS line buffers and
// the output in device memory are pre-filled with a sentinel, so a value is
// ready exactly when it is no longer the sentinel. There are no progress
// counters and no waits for store completion; a consumer that reads a
// sentinel simply reads again (rare path).
//   * Own line and earlier lines of the band: written to LDS by their waves.
//   * Earlier bands: wave 0 stages one new column of the Hy preceding lines
//     per row (lanes 0..Hy-1) from device memory into LDS, with the device
//     loads issued D rows ahead.
//   * The static factor rows and the right-hand side are loaded D rows
//     ahead into registers; LDS reads are unconditional (entries outside the
//     grid read a zero slot) so a row waits on LDS once.
//   * Results go to device memory once per group of D rows, except for the
//     band's last line, which the next band reads with no slack (every row).
__device__ inline void wait_lds() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }
// sleep 64*nap cycles, doubling nap up to 64 (about 1.7 us)
__device__ inline void backoff(int& nap) {
    for (int i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(1);
    if (nap < 64) nap <<= 1;
}

// One line of a band: wave w of the workgroup walks grid line L = first + w.
// STAGE: this wave also stages the Hy lines preceding the band (wave 0 of
// every band but the first). LAST: this line is read by the next band, so
// every value goes to device memory at once. Both are fixed for the whole
// walk, so every path through a row issues the same vector memory operations
// (all lanes load and store, idle lanes on valid dummy addresses or the same
// value); the compiler can then keep the prefetches of later rows in flight
// instead of draining them at merges of paths with different counts.
template <typename T, int MK, int D, bool REV, bool SCALE, bool STAGE, bool LAST>
__device__ inline void band_line(int n1, int64_t n, int ldl, int L, int first, int lbase, int Hx, int Hy,
                                 const int (&ody)[MK], const int (&odx)[MK], const int (&kcl)[MK],
                                 const bool (&oval)[MK], const T* __restrict__ A, const T* __restrict__ scale,
                                 const T* __restrict__ in, T* __restrict__ out, T* lb, int w, int zslot) {
    const int lane = threadIdx.x & 63;
    const int64_t rowbase = (int64_t)L * n1;
    const int64_t mbase = REV ? (n - 1 - rowbase) : rowbase;
    const T* Aline = A + rowbase * ldl;
    int loff[MK];
    bool lok[MK];
#pragma unroll
    for (int m = 0; m < MK; ++m) {
        const int ly = L + ody[m];
        lok[m] = oval[m] && ly >= 0 && ly < n1;
        loff[m] = lok[m] ? (ly - lbase) * n1 + odx[m] : 0;
    }
    T a_s[D][MK];
    T r_s[D];
    auto issue = [&](int s, int ixp) {
        ixp = min(ixp, n1 - 1);
        const T* Ar = Aline + (int64_t)ixp * ldl;
        const int64_t rm = REV ? (mbase - ixp) : (mbase + ixp);
#pragma unroll
        for (int m = 0; m < MK; ++m) a_s[s][m] = Ar[kcl[m]];
        // vector loads (a relaxed atomic is never turned into a scalar
        // load; scalar loads share lgkmcnt with LDS)
        T rv = __hip_atomic_load(&in[rm], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (SCALE) rv *= __hip_atomic_load(&scale[rm], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        r_s[s] = rv;
    };
    // staging lanes 0..Hy-1 (lines lbase..first-1 that exist)
    const bool stager = STAGE && (lane < Hy) && (lbase + lane >= 0);
    const int sline = stager ? lbase + lane : 0;
    auto saddr = [&](int x) {
        x = min(x, n1 - 1);
        const int64_t rp = (int64_t)sline * n1 + x;
        return REV ? (n - 1 - rp) : rp;
    };
    T st_v[D];
    // The line just before the band is produced one level ahead of its use,
    // so a value prefetched D rows earlier is always still the sentinel, and
    // re-reading it serially would cost one device round trip per row. Every
    // row therefore also issues one poll in which lanes Hy..63 read the next
    // columns of that line; row x uses the lane of the poll issued KP rows
    // earlier (already returned) that covers its column.
    constexpr int KP = 4;
    T pq[KP];
    const int crit_lane = Hy + KP - 1;
    auto paddr = [&](int x) {
        const int xc = (lane >= Hy) ? x + Hx + 1 + (lane - Hy) : x;
        const int64_t rp = (int64_t)(first - 1) * n1 + min(max(xc, 0), n1 - 1);
        return REV ? (n - 1 - rp) : rp;
    };
    // stage column x (value v loaded earlier; re-read while not ready)
    auto stage_now = [&](int x, T v) {
        const bool act = stager && x < n1;
        if (__builtin_expect(__any(act && Sentinel<T>::is(v)), 0)) {
            while (act && Sentinel<T>::is(v)) {
                __builtin_amdgcn_s_sleep(1);
                v = ld_coh(&out[saddr(x)]);
            }
        }
        if (act) lb[lane * n1 + x] = v;
    };
    if (STAGE) {
        for (int x = 0; x < Hx && x < n1; ++x) stage_now(x, ld_coh(&out[saddr(x)]));
#pragma unroll
        for (int s = 0; s < D; ++s) st_v[s] = ld_coh(&out[saddr(Hx + s)]);
#pragma unroll
        for (int r = 0; r < KP; ++r) pq[r] = ld_coh(&out[paddr(r - KP)]);
    }
    auto row = [&](int s, int ix) -> T {
        if (STAGE) {
            const int x = ix + Hx;
            T v = st_v[s];
            const T vc = lane_val(pq[s % KP], crit_lane);   // column ix + Hx of line first-1
            if (lane == Hy - 1 && !Sentinel<T>::is(vc)) v = vc;
            stage_now(x, v);
            st_v[s] = ld_coh(&out[saddr(x + D)]);
            pq[s % KP] = ld_coh(&out[paddr(ix)]);
        }
        int idx[MK];
#pragma unroll
        for (int m = 0; m < MK; ++m) {
            const bool ok = lok[m] && (unsigned)(ix + odx[m]) < (unsigned)n1;
            idx[m] = ok ? loff[m] + ix : zslot;
        }
        T yv[MK];
#pragma unroll
        for (int m = 0; m < MK; ++m) yv[m] = lb[idx[m]];
        bool miss = false;
#pragma unroll
        for (int m = 0; m < MK; ++m) miss |= Sentinel<T>::is(yv[m]);
        if (__builtin_expect(__any(miss), 0)) {
#pragma unroll
            for (int m = 0; m < MK; ++m) {
                while (Sentinel<T>::is(yv[m])) {
                    __builtin_amdgcn_s_sleep(1);
                    yv[m] = __hip_atomic_load(&lb[idx[m]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        }
        T acc = T(0);
#pragma unroll
        for (int m = 0; m < MK; ++m) acc += (idx[m] == zslot ? T(0) : a_s[s][m]) * yv[m];
        return wave_sum_dpp(acc);
    };
    T* lbw = lb + (Hy + w) * n1;
    auto mrow = [&](int ixp) { return REV ? (mbase - ixp) : (mbase + ixp); };
#pragma unroll
    for (int s = 0; s < D; ++s) issue(s, s);
    int ix0 = 0;
    for (; ix0 + D <= n1; ix0 += D) {
#pragma unroll
        for (int s = 0; s < D; ++s) {
            const int ix = ix0 + s;
            const T acc = row(s, ix);
            const T y = Sentinel<T>::clean(r_s[s] - acc);
            issue(s, ix + D);
            if (lane == 0) lbw[ix] = y;
            if (LAST) st_coh(&out[mrow(ix)], y);   // every lane, the same value
        }
        if (!LAST) {
            // the group's values from LDS; lanes beyond D repeat them
            wait_lds();
            const int j = ix0 + (lane % D);
            st_coh(&out[mrow(j)], lbw[j]);
        }
    }
#pragma unroll
    for (int s = 0; s < D; ++s) {
        const int ix = ix0 + s;
        if (ix < n1) {
            const T acc = row(s, ix);
            const T y = Sentinel<T>::clean(r_s[s] - acc);
            if (lane == 0) lbw[ix] = y;
        }
    }
    wait_lds();
    if (lane < n1 - ix0) st_coh(&out[mrow(ix0 + lane)], lbw[ix0 + lane]);
}

template <typename T, int MK, int D, int B, bool REV, bool SCALE>
__global__ __launch_bounds__(64 * B) void sweep2d_band_kernel(int n1, int64_t n, int nlo, int ldl,
                                                              const int4* __restrict__ offs,
                                                              const T* __restrict__ A, const T* __restrict__ scale,
                                                              const T* __restrict__ in, T* __restrict__ out,
                                                              unsigned* ticket, const int* __restrict__ stop,
                                                              int Hx, int Hy) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    T* lb = (T*)smem_raw;                     // [Hy + B][n1] line buffers, then one zero slot
    __shared__ int s_band;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (stop && *stop) return;
    const int nbands = (n1 + B - 1) / B;
    const int nl = Hy + B;
    const int zslot = nl * n1;

    int odx[MK], ody[MK], kcl[MK];
    bool oval[MK];
#pragma unroll
    for (int m = 0; m < MK; ++m) {
        const int k = lane + 64 * m;
        oval[m] = k < nlo;
        kcl[m] = oval[m] ? k : nlo - 1;
        const int4 o = offs[kcl[m]];
        odx[m] = o.x;
        ody[m] = o.y;
    }

    for (;;) {
        if (tid == 0) {
            const unsigned tk = atomicAdd(ticket, 1u);
            s_band = (tk < (unsigned)nbands) ? (int)tk : -1;
        }
        for (int e = tid; e < zslot; e += 64 * B) lb[e] = Sentinel<T>::value();
        if (tid == 0) lb[zslot] = T(0);
        __syncthreads();
        const int band = __builtin_amdgcn_readfirstlane(s_band);
        if (band < 0) break;
        const int L = band * B + w;
        const int first = band * B;
        const int lbase = first - Hy;   // line held in lb row 0
        if (L < n1) {
            const bool stage = (w == 0) && (first > 0);
            const bool last = (w == B - 1) || (L == n1 - 1);
#define LGP_BAND_LINE(ST, LA)                                                                                \
    band_line<T, MK, D, REV, SCALE, ST, LA>(n1, n, ldl, L, first, lbase, Hx, Hy, ody, odx, kcl, oval, A, scale, \
                                            in, out, lb, w, zslot)
            if (stage) {
                if (last) LGP_BAND_LINE(true, true);
                else LGP_BAND_LINE(true, false);
            } else {
                if (last) LGP_BAND_LINE(false, true);
                else LGP_BAND_LINE(false, false);
            }
#undef LGP_BAND_LINE
        }
        __syncthreads();
    }
}

// 2D substitution, two grid lines per wave. A workgroup owns a band of
// B = 2*NW consecutive lines; wave v walks lines first+2v (lanes 0..31) and
// first+2v+1 (lanes 32..63), the second trailing the first by Hx+1 columns
// so that every value it needs from the first line was produced by the same
// wave one step earlier. Each half-wave holds SL offsets per lane (k = j +
// 32m), so the reduction, the readiness test, the stores and the staging are
// paid once per two rows. Line buffers in LDS carry Hx zero columns on either
// side and lines outside the grid are all zero, so no offset needs a mask;
// entries past n_lower in the factor rows are zero or finite and meet a zero
// LDS slot. A row is ready when its dot product is not NaN (the sentinel is
// a NaN): one test per step, and the slow path re-reads only while a
// sentinel is seen. Every path through a step issues the same loads and
// stores (idle half-waves store the value already in LDS).
__device__ inline double dpp_bcast15(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x142, 0xA, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x142, 0xA, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ inline float dpp_bcast15(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));
}
template <typename T, int SL, int D, int NW, bool REV, bool SCALE, bool STAGE>
__device__ inline void pair_walk(int n1, int64_t n, int ldl, int first, int lbase, int Hx, int Hy, int Wd,
                                 int zslot, const int (&boff)[SL], const int (&bstep)[SL],
                                 const T* __restrict__ A, const T* __restrict__ scale,
                                 const T* __restrict__ in, T* __restrict__ out, T* lb, int wv) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 5, j = lane & 31;
    const int A1 = Hx + 1;
    // line within the band; a half-wave whose line lies beyond the grid
    // repeats the wave's first line (same values to the same addresses)
    const int li = (first + 2 * wv + g < n1) ? 2 * wv + g : 2 * wv;
    const int L = first + li;
    const bool lin = true;
    const int Lc = L;
    const int skew = li * A1;
    const int t0 = 2 * wv * A1;                                  // first step with work
    const int tend = min(n1 - 1 + (2 * wv + 1) * A1, n1 - 1 + (2 * NW - 1) * A1);
    const int own = (L - lbase) * Wd + Hx;                       // LDS index of column 0 of this line
    auto xcl = [&](int t) { return min(max(t - skew, 0), n1 - 1); };
    auto mrow = [&](int x) {
        const int64_t rp = (int64_t)Lc * n1 + x;
        return REV ? (n - 1 - rp) : rp;
    };
    // ring of D steps in flight: the factor row (SL entries per lane), then
    // the right-hand side of the row and, for the backward sweep, its scale
    // (multiplied at use, so the loads are not waited for when issued)
    T a_s[D][SL + 2];
    auto issue = [&](int s, int t) {
        const int x = xcl(t);
        const T* Ar = A + ((int64_t)Lc * n1 + x) * ldl + j;
#pragma unroll
        for (int m = 0; m < SL; ++m) a_s[s][m] = Ar[32 * m];
        // the two half-waves read different rows, so these stay vector loads
        const int64_t rm = mrow(x);
        a_s[s][SL] = in[rm];
        if (SCALE) a_s[s][SL + 1] = scale[rm];
    };
    // staging of the Hy lines before the band (wave 0 of every band but the
    // first): lane l < Hy stages line lbase + l; the line just before the band
    // is polled in flight as well (see below)
    constexpr int KP = 4;
    const bool stager = STAGE && (lane < Hy) && (lbase + lane >= 0);
    const int sline = stager ? lbase + lane : 0;
    const int crit_lane = Hy + KP - 1;
    auto saddr = [&](int c) {
        const int64_t rp = (int64_t)sline * n1 + min(c, n1 - 1);
        return REV ? (n - 1 - rp) : rp;
    };
    auto paddr = [&](int c) {
        const int cc = (lane >= Hy) ? c + 1 + (lane - Hy) : c;
        const int64_t rp = (int64_t)(first - 1) * n1 + min(max(cc, 0), n1 - 1);
        return REV ? (n - 1 - rp) : rp;
    };
    T st_v[D], pq[KP];
    auto stage_now = [&](int c, T v) {
        const bool act = stager && c < n1;
        if (__builtin_expect(__any(act && Sentinel<T>::is(v)), 0)) {
            while (act && Sentinel<T>::is(v)) {
                __builtin_amdgcn_s_sleep(1);
                v = ld_coh(&out[saddr(c)]);
            }
        }
        if (act) lb[lane * Wd + Hx + c] = v;
    };
    if (STAGE) {
        for (int c = 0; c < Hx && c < n1; ++c) stage_now(c, ld_coh(&out[saddr(c)]));
#pragma unroll
        for (int s = 0; s < D; ++s) st_v[s] = ld_coh(&out[saddr(Hx + s)]);
#pragma unroll
        for (int r = 0; r < KP; ++r) pq[r] = ld_coh(&out[paddr(Hx + r - KP)]);
    }
    auto step = [&](int s, int t) {
        if (STAGE) {
            // wave 0's first line is at column t and needs column t + Hx of
            // the staged lines; the poll issued KP steps ago covers it
            const int c = t + Hx;
            T v = st_v[s];
            const T vc = lane_val(pq[s % KP], crit_lane);
            if (lane == Hy - 1 && !Sentinel<T>::is(vc)) v = vc;
            stage_now(c, v);
            st_v[s] = ld_coh(&out[saddr(c + D)]);
            pq[s % KP] = ld_coh(&out[paddr(c)]);
        }
        const int xr = t - skew;
        const bool act = lin && xr >= 0 && xr < n1;
        const int x = min(max(xr, 0), n1 - 1);
        const T prev = lb[own + x];   // what LDS holds for this row (stored by idle half-waves)
        T yv[SL];
#pragma unroll
        for (int m = 0; m < SL; ++m) yv[m] = lb[boff[m] + x * bstep[m]];
        T acc0 = T(0), acc1 = T(0);
#pragma unroll
        for (int m = 0; m < SL; m += 2) acc0 += a_s[s][m] * yv[m];
#pragma unroll
        for (int m = 1; m < SL; m += 2) acc1 += a_s[s][m] * yv[m];
        T acc = act ? acc0 + acc1 : T(0);
        if (__builtin_expect(__any(acc != acc), 0)) {
            // some operand is not written yet (or a genuine NaN): wait for
            // the sentinels to go, then recompute
            for (;;) {
                bool still = false;
#pragma unroll
                for (int m = 0; m < SL; ++m)
                    if (Sentinel<T>::is(yv[m])) {
                        yv[m] = __hip_atomic_load(&lb[boff[m] + x * bstep[m]], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
                        still |= Sentinel<T>::is(yv[m]);
                    }
                if (!__any(act && still)) break;
                __builtin_amdgcn_s_sleep(1);
            }
            acc0 = T(0);
            acc1 = T(0);
#pragma unroll
            for (int m = 0; m < SL; m += 2) acc0 += a_s[s][m] * yv[m];
#pragma unroll
            for (int m = 1; m < SL; m += 2) acc1 += a_s[s][m] * yv[m];
            acc = act ? acc0 + acc1 : T(0);
        }
        // half-wave sums: rows of 16 lanes, then row 0 into row 1 and row 2
        // into row 3; lanes 16..31 and 48..63 hold the two totals
        acc += dpp_v<0xB1>(acc);
        acc += dpp_v<0x4E>(acc);
        acc += dpp_v<0x141>(acc);
        acc += dpp_v<0x140>(acc);
        acc += dpp_bcast15(acc);
        const T tot = g ? lane_val(acc, 63) : lane_val(acc, 31);
        const T rr = SCALE ? a_s[s][SL] * a_s[s][SL + 1] : a_s[s][SL];
        const T y = Sentinel<T>::clean(rr - tot);
        // the new loads of this ring slot must not move above the last use
        // of its old values, or the ring needs one register more and the
        // compiler rotates it with copies that wait for the newest loads
        asm volatile("" ::"v"(y) : "memory");
        issue(s, t + D);
        if (act && (lane == 31 || lane == 63)) lb[own + x] = y;
        // every lane stores (the same value within a half-wave); an idle
        // half-wave stores what LDS already holds for its clamped row, which
        // only it writes, so this never replaces a result
        st_coh(&out[mrow(x)], act ? y : prev);
    };
#pragma unroll
    for (int s = 0; s < D; ++s) issue(s, t0 + s);
    int t = t0;
    for (; t + D - 1 <= tend; t += D) {
#pragma unroll
        for (int s = 0; s < D; ++s) step(s, t + s);
    }
#pragma unroll
    for (int s = 0; s < D; ++s)
        if (t + s <= tend) step(s, t + s);
}

template <typename T, int SL, int D, int NW, bool REV, bool SCALE>
__global__ __launch_bounds__(64 * NW) void sweep2d_pair_kernel(int n1, int64_t n, int nlo, int ldl,
                                                               const int4* __restrict__ offs, const T* __restrict__ A0,
                                                               const T* __restrict__ scale0, const T* __restrict__ in0,
                                                               T* __restrict__ out0, unsigned* ticket,
                                                               const int* __restrict__ stop, int Hx, int Hy,
                                                               const SweepSlot<T>* __restrict__ slots, int nslots) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    T* lb = (T*)smem_raw;   // [Hy + B][n1 + 2 Hx] line buffers, then one zero slot
    __shared__ int s_band;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (stop && *stop) return;
    constexpr int B = 2 * NW;
    const int nbands = (n1 + B - 1) / B;
    const int Wd = n1 + 2 * Hx;
    const int nl = Hy + B;
    const int zslot = nl * Wd;
    const int g = lane >> 5, j = lane & 31;
    // batched: ticket t is band t / nslots of slot t % nslots, so each slot's
    // bands are taken in order
    const int ns = slots ? nslots : 1;
    for (;;) {
        if (tid == 0) {
            const unsigned tk = atomicAdd(ticket, 1u);
            s_band = (tk < (unsigned)(nbands * ns)) ? (int)tk : -1;
        }
        __syncthreads();
        const int bt = __builtin_amdgcn_readfirstlane(s_band);
        if (bt < 0) break;
        const int band = bt / ns;
        const T* A = A0;
        const T* scale = scale0;
        const T* in = in0;
        T* out = out0;
        if (slots) {
            const SweepSlot<T> sl = slots[bt - band * ns];
            if (sl.stop && *sl.stop) {   // this request has converged: its bands are skipped
                __syncthreads();
                continue;
            }
            A = sl.A;
            scale = sl.scale;
            in = sl.in;
            out = sl.out;
        }
        const int first = band * B;
        const int lbase = first - Hy;
        // lines above the grid and the Hx columns either side are zero; the
        // rest waits for its values
        for (int e = tid; e < nl * Wd; e += 64 * NW) {
            const int r = e / Wd, c = e - r * Wd;
            const bool zero = (lbase + r < 0) || c < Hx || c >= Hx + n1;
            lb[e] = zero ? T(0) : Sentinel<T>::value();
        }
        if (tid == 0) lb[zslot] = T(0);
        __syncthreads();
        if (first + 2 * wv < n1) {
            const int L = (first + 2 * wv + g < n1) ? first + 2 * wv + g : first + 2 * wv;
            int boff[SL], bstep[SL];
#pragma unroll
            for (int m = 0; m < SL; ++m) {
                const int k = j + 32 * m;
                const bool ok = k < nlo;
                const int4 o = offs[ok ? k : 0];
                boff[m] = ok ? (L + o.y - lbase) * Wd + Hx + o.x : zslot;
                bstep[m] = ok ? 1 : 0;
            }
            if (wv == 0 && first > 0)
                pair_walk<T, SL, D, NW, REV, SCALE, true>(n1, n, ldl, first, lbase, Hx, Hy, Wd, zslot, boff, bstep,
                                                          A, scale, in, out, lb, wv);
            else
                pair_walk<T, SL, D, NW, REV, SCALE, false>(n1, n, ldl, first, lbase, Hx, Hy, Wd, zslot, boff,
                                                           bstep, A, scale, in, out, lb, wv);
        }
        __syncthreads();
    }
}

__global__ void reset_kernel(unsigned* p, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// ------------------------------------------- factorisation, dataflow -----
// Same recurrence as ilu_factor_kernel (left-looking rows of Alg. 2 with
// U = D L^T), organised for latency:
//   * Every row of L (n_lower entries, then 1/D(i)) is written exactly once
//     into storage pre-filled with the sentinel, so each value is its own
//     readiness flag. Gathers use ordinary cached loads; a sentinel (possibly
//     a stale cached copy) sends the wave to coherent re-reads.
//   * The lower offsets j of a row are visited in a dataflow order fixed on
//     the host: a topological order of the in-row dependencies (u_k feeds
//     u_j when offset(k) - offset(j) is a lower offset) that visits first
//     the offsets whose rows finished longest ago. The loads of the next PD
//     steps are in flight while a step is reduced.
//   * Pair words hold byte offsets: k*8 (into the row's u vector in LDS) in
//     the low half, l*8 (into the gathered row) in the high half, so a
//     gather address is a scalar row pointer plus one shifted lane value.
//   * The pivot sum over u_j^2 / D(i + delta_j) is formed once per row,
//     from the LDS vectors, just before the last steps.
//   * Each wave works on its own rows; the waves of a workgroup share the
//     step and pair tables in LDS.
template <int Q, int PD>
__global__ __launch_bounds__(768) void ilu_factor2_kernel(
    int d, int n1, int64_t n, int nlo, int ldl, int nsteps, int npairs, int T, int h,
    const int4* __restrict__ offs, const int4* __restrict__ steps, const int* __restrict__ sdxyz,
    const unsigned* __restrict__ pairw, const int* __restrict__ row_order, const double* __restrict__ band,
    const double* __restrict__ fold, double* __restrict__ LD, double* __restrict__ Dg,
    double* __restrict__ invD, unsigned* ticket, int* flag) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    int4* st_s = (int4*)smem_raw;                 // [nsteps]
    int4* of_s = st_s + nsteps;                   // [nlo + 1] offsets (dx, dy, dz, linear)
    int* sd_s = (int*)(of_s + nlo + 1);           // [nsteps]
    unsigned* pw_s = (unsigned*)(sd_s + nsteps);  // [npairs + 64 Q]: reads past a list stay inside
    const size_t tab_bytes =
        (((size_t)nsteps * 20 + (size_t)(nlo + 1) * 16 + (size_t)(npairs + 64 * Q) * 4) + 15) & ~(size_t)15;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    // per wave: u[0..nlo] (u[nlo] = M(i,i)), u[nlo+1] = 0, then w[0..nlo+1]
    // (w[k] = 1/D(i + delta_k); w[nlo+1] absorbs the writes of padding steps)
    double* u = (double*)(smem_raw + tab_bytes) + (size_t)wv * (2 * nlo + 4);
    double* w = u + nlo + 2;
    for (int e = tid; e < nsteps; e += blockDim.x) {
        st_s[e] = steps[e];
        sd_s[e] = sdxyz[e];
    }
    for (int e = tid; e <= nlo; e += blockDim.x) of_s[e] = offs[e];
    for (int e = tid; e < npairs + 64 * Q; e += blockDim.x) pw_s[e] = e < npairs ? pairw[e] : 0u;
    __syncthreads();

    const int W = 2 * h + 1;
    const int T1 = T + 1;
    const int bandT = n1 * W;
    const int nzW = (d == 3) ? W : 1;
    const int zoff = (int)(n * ldl);   // a row of zeros after the factor rows
    // the ring is a whole number of PD-step chunks: npad no-op steps lead
    const int nring = ((nsteps + PD - 1) / PD) * PD;
    const int npad = nring - nsteps;
    // Control flow: the only lane-dependent branches sit in the middle of the
    // row loop; the loop head and tail are wave-uniform (scalar tickets and
    // pivots), so the compiler cannot turn a lane-0 block that straddles the
    // back edge into a loop exit that leaves lane 0 behind.
    unsigned tk0 = 0;
    if (lane == 0) tk0 = atomicAdd(ticket, 1u);
    unsigned tk = __builtin_amdgcn_readfirstlane(tk0);
    while (tk < (unsigned)n) {
        const int i = __builtin_amdgcn_readfirstlane(row_order[tk]);
        const int ix = i % n1;
        const int iy = (i / n1) % n1;
        const int iz = (d == 3) ? i / (n1 * n1) : 0;
        const int line = i / n1;
        // M(i, i + delta_k) for the lower offsets and the diagonal (Sec. 4.2):
        // sum_t S^(t)(ix, ix+dx) Fa_t + M^(t)(ix, ix+dx) Fb_t over the folded
        // line coefficients; every address is valid (clamped), entries whose
        // column leaves the grid are masked to zero.
        {
            const double* pS[Q];
            const double* pF[Q];
            double msk[Q], v[Q];
#pragma unroll
            for (int m = 0; m < Q; ++m) {
                const int k = min(lane + 64 * m, nlo);
                const int4 o = of_s[k];
                const bool in = (lane + 64 * m <= nlo) && (unsigned)(ix + o.x) < (unsigned)n1 &&
                                (unsigned)(iy + o.y) < (unsigned)n1 && (unsigned)(iz + o.z) < (unsigned)n1;
                msk[m] = in ? 1.0 : 0.0;
                pS[m] = band + ix * W + (o.x + h);
                pF[m] = fold + ((int64_t)line * nzW * W + (int64_t)(d == 3 ? (o.z + h) * W : 0) + (o.y + h)) * 2 * T1;
                v[m] = 0.0;
            }
            for (int t0 = 0; t0 < T1; t0 += 3) {
                double bs[3][Q], bm[3][Q], fa[3][Q], fb[3][Q];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int t = min(t0 + c, T1 - 1);
#pragma unroll
                    for (int m = 0; m < Q; ++m) {
                        bs[c][m] = pS[m][t * bandT];
                        bm[c][m] = pS[m][(T1 + t) * bandT];
                        fa[c][m] = pF[m][t];
                        fb[c][m] = pF[m][T1 + t];
                    }
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double on = (t0 + c < T1) ? 1.0 : 0.0;
#pragma unroll
                    for (int m = 0; m < Q; ++m) v[m] += on * (bs[c][m] * fa[c][m] + bm[c][m] * fb[c][m]);
                }
            }
#pragma unroll
            for (int m = 0; m < Q; ++m) {
                const int k = lane + 64 * m;
                if (k <= nlo) u[k] = v[m] * msk[m];
                if (k < nlo + 2) w[k] = 0.0;
            }
            if (lane == 0) u[nlo + 1] = 0.0;
        }

        // Steps. Every step issues the same loads (a step whose row i+delta_j
        // leaves the grid, or a padding step past the end, reads the zero row
        // and leaves u_j = 0), so the load counter of each ring slot is static.
        // ring of PD steps in flight: the gathered values, the pair word of
        // each lane (~0u when the lane has no pair), the row offset of the step
        // Pair words hold k (low 16 bits) and the slot l of the gathered
        // entry L(i+delta_j, i+delta_j+delta_l) (high 16 bits). Lanes past
        // a step's pair list take k = nlo+1 (u = 0) and l = the first step's
        // slot: a real entry of the same row, published no later than the
        // ones the step needs. A step whose row leaves the grid (or a
        // padding step) gathers from the zero row.
        double g[PD][Q];
        unsigned pw[PD][Q];
        double dv[PD];
        int jj[PD], rb[PD];
        const int k0 = __builtin_amdgcn_readfirstlane(st_s[0].x);
        const unsigned padw = (unsigned)(nlo + 1) * 8u | ((unsigned)k0 * 8u << 16);
        const char* ub = (const char*)u;
        auto issue = [&](int b, int s) {
            s -= npad;   // the ring runs over npad no-op steps first
            const bool live = s >= 0 && s < nsteps;
            const int sc = live ? s : 0;
            const int4 S = steps[sc];   // wave-uniform: scalar loads
            const int dd = sdxyz[sc];
            const int dx = (dd & 0xFF) - 128, dy = ((dd >> 8) & 0xFF) - 128, dz = ((dd >> 16) & 0xFF) - 128;
            const bool valid = live && (unsigned)(ix + dx) < (unsigned)n1 && (unsigned)(iy + dy) < (unsigned)n1 &&
                               (unsigned)(iz + dz) < (unsigned)n1;
            jj[b] = live ? S.x : nlo + 1;
            const int r0 = valid ? (i + S.y) * ldl : zoff;
            rb[b] = r0;
            const int np = S.w - S.z;
            const unsigned* pwp = pw_s + S.z + lane;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const unsigned wd = pwp[64 * q];
                pw[b][q] = (lane + 64 * q < np) ? wd : padw;
            }
            const char* rowp = (const char*)(LD + r0);
#pragma unroll
            for (int q = 0; q < Q; ++q)
                g[b][q] = __hip_atomic_load((const double*)(rowp + (pw[b][q] >> 16)), __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_WORKGROUP);
            dv[b] = __hip_atomic_load(LD + r0 + nlo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        };
        // A poll re-reads the values of a slot that are still sentinels (in
        // place, in the lanes that hold them), all before the first check:
        // one round trip however many values it waits for.
        auto reload = [&](int c) {
            if (Sentinel<double>::is(dv[c])) dv[c] = ld_coh(LD + rb[c] + nlo);
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (Sentinel<double>::is(g[c][q]))
                    g[c][q] = ld_coh((const double*)((const char*)(LD + rb[c]) + (pw[c][q] >> 16)));
        };
        auto pending = [&](int c) {
            bool bad = Sentinel<double>::is(dv[c]);
#pragma unroll
            for (int q = 0; q < Q; ++q) bad |= Sentinel<double>::is(g[c][q]);
            return bad;
        };
        // The step's sum is formed first; a sentinel among its values makes
        // the sum NaN (sentinels are NaNs and u is finite), so one test of
        // the wave total replaces a test per value. Then the values that
        // are still sentinels are polled and the sum is formed again.
        auto dot = [&](int b) {
            double acc = 0.0;
#pragma unroll
            for (int q = 0; q < Q; ++q) acc += *(const double*)(ub + (pw[b][q] & 0xFFFFu)) * g[b][q];
            return wave_total_bcast(acc);
        };
        auto consume = [&](int b) {   // returns u_j
            const double mj = u[jj[b]];   // M(i, i+delta_j) (0 when invalid); u_j is written only by step j
            double acc = dot(b);
            if (__builtin_expect(__any(isnan(acc) | Sentinel<double>::is(dv[b])), 0)) {
                // a step whose rows are not finished yet: poll its values
                for (;;) {
                    reload(b);
                    if (!__any(pending(b))) break;
                    __builtin_amdgcn_s_sleep(1);
                }
                acc = dot(b);
            }
            const double uj = mj - acc;
            if (lane == 0) {
                u[jj[b]] = uj;
                w[jj[b]] = dv[b];
            }
            return uj;
        };
        // sum of u_j^2 / D(i + delta_j) over the steps done so far (late
        // steps excluded); u and w are zero at the padding index
        auto pivot_sum = [&]() {
            double acc = 0.0;
#pragma unroll
            for (int m = 0; m < Q; ++m) {
                const int k = lane + 64 * m;
                bool own = k < nlo;
#pragma unroll
                for (int b = 0; b < PD; ++b) own &= (k != jj[b]);
                const int kk = own ? k : nlo + 1;
                acc += u[kk] * u[kk] * w[kk];
            }
            return wave_total_bcast(acc);
        };
#pragma unroll
        for (int b = 0; b < PD; ++b) issue(b, b);
        // next row, fetched while this row's first loads are in flight
        unsigned tkn = 0;
        if (lane == 0) tkn = atomicAdd(ticket, 1u);
        for (int s0 = 0; s0 < nring - PD; s0 += PD) {
#pragma unroll
            for (int b = 0; b < PD; ++b) {
                consume(b);
                issue(b, s0 + b + PD);
            }
        }
        // The last PD steps wait for the rows one and two levels back: the
        // hyperplane chain runs through them, so from here on the wave runs
        // at raised priority. The entries of the other steps are final:
        // publish them first, then poll the late steps together (one round
        // trip per poll), finish them and publish their entries, 1/D and D. Every
        // store instruction runs in all lanes (the counters stay static):
        // a lane without an entry of its own repeats the store of another
        // lane (same address, same value) -- never a shared location, which
        // would turn into one hot line for the whole chip.
        __builtin_amdgcn_s_setprio(3);
        double* Li = LD + (int64_t)i * ldl;
        if (nsteps > PD) {   // wave-uniform; false only for tiny stencils
            const int k0 = __builtin_amdgcn_readfirstlane(st_s[0].x);   // first step: never a late one
#pragma unroll
            for (int m = 0; m < Q; ++m) {
                const int k = lane + 64 * m;
                bool own = k < nlo;
#pragma unroll
                for (int b = 0; b < PD; ++b) own &= (k != jj[b]);
                const int kk = own ? k : k0;
                st_coh(Li + kk, Sentinel<double>::clean(u[kk] * w[kk]));
            }
        }
        double piv = pivot_sum();
        for (;;) {
            bool still = false;
#pragma unroll
            for (int c = 0; c < PD; ++c)
                if (__any(pending(c))) {   // wave-uniform
                    reload(c);
                    still = true;
                }
            if (!still) break;
            // one wait for all re-reads, at the next check
            __builtin_amdgcn_s_sleep(1);
        }
#pragma unroll
        for (int b = 0; b < PD; ++b) {
            const double uj = consume(b);   // zero for padding steps
            piv += uj * uj * dv[b];
        }
        // L(i, i+delta_k) = u_k / D(i+delta_k); D(i) = M(i,i) - sum_k u_k L(i, i+delta_k).
        // D(i) is the same in every lane; taking it from lane 0 makes the
        // pivot test and the stores below wave-uniform.
        const double Dr = u[nlo] - piv;
        const double Dii = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(Dr)),
                                            __builtin_amdgcn_readfirstlane(__double2loint(Dr)));
        const double iv = 1.0 / Dii;
        if (nsteps > PD) {
            // lanes 0..PD-1: the late steps' entries; the other lanes (and
            // padding steps) store 1/D
            int kl = nlo;
#pragma unroll
            for (int b = 0; b < PD; ++b) kl = (lane == b && jj[b] < nlo) ? jj[b] : kl;
            st_coh(Li + kl, Sentinel<double>::clean(kl < nlo ? u[kl] * w[kl] : iv));
        } else {
            for (int k = lane; k <= nlo; k += 64)
                st_coh(Li + k, Sentinel<double>::clean(k < nlo ? u[k] * w[k] : iv));
        }
        Dg[i] = Dii;    // the same value from every lane
        invD[i] = iv;
        __builtin_amdgcn_s_setprio(0);
        if (!(Dii > 0.0) || !isfinite(Dii)) atomicOr(flag, 1);   // uniform branch; one atomic per lane, rare
        tk = __builtin_amdgcn_readfirstlane(tkn);
    }
}

// ------------------------------------------------------- d = 1 --------
// In one dimension M is banded (half-width h = T + 2) and NZ(M) is the whole
// band, so ILU(0) is the exact banded factorisation M = L D L^T: rows in
// order, one wavefront, lane m holding lower offset m. The left-looking
// recurrence of the 2D/3D kernels (u_j = M(i,j) - sum_k u_k L(j,k),
// L(i,j) = u_j / D(j), D(i) = M(i,i) - sum_j u_j L(i,j)) is evaluated with
// the previous h rows kept in LDS.
__global__ __launch_bounds__(64) void band1d_factor_kernel(int n1, int nlo, int ldl, int T, int h,
                                                           const int4* __restrict__ offs,
                                                           const double* __restrict__ band,
                                                           const double* __restrict__ ca,
                                                           const double* __restrict__ cb, double* __restrict__ L,
                                                           double* __restrict__ Dg, double* __restrict__ invD,
                                                           int* flag) {
    __shared__ double ring[64][65];   // rows i-1 .. i-64 (by i mod 64): L entries, then 1/D at nlo
    __shared__ double uu[64];
    const int lane = threadIdx.x;
    const int W = 2 * h + 1, T1 = T + 1;
    const int64_t bandT = (int64_t)n1 * W;
    const int dl = lane < nlo ? offs[lane].x : 0;   // this lane's lower offset (negative)
    auto Mentry = [&](int i, int dx) {
        double v = 0.0;
        for (int t = 0; t < T1; ++t) {
            const int64_t e = t * bandT + (int64_t)i * W + (dx + h);
            v += ca[t] * band[e] + cb[t] * band[e + (int64_t)T1 * bandT];
        }
        return v;
    };
    for (int i = 0; i < n1; ++i) {
        // M(i, i + offset_lane) and M(i, i)
        const bool inl = lane < nlo && i + dl >= 0;
        const double mrow = inl ? Mentry(i, dl) : 0.0;
        const double mii = Mentry(i, 0);
        double piv = 0.0;
        for (int jl = 0; jl < nlo; ++jl) {
            const int dj = offs[jl].x;
            const int j = i + dj;
            // u_j = M(i,j) - sum over earlier offsets m of u_m L(j, j + (d_m - d_j))
            double acc = 0.0;
            if (lane < jl && j >= 0) {
                const int dk = dl - dj;          // < 0: offset from row j
                const int sk = dk + nlo;         // its slot (lower offsets are -nlo .. -1)
                if (i + dl >= 0 && sk >= 0) acc = uu[lane] * ring[j & 63][sk];
            }
            acc = wave_sum(acc);
            const double mj = __shfl(mrow, jl, 64);
            const double uj = (j >= 0) ? mj - acc : 0.0;
            if (lane == jl) uu[jl] = uj;
            const double dinv = (j >= 0) ? ring[j & 63][nlo] : 0.0;
            piv += (lane == jl) ? uj * uj * dinv : 0.0;
            __syncthreads();   // uu[jl] visible to the next offsets
        }
        piv = wave_sum(piv);
        const double Dii = mii - piv;
        const double iv = 1.0 / Dii;
        double* Li = L + (int64_t)i * ldl;
        if (lane < nlo) {
            const int j = i + dl;
            const double lij = (j >= 0) ? uu[lane] * ring[j & 63][nlo] : 0.0;
            Li[lane] = lij;
            ring[i & 63][lane] = lij;
        }
        if (lane == 0) {
            Li[nlo] = iv;
            ring[i & 63][nlo] = iv;
            Dg[i] = Dii;
            invD[i] = iv;
            if (!(Dii > 0.0) || !isfinite(Dii)) atomicOr(flag, 1);
        }
        for (int k = nlo + 1 + lane; k < ldl; k += 64) Li[k] = 0.0;
        __syncthreads();
    }
}

// Substitutions on the band, one wavefront, rows in order (forward) or in
// reverse order (backward, U = D L^T: z_i = y_i / D_i - sum_k L(i - d_k, k)
// z(i - d_k)); the last 64 results stay in LDS.
template <typename T, bool REV>
__global__ __launch_bounds__(64) void band1d_sweep_kernel(int n1, int nlo, int ldl, const int4* __restrict__ offs,
                                                          const T* __restrict__ A, const T* __restrict__ invd,
                                                          const T* __restrict__ in, T* __restrict__ out,
                                                          const int* __restrict__ stop) {
    __shared__ T win[64];
    const int lane = threadIdx.x;
    if (stop && *stop) return;   // the solver has converged: nothing to do
    const int dl = lane < nlo ? offs[lane].x : 0;
    win[lane] = T(0);
    __syncthreads();
    // this lane's coefficient and the right-hand side of row i: independent
    // of the recurrence, so row i+1's are loaded while row i is reduced
    auto coef = [&](int i) -> T {
        const int src = REV ? i - dl : i + dl;
        if (lane >= nlo || src < 0 || src >= n1) return T(0);
        return REV ? A[(int64_t)src * ldl + lane] : A[(int64_t)i * ldl + lane];
    };
    auto rhs = [&](int i) -> T { return REV ? in[i] * invd[i] : in[i]; };
    int i = REV ? n1 - 1 : 0;
    T a = coef(i), r = rhs(i);
    for (int s = 0; s < n1; ++s) {
        const int inext = REV ? i - 1 : i + 1;
        T an = T(0), rn = T(0);
        if (s + 1 < n1) {
            an = coef(inext);
            rn = rhs(inext);
        }
        const int src = REV ? i - dl : i + dl;
        const T acc = wave_sum(lane < nlo && src >= 0 && src < n1 ? a * win[src & 63] : T(0));
        const T y = r - acc;
        __syncthreads();
        if (lane == 0) {
            win[i & 63] = y;
            out[i] = y;
        }
        __syncthreads();
        a = an;
        r = rn;
        i = inext;
    }
}

static lgp_status band1d_build(Factor& F, std::vector<int>& off4, hipStream_t s) {
    const int n1 = F.n1, T = F.T, h = F.h;
    const int64_t n = F.n;
    if (F.nlo > 63 || F.ldl > 4096) return LGP_E_UNSUPPORTED;
    {
        const int64_t total = (int64_t)(T + 1) * n1 * (2 * h + 1);
        hipLaunchKernelGGL(band_kernel, dim3((unsigned)std::min<int64_t>(4096, (total + 255) / 256)), dim3(256), 0,
                           s, T, n1, h, F.band);
    }
    off4.assign((size_t)4 * (F.nlo + 1), 0);
    for (int k = 0; k <= F.nlo; ++k) {
        off4[4 * k + 0] = F.offs[3 * k];
        off4[4 * k + 3] = F.offs[3 * k];
    }
    LGP_HIP(hipMemcpyAsync(F.d_offs, off4.data(), off4.size() * 4, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemsetAsync(F.flag, 0, 16, s));
    LGP_HIP(hipMemsetAsync(F.L + (size_t)n * F.ldl, 0, (size_t)F.ldl * 8, s));   // zero row
    hipLaunchKernelGGL(band1d_factor_kernel, dim3(1), dim3(64), 0, s, n1, F.nlo, F.ldl, T, h,
                       (const int4*)F.d_offs, (const double*)F.band, (const double*)F.coefA,
                       (const double*)F.coefB, F.L, F.Dg, F.invD, F.flag);
    if (F.has32) {
        hipLaunchKernelGGL(to_f32_kernel, dim3(4096), dim3(256), 0, s, (int64_t)n * F.ldl, (const double*)F.L, F.L32);
        hipLaunchKernelGGL(to_f32_kernel, dim3(4096), dim3(256), 0, s, (int64_t)n, (const double*)F.invD, F.invD32);
    }
    LGP_CHECK_LAUNCH();
    F.factor_kernel = 1;
    F.levels = n1;
    return LGP_OK;
}

template <typename T>
static lgp_status band1d_sweep(Factor& F, bool backward, const T* A, const T* invd, const T* in, T* out,
                               hipStream_t s, const int* stop) {
    if (backward)
        hipLaunchKernelGGL((band1d_sweep_kernel<T, true>), dim3(1), dim3(64), 0, s, F.n1, F.nlo, F.ldl,
                           (const int4*)F.d_offs, A, invd, in, out, stop);
    else
        hipLaunchKernelGGL((band1d_sweep_kernel<T, false>), dim3(1), dim3(64), 0, s, F.n1, F.nlo, F.ldl,
                           (const int4*)F.d_offs, A, invd, in, out, stop);
    LGP_CHECK_LAUNCH();
    return LGP_OK;
}

// ------------------------------------------------------------- host ------
static int persistent_grid(const void* kernel, int block, size_t shmem, int64_t units) {
    int dev = 0, cus = 256, per = 1;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, shmem) != hipSuccess || per < 1)
        per = 1;
    int64_t g = (int64_t)cus * per;
    if (g > units) g = units;
    if (g < 1) g = 1;
    return (int)g;
}

// Host tables whose contents are copied to the device with hipMemcpyAsync;
// they must stay alive until the stream has executed the copies.
struct FactorHostTables {
    std::vector<int> off4, ptr, pk, pl, st4, sd, lines, lstart, runs;
    std::vector<unsigned> pw;
};

static lgp_status factor_build_impl(Factor& F, hipStream_t s, FactorHostTables& H, hipEvent_t* ev);

void factor_release(Factor& F) { (void)F; }

lgp_status factor_build(Factor& F, hipStream_t s) {
    FactorHostTables H;
    hipEvent_t ev[2] = {nullptr, nullptr};
    const bool timed = hipEventCreate(&ev[0]) == hipSuccess && hipEventCreate(&ev[1]) == hipSuccess;
    F.factor_kernel_ms = -1.0f;
    F.factor_launches = 1;
    F.factor_waits = 0;
    lgp_status st = factor_build_impl(F, s, H, timed ? ev : nullptr);
    // drain the stream before H goes away, on success and on failure alike
    if (hipStreamSynchronize(s) != hipSuccess && st == LGP_OK) st = LGP_E_HIP;
    if (timed && st == LGP_OK) {
        float ms = -1.0f;
        if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) F.factor_kernel_ms = ms;
    }
    for (auto& e : ev)
        if (e) hipEventDestroy(e);
    return st;
}

lgp_status factor3_run(Factor& F, hipStream_t s, const std::vector<int>& st4, const std::vector<unsigned>& pw,
                       hipEvent_t* ev);
lgp_status factor3_generic_finish(Factor& F, hipStream_t s);

// d = 3: folded coefficients, then the chunked kernel (offset-major output
// through the FP64 window) or, for stencils whose rows do not fit LDS, the
// generic kernel on row-major rows followed by the conversion.
static lgp_status factor_build3_impl(Factor& F, hipStream_t s, FactorHostTables& H, hipEvent_t* ev) {
    const int d = 3, n1 = F.n1, T = F.T, h = F.h;
    const int64_t n = F.n;
    // pair words: the packets of the chunked kernel read up to 64 * 8 words past a list
    LGP_HIP(hipMemsetAsync(F.pairw + F.npairs, 0, 64 * 8 * 4, s));
    hipLaunchKernelGGL(fold_kernel, dim3(std::min(F.nlines, 4096)), dim3(256), 0, s, d, n1, T, h,
                       (const double*)F.band, (const double*)F.coefA, (const double*)F.coefB, F.fold3, F.nlines);
    LGP_CHECK_LAUNCH();
    if (F.fB > 0) return factor3_run(F, s, H.st4, H.pw, ev);
    // generic kernel: rows in level order, done flags in y_tmp, rows of L in
    // the window (which holds the whole grid here)
    F.factor_kernel = 1;
    const int64_t A1 = F.Hx + 1, B1 = (int64_t)(F.Hx + 1) * (F.Hy + 1);
    const int64_t maxlev = (n1 - 1) * (1 + A1 + B1) + 1;
    if (maxlev > F.maxlev) return LGP_E_ARG;
    F.levels = (int)maxlev;
    std::vector<int>& lstart = H.lstart;
    lstart.assign(2 * maxlev + 2, 0);
    {
        std::vector<int> diff(maxlev + 1, 0);
        for (int iz = 0; iz < n1; ++iz)
            for (int iy = 0; iy < n1; ++iy) {
                const int64_t b0 = A1 * iy + B1 * iz;
                diff[b0] += 1;
                diff[b0 + n1] -= 1;
            }
        int run = 0, acc = 0;
        for (int64_t l = 0; l < maxlev; ++l) {
            run += diff[l];
            lstart[l] = acc;
            acc += run;
        }
        lstart[maxlev] = acc;
        if (acc != n) return LGP_E_ARG;
    }
    LGP_HIP(hipMemcpyAsync(F.lev, lstart.data(), lstart.size() * 4, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(F.pair_ptr, H.ptr.data(), H.ptr.size() * 4, hipMemcpyHostToDevice, s));
    if (F.npairs > 0) {
        LGP_HIP(hipMemcpyAsync(F.pair_j, H.pk.data(), H.pk.size() * 4, hipMemcpyHostToDevice, s));
        LGP_HIP(hipMemcpyAsync(F.pair_l, H.pl.data(), H.pl.size() * 4, hipMemcpyHostToDevice, s));
    }
    int* d_order = F.line_order;
    hipLaunchKernelGGL(level_order_kernel, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, s,
                       d, n1, n, (int)A1, (int)B1, (const int*)F.lev, F.lev + maxlev + 1, d_order);
    LGP_HIP(hipMemsetAsync(F.ticket, 0, 16, s));
    LGP_HIP(hipMemsetAsync(F.flag, 0, 16, s));
    unsigned* done = (unsigned*)F.y_tmp;
    LGP_HIP(hipMemsetAsync(done, 0, (size_t)n * 4, s));
    const size_t shmem = (size_t)(F.nlo + 1) * 8;
    const int grid = persistent_grid((const void*)ilu_factor_kernel, 64, shmem, n);
    if (ev) hipEventRecord(ev[0], s);
    hipLaunchKernelGGL(ilu_factor_kernel, dim3(grid), dim3(64), shmem, s, d, n1, n, F.nlo, F.ldl, T, h,
                       (const int4*)F.d_offs, (const int*)d_order, (const double*)F.band, (const double*)F.fold3,
                       (const int*)F.pair_ptr, (const int*)F.pair_j, (const int*)F.pair_l, F.ring, F.Dg, F.invD,
                       done, F.ticket, F.flag);
    LGP_CHECK_LAUNCH();
    if (ev) hipEventRecord(ev[1], s);
    return factor3_generic_finish(F, s);
}

static lgp_status factor_build_impl(Factor& F, hipStream_t s, FactorHostTables& H, hipEvent_t* ev) {
    if (F.d == 1) {
        if (ev) hipEventRecord(ev[0], s);
        const lgp_status st1 = band1d_build(F, H.off4, s);
        if (ev) hipEventRecord(ev[1], s);
        return st1;
    }
    const int d = F.d, n1 = F.n1, T = F.T, h = F.h;
    const int W = 2 * h + 1, T1 = T + 1;
    const int64_t n = F.n;
    // 1D band tables S^(t)(i, i+delta), M^(t)(i, i+delta)
    {
        const int64_t total = (int64_t)T1 * n1 * W;
        hipLaunchKernelGGL(band_kernel, dim3((unsigned)std::min<int64_t>(4096, (total + 255) / 256)), dim3(256), 0,
                           s, T, n1, h, F.band);
        LGP_CHECK_LAUNCH();
    }
    // offsets (lower + diagonal) with linear offsets
    std::vector<int>& off4 = H.off4;
    off4.assign((size_t)4 * (F.nlo + 1), 0);
    for (int k = 0; k <= F.nlo; ++k) {
        const int* o = &F.offs[3 * k];
        off4[4 * k + 0] = o[0];
        off4[4 * k + 1] = o[1];
        off4[4 * k + 2] = o[2];
        off4[4 * k + 3] = o[0] + n1 * o[1] + n1 * n1 * o[2];
    }
    LGP_HIP(hipMemcpyAsync(F.d_offs, off4.data(), off4.size() * 4, hipMemcpyHostToDevice, s));
    // left-looking pair lists: for lower j, all lower k < j with
    // offset(k) - offset(j) in the lower list (and its index)
    std::vector<int>&ptr = H.ptr, &pk = H.pk, &pl = H.pl;
    ptr.assign(F.nlo + 2, 0);
    {
        const int R = 4 * h + 1;
        std::vector<int> lut((size_t)R * R * R, -1);
        auto key = [&](int a, int b, int c) { return ((size_t)(c + 2 * h) * R + (b + 2 * h)) * R + (a + 2 * h); };
        for (int k = 0; k < F.nlo; ++k) lut[key(F.offs[3 * k], F.offs[3 * k + 1], F.offs[3 * k + 2])] = k;
        for (int j = 0; j < F.nlo; ++j) {
            ptr[j] = (int)pk.size();
            for (int k = 0; k < j; ++k) {
                const int a = F.offs[3 * k] - F.offs[3 * j];
                const int b = F.offs[3 * k + 1] - F.offs[3 * j + 1];
                const int c = F.offs[3 * k + 2] - F.offs[3 * j + 2];
                if (std::abs(a) > 2 * h || std::abs(b) > 2 * h || std::abs(c) > 2 * h) continue;
                const int l = lut[key(a, b, c)];
                if (l >= 0) {
                    pk.push_back(k);
                    pl.push_back(l);
                }
            }
        }
        ptr[F.nlo] = (int)pk.size();
        ptr[F.nlo + 1] = (int)pk.size();
    }
    if ((int)pk.size() != F.npairs) return LGP_E_ARG;   // planner and builder disagree
    F.maxpairs = 0;
    for (int j = 0; j < F.nlo; ++j) F.maxpairs = std::max(F.maxpairs, ptr[j + 1] - ptr[j]);
    // Dataflow order of the lower offsets for the factorisation: a topological
    // order of "u_k feeds u_j" (k in the pair list of j) that prefers the
    // offsets whose rows lie most hyperplane levels back.
    {
        const int64_t A1 = F.Hx + 1, B1 = (int64_t)(F.Hx + 1) * (F.Hy + 1);
        std::vector<int64_t> lag(F.nlo);
        for (int k = 0; k < F.nlo; ++k)
            lag[k] = -((int64_t)F.offs[3 * k] + A1 * F.offs[3 * k + 1] + B1 * F.offs[3 * k + 2]);
        std::vector<int> indeg(F.nlo, 0), sptr(F.nlo + 1, 0), succ(pk.size());
        for (int j = 0; j < F.nlo; ++j) indeg[j] = ptr[j + 1] - ptr[j];
        for (size_t e = 0; e < pk.size(); ++e) sptr[pk[e] + 1]++;
        for (int k = 0; k < F.nlo; ++k) sptr[k + 1] += sptr[k];
        {
            std::vector<int> fill(sptr.begin(), sptr.end() - 1);
            for (int j = 0; j < F.nlo; ++j)
                for (int e = ptr[j]; e < ptr[j + 1]; ++e) succ[fill[pk[e]]++] = j;
        }
        auto later = [&](int a, int b) { return lag[a] != lag[b] ? lag[a] < lag[b] : a > b; };
        std::vector<int> heap, order;
        for (int j = 0; j < F.nlo; ++j)
            if (indeg[j] == 0) heap.push_back(j);
        std::make_heap(heap.begin(), heap.end(), later);
        while (!heap.empty()) {
            std::pop_heap(heap.begin(), heap.end(), later);
            const int k = heap.back();
            heap.pop_back();
            order.push_back(k);
            for (int e = sptr[k]; e < sptr[k + 1]; ++e)
                if (--indeg[succ[e]] == 0) {
                    heap.push_back(succ[e]);
                    std::push_heap(heap.begin(), heap.end(), later);
                }
        }
        if ((int)order.size() != F.nlo) return LGP_E_ARG;
        std::vector<int>&st4 = H.st4, &sd = H.sd;
        std::vector<unsigned>& pw = H.pw;
        st4.assign((size_t)4 * (F.nlo + 1), 0);
        sd.assign(F.nlo + 1, 0);
        pw.reserve(pk.size());
        for (int s2 = 0; s2 < F.nlo; ++s2) {
            const int j = order[s2];
            st4[4 * s2 + 0] = j;
            st4[4 * s2 + 1] = off4[4 * j + 3];
            st4[4 * s2 + 2] = (int)pw.size();
            for (int e = ptr[j]; e < ptr[j + 1]; ++e) pw.push_back((unsigned)pk[e] * 8u | ((unsigned)pl[e] * 8u << 16));
            st4[4 * s2 + 3] = (int)pw.size();
            sd[s2] = (F.offs[3 * j] + 128) | ((F.offs[3 * j + 1] + 128) << 8) | ((F.offs[3 * j + 2] + 128) << 16);
        }
        LGP_HIP(hipMemcpyAsync(F.steps, st4.data(), st4.size() * 4, hipMemcpyHostToDevice, s));
        LGP_HIP(hipMemcpyAsync(F.sdxyz, sd.data(), sd.size() * 4, hipMemcpyHostToDevice, s));
        if (!pw.empty()) LGP_HIP(hipMemcpyAsync(F.pairw, pw.data(), pw.size() * 4, hipMemcpyHostToDevice, s));
    }
    if (d == 3) return factor_build3_impl(F, s, H, ev);
    LGP_HIP(hipMemcpyAsync(F.pair_ptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice, s));
    if (F.npairs > 0) {
        LGP_HIP(hipMemcpyAsync(F.pair_j, pk.data(), pk.size() * 4, hipMemcpyHostToDevice, s));
        LGP_HIP(hipMemcpyAsync(F.pair_l, pl.data(), pl.size() * 4, hipMemcpyHostToDevice, s));
    }
    // line order for the sweeps: key iy + (Hy+1) iz
    std::vector<int>& lines = H.lines;
    lines.resize(F.nlines);
    for (int l = 0; l < F.nlines; ++l) lines[l] = l;
    std::stable_sort(lines.begin(), lines.end(), [&](int a, int b) {
        const int ka = (a % n1) + (F.Hy + 1) * (a / n1), kb = (b % n1) + (F.Hy + 1) * (b / n1);
        return ka < kb;
    });
    LGP_HIP(hipMemcpyAsync(F.line_order, lines.data(), lines.size() * 4, hipMemcpyHostToDevice, s));
    // row order for the factorisation: level ix + (Hx+1) iy + (Hx+1)(Hy+1) iz.
    // Each grid line covers the consecutive levels base .. base+n1-1, so the
    // level sizes come from the lines alone; the rows are placed on the
    // device. The order and the per-line folded coefficients live in the Ut
    // buffer (not yet needed) to avoid extra storage.
    const int64_t A1 = F.Hx + 1, B1 = (int64_t)(F.Hx + 1) * (F.Hy + 1);
    const int64_t maxlev = (n1 - 1) * (1 + A1 + (d == 3 ? B1 : 0)) + 1;
    if (maxlev > F.maxlev) return LGP_E_ARG;   // planner and builder disagree
    F.levels = (int)maxlev;
    std::vector<int>& lstart = H.lstart;
    lstart.assign(2 * maxlev + 2, 0);
    {
        std::vector<int> diff(maxlev + 1, 0);
        const int nlz = (d == 3) ? n1 : 1;
        for (int iz = 0; iz < nlz; ++iz)
            for (int iy = 0; iy < n1; ++iy) {
                const int64_t b0 = A1 * iy + B1 * iz;
                diff[b0] += 1;
                diff[b0 + n1] -= 1;
            }
        int run = 0, acc = 0;
        for (int64_t l = 0; l < maxlev; ++l) {
            run += diff[l];
            lstart[l] = acc;
            acc += run;
        }
        lstart[maxlev] = acc;
        if (acc != n) return LGP_E_ARG;
    }
    int* d_order = (int*)F.Ut;
    double* fold = (double*)((char*)F.Ut + (((size_t)n * 4 + 255) & ~(size_t)255));
    const int nzW = (d == 3) ? W : 1;
    // (plan_factor sized the Ut buffer for this scratch)
    LGP_HIP(hipMemcpyAsync(F.lev, lstart.data(), lstart.size() * 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(level_order_kernel, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, s,
                       d, n1, n, (int)A1, (int)B1, (const int*)F.lev, F.lev + maxlev + 1, d_order);
    LGP_CHECK_LAUNCH();
    hipLaunchKernelGGL(fold_kernel, dim3(std::min(F.nlines, 4096)), dim3(256), 0, s, d, n1, T, h,
                       (const double*)F.band, (const double*)F.coefA, (const double*)F.coefB, fold, F.nlines);
    LGP_CHECK_LAUNCH();
    LGP_HIP(hipMemsetAsync(F.ticket, 0, 16, s));
    LGP_HIP(hipMemsetAsync(F.flag, 0, 16, s));
    LGP_HIP(hipMemsetAsync(F.L + (size_t)n * F.ldl, 0, (size_t)F.ldl * 8, s));   // zero row
    // dataflow kernel: pair table in LDS, at most 64*Q pairs per step, 32-bit
    // element offsets, pair indices in 16 bits
    constexpr int FQ = 4, FPD = 4;
    const size_t tab_bytes =
        (((size_t)F.nlo * 20 + (size_t)(F.nlo + 1) * 16 + (size_t)(F.npairs + 64 * FQ) * 4) + 15) & ~(size_t)15;
    const size_t wave_bytes = (size_t)(2 * F.nlo + 4) * 8;
    // 12 waves per workgroup: the register budget of 3 waves per SIMD keeps
    // the step ring free of spills, which beats a fourth wave per SIMD
    int wpb = 12;
    while (wpb > 3 && tab_bytes + wpb * wave_bytes > 150 * 1024) wpb /= 2;
    // LGP_FACTOR_KERNEL = 1 or 2 restricts the choice to that kernel where it
    // applies (for tests of both); 0 or unset takes the dataflow kernel (2)
    // where it applies, else the generic one (1)
    const char* kenv = std::getenv("LGP_FACTOR_KERNEL");
    const int kpick = kenv ? std::atoi(kenv) : 0;
    const bool dataflow = F.maxpairs <= 64 * FQ && F.nlo + 1 <= 64 * FQ &&
                          (int64_t)(n + 1) * F.ldl < (int64_t)INT32_MAX &&
                          tab_bytes + wpb * wave_bytes <= 150 * 1024 && (kpick == 0 || kpick == 2);
    if (dataflow) {
        F.factor_kernel = 2;
        hipLaunchKernelGGL(fill_sentinel_kernel<double>, dim3(std::min<int64_t>(8192, (n * F.ldl + 255) / 256)),
                           dim3(256), 0, s, (int64_t)n * F.ldl, F.L, (const int*)nullptr);
        LGP_CHECK_LAUNCH();
        auto kf = ilu_factor2_kernel<FQ, FPD>;
        const size_t shmem = tab_bytes + wpb * wave_bytes;
        hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
        const int grid = persistent_grid((const void*)kf, 64 * wpb, shmem, (n + wpb - 1) / wpb);
        if (ev) hipEventRecord(ev[0], s);
        hipLaunchKernelGGL(kf, dim3(grid), dim3(64 * wpb), shmem, s, d, n1, n, F.nlo, F.ldl, F.nlo, F.npairs, T, h,
                           (const int4*)F.d_offs, (const int4*)F.steps, (const int*)F.sdxyz,
                           (const unsigned*)F.pairw, (const int*)d_order, (const double*)F.band,
                           (const double*)fold, F.L, F.Dg, F.invD, F.ticket, F.flag);
        LGP_CHECK_LAUNCH();
        if (ev) hipEventRecord(ev[1], s);
    } else {
        F.factor_kernel = 1;
        // done flags live in the y_tmp buffer (n doubles >= n unsigned)
        unsigned* done = (unsigned*)F.y_tmp;
        LGP_HIP(hipMemsetAsync(done, 0, (size_t)n * 4, s));
        const size_t shmem = (size_t)(F.nlo + 1) * 8;
        const int grid = persistent_grid((const void*)ilu_factor_kernel, 64, shmem, n);
        if (ev) hipEventRecord(ev[0], s);
        hipLaunchKernelGGL(ilu_factor_kernel, dim3(grid), dim3(64), shmem, s, d, n1, n, F.nlo, F.ldl, T, h,
                           (const int4*)F.d_offs, (const int*)d_order, (const double*)F.band, (const double*)fold,
                           (const int*)F.pair_ptr, (const int*)F.pair_j, (const int*)F.pair_l, F.L, F.Dg,
                           F.invD, done, F.ticket, F.flag);
        LGP_CHECK_LAUNCH();
        if (ev) hipEventRecord(ev[1], s);
    }
    // runs of lower offsets with equal (dy, dz)
    std::vector<int>& runs = H.runs;
    int maxK = 0, maxspan = 0;
    for (int k = 0; k < F.nlo;) {
        int e = k + 1;
        while (e < F.nlo && F.offs[3 * e + 1] == F.offs[3 * k + 1] && F.offs[3 * e + 2] == F.offs[3 * k + 2]) ++e;
        runs.insert(runs.end(), {k, e, F.offs[3 * k], F.offs[3 * (e - 1)]});
        maxK = std::max(maxK, e - k);
        maxspan = std::max(maxspan, F.offs[3 * (e - 1)] - F.offs[3 * k]);
        k = e;
    }
    F.nruns = (int)runs.size() / 4;
    int R = 256;
    while (R > 16 && (size_t)(R + maxspan) * maxK * 8 > 64 * 1024) R /= 2;
    const bool tiled = F.nruns > 0 && (size_t)(R + maxspan) * maxK * 8 <= 64 * 1024;
    if (tiled) LGP_HIP(hipMemcpyAsync(F.runs, runs.data(), runs.size() * 4, hipMemcpyHostToDevice, s));
    // after 1/D at n_lower, rows of L end in zeros; the forward sweep needs L only
    if (F.ldl > F.nlo + 1)
        hipLaunchKernelGGL(zero_pad_kernel, dim3(4096), dim3(256), 0, s, n, F.ldl, F.nlo + 1, F.L);
    if (F.has32) {
        hipLaunchKernelGGL(to_f32_kernel, dim3(4096), dim3(256), 0, s, (int64_t)n * F.ldl, (const double*)F.L, F.L32);
        hipLaunchKernelGGL(to_f32_kernel, dim3(4096), dim3(256), 0, s, (int64_t)n, (const double*)F.invD, F.invD32);
    }
    LGP_CHECK_LAUNCH();
    // The backward operator Ut, on the caller's stream after the factor
    // (reads of L, entries < n_lower, do not meet the padding writes above).
    if (tiled) {
        const size_t shmem = (size_t)(R + maxspan) * maxK * 8;
        hipFuncSetAttribute((const void*)build_ut_tiled_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)shmem);
        hipLaunchKernelGGL(build_ut_tiled_kernel, dim3((unsigned)((n + R - 1) / R), F.nruns), dim3(256), shmem, s,
                           d, n1, n, F.ldl, (const int4*)F.d_offs, (const int4*)F.runs, R, (const double*)F.L, F.Ut);
    } else {
        hipLaunchKernelGGL(build_ut_kernel, dim3(4096), dim3(256), 0, s, d, n1, n, F.nlo, F.ldl,
                           (const int4*)F.d_offs, (const double*)F.L, F.Ut);
    }
    hipLaunchKernelGGL(zero_pad_kernel, dim3(4096), dim3(256), 0, s, n, F.ldl, F.nlo, F.Ut);
    if (F.has32)
        hipLaunchKernelGGL(to_f32_kernel, dim3(4096), dim3(256), 0, s, (int64_t)n * F.ldl, (const double*)F.Ut,
                           F.Ut32);
    LGP_CHECK_LAUNCH();
    return LGP_OK;
}

template <typename T>
static lgp_status sweep_t(Factor& F, bool backward, const T* A, const T* scale, const T* in, T* out,
                          hipStream_t s, const int* stop) {
    unsigned* prog = F.prog + (backward ? F.nlines : 0);
    unsigned* tick = F.ticket + (backward ? 1 : 0);
    hipLaunchKernelGGL(reset_kernel, dim3(std::min(1024, (F.nlines + 255) / 256 + 1)), dim3(256), 0, s, prog,
                       F.nlines);
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, tick, 1);
    LGP_CHECK_LAUNCH();
    const int64_t n = F.n;
    constexpr int BB = 8, DD = 8;
    // two lines per wave, NW = 4 waves: bands of 8 lines
    constexpr int PNW = 4;
    const size_t pair_shmem = ((size_t)(2 * PNW + F.Hy) * (F.n1 + 2 * F.Hx) + 1) * sizeof(T);
    const int SLn = (F.nlo + 31) / 32;
    const size_t band_shmem = ((size_t)(BB + F.Hy) * F.n1 + 1) * sizeof(T);
    if (F.d == 2 && SLn >= 1 && SLn <= 8 && 32 * SLn <= F.ldl && F.Hy + 4 <= 64 && pair_shmem <= 150 * 1024) {
        const int nbands = (F.n1 + 2 * PNW - 1) / (2 * PNW);
        hipLaunchKernelGGL(fill_sentinel_kernel<T>, dim3(std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, s,
                           n, out, stop);
        auto pick = [&](auto kf) {
            hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pair_shmem);
            const int grid = persistent_grid((const void*)kf, 64 * PNW, pair_shmem, nbands);
            hipLaunchKernelGGL(kf, dim3(grid), dim3(64 * PNW), pair_shmem, s, F.n1, n, F.nlo, F.ldl,
                               (const int4*)F.d_offs, A, scale, in, out, tick, stop, F.Hx, F.Hy,
                               (const SweepSlot<T>*)nullptr, 0);
        };
#define LGP_PAIR(SLv)                                                                    \
    case SLv:                                                                            \
        if (backward) pick(sweep2d_pair_kernel<T, SLv, DD, PNW, true, true>);            \
        else pick(sweep2d_pair_kernel<T, SLv, DD, PNW, false, false>);                   \
        break;
        switch (SLn) {
            LGP_PAIR(1) LGP_PAIR(2) LGP_PAIR(3) LGP_PAIR(4) LGP_PAIR(5) LGP_PAIR(6) LGP_PAIR(7) LGP_PAIR(8)
        }
#undef LGP_PAIR
    } else if (F.d == 2 && F.nlo <= 8 * 64 && band_shmem <= 150 * 1024) {
        const int nbands = (F.n1 + BB - 1) / BB;
        hipLaunchKernelGGL(fill_sentinel_kernel<T>, dim3(std::min<int64_t>(4096, (n + 255) / 256)), dim3(256), 0, s,
                           n, out, stop);
        auto pick = [&](auto kf) {
            hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)band_shmem);
            const int grid = persistent_grid((const void*)kf, 64 * BB, band_shmem, nbands);
            hipLaunchKernelGGL(kf, dim3(grid), dim3(64 * BB), band_shmem, s, F.n1, n, F.nlo, F.ldl,
                               (const int4*)F.d_offs,
                               A, scale, in, out, tick, stop, F.Hx, F.Hy);
        };
        if (F.nlo <= 128) {
            if (backward) pick(sweep2d_band_kernel<T, 2, DD, BB, true, true>);
            else pick(sweep2d_band_kernel<T, 2, DD, BB, false, false>);
        } else if (F.nlo <= 256) {
            if (backward) pick(sweep2d_band_kernel<T, 4, DD, BB, true, true>);
            else pick(sweep2d_band_kernel<T, 4, DD, BB, false, false>);
        } else {
            if (backward) pick(sweep2d_band_kernel<T, 8, DD, BB, true, true>);
            else pick(sweep2d_band_kernel<T, 8, DD, BB, false, false>);
        }
    } else if (F.d == 2) {
        auto kf = backward ? sweep_kernel<T, 64, true, true> : sweep_kernel<T, 64, false, false>;
        const int grid = persistent_grid((const void*)kf, 64, 0, F.nlines);
        hipLaunchKernelGGL(kf, dim3(grid), dim3(64), 0, s, F.d, F.n1, n, F.nlo, F.ldl, (const int4*)F.d_offs,
                           (const int*)F.line_order, F.nlines, F.Hx, F.Hy, A, scale, in, out, prog, tick,
                           stop);
    } else {
        auto kf = backward ? sweep_kernel<T, 256, true, true> : sweep_kernel<T, 256, false, false>;
        const int grid = persistent_grid((const void*)kf, 256, 0, F.nlines);
        hipLaunchKernelGGL(kf, dim3(grid), dim3(256), 0, s, F.d, F.n1, n, F.nlo, F.ldl, (const int4*)F.d_offs,
                           (const int*)F.line_order, F.nlines, F.Hx, F.Hy, A, scale, in, out, prog, tick,
                           stop);
    }
    LGP_CHECK_LAUNCH();
    return LGP_OK;
}

template <typename T>
__global__ void fill_sentinel_slots_kernel(int64_t n, const SweepSlot<T>* __restrict__ slots) {
    const SweepSlot<T> sl = slots[blockIdx.y];
    if (sl.stop && *sl.stop) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        sl.out[i] = Sentinel<T>::value();
}

lgp_status sweep_batch(const Factor& F, int nslots, const SweepSlot<double>* slots, bool backward, unsigned* ticket,
                       hipStream_t s) {
    if (F.layout == 1) return sweep3_batch(F, nslots, slots, backward, ticket, s);
    using T = double;
    const int64_t n = F.n;
    constexpr int DD = 8, PNW = 4;
    const size_t pair_shmem = ((size_t)(2 * PNW + F.Hy) * (F.n1 + 2 * F.Hx) + 1) * sizeof(T);
    const int SLn = (F.nlo + 31) / 32;
    if (!(F.d == 2 && SLn >= 1 && SLn <= 8 && 32 * SLn <= F.ldl && F.Hy + 4 <= 64 && pair_shmem <= 150 * 1024))
        return LGP_E_UNSUPPORTED;
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, ticket, 1);
    hipLaunchKernelGGL(fill_sentinel_slots_kernel<T>, dim3((unsigned)std::min<int64_t>(2048, (n + 255) / 256), nslots),
                       dim3(256), 0, s, n, slots);
    const int nbands = (F.n1 + 2 * PNW - 1) / (2 * PNW);
    auto pick = [&](auto kf) {
        set_dyn_shmem((const void*)kf, pair_shmem, s);
        const int grid = persistent_grid((const void*)kf, 64 * PNW, pair_shmem, (int64_t)nbands * nslots);
        hipLaunchKernelGGL(kf, dim3(grid), dim3(64 * PNW), pair_shmem, s, F.n1, n, F.nlo, F.ldl,
                           (const int4*)F.d_offs, (const T*)nullptr, (const T*)nullptr, (const T*)nullptr, (T*)nullptr,
                           ticket, (const int*)nullptr, F.Hx, F.Hy, slots, nslots);
    };
#define LGP_PAIRB(SLv)                                                                   \
    case SLv:                                                                            \
        if (backward) pick(sweep2d_pair_kernel<T, SLv, DD, PNW, true, true>);            \
        else pick(sweep2d_pair_kernel<T, SLv, DD, PNW, false, false>);                   \
        break;
    switch (SLn) {
        LGP_PAIRB(1) LGP_PAIRB(2) LGP_PAIRB(3) LGP_PAIRB(4) LGP_PAIRB(5) LGP_PAIRB(6) LGP_PAIRB(7) LGP_PAIRB(8)
    }
#undef LGP_PAIRB
    LGP_CHECK_LAUNCH();
    return LGP_OK;
}

lgp_status sweep(Factor& F, bool backward, const double* in, double* out, hipStream_t s, const int* stop) {
    if (F.layout == 1) return sweep3(F, backward, false, in, out, s, stop);
    if (F.d == 1) return band1d_sweep<double>(F, backward, F.L, F.invD, in, out, s, stop);
    return backward ? sweep_t<double>(F, true, F.Ut, F.invD, in, out, s, stop)
                    : sweep_t<double>(F, false, F.L, nullptr, in, out, s, stop);
}

lgp_status sweep32(Factor& F, bool backward, const float* in, float* out, hipStream_t s, const int* stop) {
    if (!F.has32) return LGP_E_ARG;
    if (F.layout == 1) return sweep3(F, backward, true, in, out, s, stop);
    if (F.d == 1) return band1d_sweep<float>(F, backward, F.L32, F.invD32, in, out, s, stop);
    return backward ? sweep_t<float>(F, true, F.Ut32, F.invD32, in, out, s, stop)
                    : sweep_t<float>(F, false, F.L32, nullptr, in, out, s, stop);
}

}  // namespace lgp

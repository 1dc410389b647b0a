// Fast discrete Legendre transforms (Sec. 2.2, the BDLT and FDLT sums) in
// the manner of Hale and Townsend (2016): an asymptotic expansion of L_n
// evaluated with FFTs where it is accurate, direct three-term recurrence
// elsewhere, O(N (log N)^2) per transform; and the product of Sec. 4.3
// through them (steps 1-4: phi to Legendre coefficients, BDLT, pointwise
// coefficients, FDLT, recombination onto the test functions).
//
// Expansion. For 0 < theta < pi and M terms,
//   L_n(cos theta) = C_n sum_{m<M} h_{m,n} cos((n+m+1/2) theta - (m+1/2) pi/2)
//                    / (2 sin theta)^{m+1/2} + R,
//   C_n = sqrt(4/pi) Gamma(n+1) / Gamma(n+3/2),
//   h_{m,n} = prod_{j=1..m} (j-1/2)^2 / (j (n+j+1/2)),
//   |R| <= 2 C_n h_{M,n} / (2 sin theta)^{M+1/2}.
// Degrees are split into blocks [n_j, 2 n_j) (n_0 = 64 .. N); block j uses the
// expansion at the nodes with sin theta >= alpha_j, where the bound at n_j
// is below 1e-16; all other (node, degree) pairs are summed directly. So the
// direct part of node k is the prefix n < nd(k), and its direct work over
// all nodes is O(N log N).
//
// Sums over a block at non-equispaced theta_k: with n = nc + v (|v| <= hw),
// theta_k = t_{q_k} + delta_k on the grid t_q = 2 pi q / L (L a power of two
// >= 2(N+1), |delta_k| <= pi / L),
//   sum_v u_v e^{i v theta_k} = sum_p (i delta_k hw)^p / p! * G_p(q_k),
//   G_p(q) = sum_v (v / hw)^p u_v e^{2 pi i v q / L},
// one FFT of length L per Taylor term p (|v delta| <= pi/4, so about 15
// terms reach 1e-17). The forward transform is the transpose of each piece
// (node values spread to the grid, the same FFT, read at the frequencies).
//
// Layout: transforms act on `count` contiguous vectors of q = N+1 values;
// tensor transforms gather the lines of each axis into contiguous rows.
#include <algorithm>
#include <cmath>
#include <vector>

#include "devutil.h"
#include "lgp_internal.h"

namespace lgp {

constexpr int kDltM = 20;         // expansion terms
constexpr int kDltT = 256;        // threads per workgroup
constexpr int kDltMaxL = 4096;    // largest FFT (LDS: L complex doubles)
constexpr int kDltMaxNode = 8;    // nodes per thread (q <= 8 * 256)
constexpr int kDltMaxFreq = 4;    // block frequencies per thread

struct DltBlock {
    int n0, n1, K, nc;   // degrees [n0, n1), Taylor terms, centre
    double alpha;        // expansion used where sin(theta) >= alpha
    double hw;           // half width (scale of v)
};

// device tables of a plan (kernel argument)
struct DltDev {
    double* xk;      // [q] nodes
    double* wk;      // [q] weights
    double* th;      // [q] theta_k
    double* sn;      // [q] sin(theta_k)
    double* dl;      // [q] delta_k
    int* qk;         // [q] grid index of theta_k
    int* nd;         // [q] direct degrees n < nd(k)
    double* ch;      // [M][q] C_n h_{m,n}
    double2* tw;     // [L/2] e^{2 pi i t / L}
    int4* blk;       // [nb] {n0, n1, K, nc}
    double2* bdev;   // [nb] {alpha, hw}
};

struct Dlt {
    Problem* P;
    int d, N, q, L, lgL, nb;
    int64_t lines_max;                 // q^(d-1): lines of a tensor transform
    int64_t lines_cap;                 // most lines of one call (at least 16)
    std::vector<DltBlock> blocks;
    DltDev v;
    // scratch
    double* part;    // [(nb + 1) * lines_max * q]
    double* f0; double* f1;            // [q^d] a field: coefficients, node values
    double* s0; double* s1; double* s2; double* s3;   // [q^d] tensor-transform scratch
    size_t bytes;
};

// ------------------------------------------------------------ plan -------
static double log_c(int n) { return 0.5 * std::log(4.0 / M_PI) + std::lgamma(n + 1.0) - std::lgamma(n + 1.5); }
static double log_h(int m, int n) {
    double v = 0.0;
    for (int j = 1; j <= m; ++j) v += 2.0 * std::log(j - 0.5) - std::log((double)j) - std::log(n + j + 0.5);
    return v;
}

static void plan_blocks(Dlt& D) {
    const int N = D.N;
    D.blocks.clear();
    for (int n0 = 64; n0 <= N;) {
        const int n1 = std::min(2 * n0, N + 1);
        DltBlock b;
        b.n0 = n0;
        b.n1 = n1;
        b.nc = (n0 + n1) / 2;
        b.hw = std::max(1.0, 0.5 * (n1 - n0));
        b.alpha = 0.5 * std::exp((std::log(2.0) + log_c(n0) + log_h(kDltM, n0) - std::log(1e-16)) / (kDltM + 0.5));
        // Taylor terms: (hw pi / L)^K / K! < 1e-17
        const double z = b.hw * M_PI / D.L;
        int K = 1;
        double t = z;
        while (t > 1e-17 && K < 40) {
            ++K;
            t *= z / K;
        }
        b.K = K;
        if (b.alpha < 1.0) D.blocks.push_back(b);
        n0 = n1;
    }
    D.nb = (int)D.blocks.size();
}

static size_t plan_dlt(Dlt& D, Problem& P, void* buf) {
    Carver c(buf);
    D.P = &P;
    D.d = P.d;
    D.N = P.N;
    D.q = P.q;
    D.L = 1;
    D.lgL = 0;
    while (D.L < 2 * D.q) {
        D.L *= 2;
        ++D.lgL;
    }
    plan_blocks(D);
    D.lines_max = 1;
    for (int k = 1; k < D.d; ++k) D.lines_max *= D.q;
    D.lines_cap = std::max<int64_t>(D.lines_max, 16);
    const int64_t nq = D.lines_cap * D.q;
    D.v.xk = c.take<double>(D.q);
    D.v.wk = c.take<double>(D.q);
    D.v.th = c.take<double>(D.q);
    D.v.sn = c.take<double>(D.q);
    D.v.dl = c.take<double>(D.q);
    D.v.qk = c.take<int>(D.q);
    D.v.nd = c.take<int>(D.q);
    D.v.ch = c.take<double>((size_t)kDltM * D.q);
    D.v.tw = c.take<double2>(D.L / 2);
    D.v.blk = c.take<int4>(std::max(1, D.nb));
    D.v.bdev = c.take<double2>(std::max(1, D.nb));
    D.part = c.take<double>((size_t)(D.nb + 1) * nq);
    D.f0 = c.take<double>(nq);
    D.f1 = c.take<double>(nq);
    D.s0 = c.take<double>(nq);
    D.s1 = c.take<double>(nq);
    D.s2 = c.take<double>(nq);
    D.s3 = c.take<double>(nq);
    D.bytes = c.off + 256;
    return D.bytes;
}

bool dlt_supported(const Problem& P) {
    int L = 1;
    while (L < 2 * P.q) L *= 2;
    return L <= kDltMaxL && P.q <= kDltT * kDltMaxNode;
}

size_t dlt_bytes(Problem& P) {
    Dlt D;
    return plan_dlt(D, P, nullptr);
}

static lgp_status upload_dlt(Dlt& D, hipStream_t s) {
    const int q = D.q, L = D.L;
    std::vector<double> th(q), sn(q), dl(q), ch((size_t)kDltM * q, 0.0);
    std::vector<int> qk(q), nd(q);
    for (int k = 0; k < q; ++k) {
        th[k] = std::acos(D.P->x[k]);
        sn[k] = std::sin(th[k]);
        int g = (int)std::lround(th[k] * L / (2.0 * M_PI));
        dl[k] = th[k] - 2.0 * M_PI * g / L;
        qk[k] = ((g % L) + L) % L;
        // the blocks' cut-offs decrease with n, so the expansion covers
        // every degree from the first block the node qualifies for
        nd[k] = q;
        for (int j = 0; j < D.nb; ++j)
            if (sn[k] >= D.blocks[j].alpha) {
                nd[k] = D.blocks[j].n0;
                break;
            }
    }
    for (int n = 0; n < q; ++n) {
        const double lc = log_c(n);
        for (int m = 0; m < kDltM; ++m) ch[(size_t)m * q + n] = std::exp(lc + log_h(m, n));
    }
    std::vector<double2> tw(L / 2);
    for (int t = 0; t < L / 2; ++t) tw[t] = make_double2(std::cos(2.0 * M_PI * t / L), std::sin(2.0 * M_PI * t / L));
    std::vector<int4> blk(std::max(1, D.nb));
    std::vector<double2> bd(std::max(1, D.nb));
    for (int j = 0; j < D.nb; ++j) {
        blk[j] = make_int4(D.blocks[j].n0, D.blocks[j].n1, D.blocks[j].K, D.blocks[j].nc);
        bd[j] = make_double2(D.blocks[j].alpha, D.blocks[j].hw);
    }
    LGP_HIP(hipMemcpyAsync(D.v.xk, D.P->x.data(), q * 8, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(D.v.wk, D.P->w.data(), q * 8, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(D.v.th, th.data(), q * 8, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(D.v.sn, sn.data(), q * 8, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(D.v.dl, dl.data(), q * 8, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(D.v.qk, qk.data(), q * 4, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(D.v.nd, nd.data(), q * 4, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(D.v.ch, ch.data(), ch.size() * 8, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(D.v.tw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(D.v.blk, blk.data(), blk.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(D.v.bdev, bd.data(), bd.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    LGP_HIP(hipStreamSynchronize(s));   // the host tables go out of scope
    return LGP_OK;
}

// ------------------------------------------------------------ FFT --------
// In place, input in bit-reversed order, output natural:
// X[t] = sum_v x[v] e^{+2 pi i v t / L}. 256 threads, L <= kDltMaxL.
// Radix-2 butterflies, stage s pairing elements h = 2^s apart with the
// twiddle of their position p in the pair's block, tw[p L / 2h]. R
// consecutive stages are taken in one pass over LDS: the 2^R elements
// base + m h (m < 2^R) that those stages combine only with each other sit
// in registers while the same butterflies run on them in the same order,
// so a pass replaces R rounds of LDS traffic and barriers.
template <int R>
__device__ inline void fft_pass(double2* X, int L, int s, const double2* __restrict__ tw) {
    constexpr int E = 1 << R;
    const int h = 1 << s;
    for (int g = threadIdx.x; g < (L >> R); g += kDltT) {
        const int pos0 = g & (h - 1);
        const int base = ((g >> s) << (s + R)) + pos0;
        double2 v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = X[base + m * h];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            const int step = L >> (s + t + 1);   // twiddle stride of stage s + t
#pragma unroll
            for (int m = 0; m < E; ++m) {
                if (m & (1 << t)) continue;
                const int p = pos0 + (m & ((1 << t) - 1)) * h;   // position in the pair's block
                const double2 w = tw[p * step];
                const double2 u = v[m], x = v[m + (1 << t)];
                const double2 tt = make_double2(w.x * x.x - w.y * x.y, w.x * x.y + w.y * x.x);
                v[m] = make_double2(u.x + tt.x, u.y + tt.y);
                v[m + (1 << t)] = make_double2(u.x - tt.x, u.y - tt.y);
            }
        }
#pragma unroll
        for (int m = 0; m < E; ++m) X[base + m * h] = v[m];
    }
    __syncthreads();
}

__device__ inline void fft_lds(double2* X, int L, int lgL, const double2* __restrict__ tw) {
    int s = 0;
    for (; s + 3 <= lgL; s += 3) fft_pass<3>(X, L, s, tw);
    if (lgL - s == 2) fft_pass<2>(X, L, s, tw);
    if (lgL - s == 1) fft_pass<1>(X, L, s, tw);
}

__device__ inline int bitrev(int v, int lg) { return (int)(__brev((unsigned)v) >> (32 - lg)); }

// ------------------------------------------------------ kernels ----------
// Backward, direct part: out[l][k] = sum_{n < nd(k)} c[l][n] L_n(x_k).
__global__ __launch_bounds__(kDltT) void dlt_bwd_direct_kernel(int q, const double* __restrict__ c,
                                                              double* __restrict__ out,
                                                              const double* __restrict__ xk,
                                                              const int* __restrict__ nd) {
    extern __shared__ double cs[];
    const int64_t l = blockIdx.x;
    for (int n = threadIdx.x; n < q; n += kDltT) cs[n] = c[l * q + n];
    __syncthreads();
    for (int k = threadIdx.x; k < q; k += kDltT) {
        const double x = xk[k];
        const int m = nd[k];
        double p0 = 1.0, p1 = x, acc = 0.0;
        if (m > 0) acc = cs[0];
        if (m > 1) acc += cs[1] * x;
        for (int n = 1; n + 1 < m; ++n) {
            const double p2 = ((2 * n + 1) * x * p1 - n * p0) / (n + 1);
            acc += cs[n + 1] * p2;
            p0 = p1;
            p1 = p2;
        }
        out[l * q + k] = acc;
    }
}

// Backward, block j by the expansion: part[j][l][k] for the nodes the block
// covers (zero elsewhere).
__global__ __launch_bounds__(kDltT) void dlt_bwd_asym_kernel(int q, int L, int lgL, int64_t lines,
                                                            const double* __restrict__ c,
                                                            double* __restrict__ part, const DltDev D) {
    extern __shared__ double2 X[];
    const int j = blockIdx.y;
    const int64_t l = blockIdx.x;
    const int4 B = D.blk[j];
    const double hw = D.bdev[j].y;
    const int n0 = B.x, n1 = B.y, K = B.z, nc = B.w;
    // this thread's frequencies v = n - nc and nodes
    double base[kDltMaxFreq], sc[kDltMaxFreq];
    int pos[kDltMaxFreq];
    const int nf = n1 - n0;
    for (int f = 0; f < kDltMaxFreq; ++f) {
        const int i = threadIdx.x + f * kDltT;
        pos[f] = -1;
        if (i < nf) {
            const int v = n0 + i - nc;
            pos[f] = bitrev(((v % L) + L) % L, lgL);
            sc[f] = v / hw;
        }
    }
    double g[kDltMaxNode];
    double2 acc[kDltMaxNode];
    for (int r = 0; r < kDltMaxNode; ++r) g[r] = 0.0;
    for (int m = 0; m < kDltM; ++m) {
        for (int f = 0; f < kDltMaxFreq; ++f) {
            const int i = threadIdx.x + f * kDltT;
            base[f] = (i < nf) ? c[l * q + n0 + i] * D.ch[(size_t)m * q + n0 + i] : 0.0;
        }
        for (int r = 0; r < kDltMaxNode; ++r) acc[r] = make_double2(0.0, 0.0);
        for (int p = 0; p < K; ++p) {
            for (int t = threadIdx.x; t < L; t += kDltT) X[t] = make_double2(0.0, 0.0);
            __syncthreads();
            for (int f = 0; f < kDltMaxFreq; ++f)
                if (pos[f] >= 0) X[pos[f]] = make_double2(base[f], 0.0);
            __syncthreads();
            fft_lds(X, L, lgL, D.tw);
            // acc_k += (i delta_k hw)^p / p! * X[q_k]
            for (int r = 0; r < kDltMaxNode; ++r) {
                const int k = threadIdx.x + r * kDltT;
                if (k < q && D.nd[k] <= n0) {
                    const double z = D.dl[k] * hw;
                    // (i z)^p / p!
                    double mag = 1.0;
                    for (int t = 1; t <= p; ++t) mag *= z / t;
                    const int ph = p & 3;   // i^p
                    const double2 co = ph == 0 ? make_double2(mag, 0.0)
                                       : ph == 1 ? make_double2(0.0, mag)
                                       : ph == 2 ? make_double2(-mag, 0.0)
                                                 : make_double2(0.0, -mag);
                    const double2 F = X[D.qk[k]];
                    acc[r].x += co.x * F.x - co.y * F.y;
                    acc[r].y += co.x * F.y + co.y * F.x;
                }
            }
            __syncthreads();
            for (int f = 0; f < kDltMaxFreq; ++f) base[f] *= sc[f];
        }
        // g_k += (2 sin theta_k)^{-(m+1/2)} Re[e^{i((m+1/2)(theta_k - pi/2) + nc theta_k)} acc_k]
        for (int r = 0; r < kDltMaxNode; ++r) {
            const int k = threadIdx.x + r * kDltT;
            if (k < q && D.nd[k] <= n0) {
                const double thk = D.th[k];
                const double ph = (m + 0.5) * (thk - 0.5 * M_PI) + nc * thk;
                const double amp = std::pow(2.0 * D.sn[k], -(m + 0.5));
                g[r] += amp * (std::cos(ph) * acc[r].x - std::sin(ph) * acc[r].y);
            }
        }
    }
    double* out = part + ((int64_t)j * lines + l) * q;
    for (int r = 0; r < kDltMaxNode; ++r) {
        const int k = threadIdx.x + r * kDltT;
        if (k < q) out[k] = (D.nd[k] <= n0) ? g[r] : 0.0;
    }
}

// out = direct + sum of the block parts (fixed order)
__global__ void dlt_sum_kernel(int64_t total, int nb, const double* __restrict__ direct,
                               const double* __restrict__ part, double* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        double v = direct[e];
        for (int j = 0; j < nb; ++j) v += part[(int64_t)j * total + e];
        out[e] = v;
    }
}

// Forward, direct part: out[l][n] = (2n+1)/2 sum_{k: n < nd(k)} w_k f[l][k] L_n(x_k).
// Degrees in chunks of 16: each thread keeps its nodes' recurrences and
// adds their terms, then the workgroup reduces the 16 sums.
constexpr int kFwdChunk = 16;
__global__ __launch_bounds__(kDltT) void dlt_fwd_direct_kernel(int q, const double* __restrict__ f,
                                                              double* __restrict__ out,
                                                              const double* __restrict__ xk,
                                                              const double* __restrict__ wk,
                                                              const int* __restrict__ nd) {
    __shared__ double red[kDltT / 64][kFwdChunk];
    const int64_t l = blockIdx.x;
    double x[kDltMaxNode], v[kDltMaxNode], p0[kDltMaxNode], p1[kDltMaxNode];
    int lim[kDltMaxNode];
    for (int r = 0; r < kDltMaxNode; ++r) {
        const int k = threadIdx.x + r * kDltT;
        lim[r] = 0;
        x[r] = 0.0;
        v[r] = 0.0;
        if (k < q) {
            x[r] = xk[k];
            v[r] = wk[k] * f[l * q + k];
            lim[r] = nd[k];
        }
        p0[r] = 0.0;   // L_{-1}
        p1[r] = 1.0;   // L_0
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int nb0 = 0; nb0 < q; nb0 += kFwdChunk) {
        double s[kFwdChunk];
        for (int t = 0; t < kFwdChunk; ++t) {
            const int n = nb0 + t;
            double acc = 0.0;
            for (int r = 0; r < kDltMaxNode; ++r) {
                if (n < lim[r]) acc += v[r] * p1[r];
                // advance: p1 <- L_{n+1}
                const double p2 = n == 0 ? x[r] : ((2 * n + 1) * x[r] * p1[r] - n * p0[r]) / (n + 1);
                p0[r] = p1[r];
                p1[r] = p2;
            }
            s[t] = acc;
        }
        for (int t = 0; t < kFwdChunk; ++t) {
            double a = s[t];
            for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
            if (lane == 0) red[wv][t] = a;
        }
        __syncthreads();
        if (threadIdx.x < kFwdChunk) {
            const int n = nb0 + threadIdx.x;
            double a = 0.0;
            for (int w = 0; w < kDltT / 64; ++w) a += red[w][threadIdx.x];
            if (n < q) out[l * q + n] = 0.5 * (2 * n + 1) * a;
        }
        __syncthreads();
    }
}

// Forward, block j by the expansion (transpose of the backward block):
// part[j][l][n] = (2n+1)/2 C_n sum_m h_{m,n} Re[e^{-i(m+1/2)pi/2} T_m(n - nc)],
// T_m(v) = sum_k z_{m,k} e^{i v theta_k},
// z_{m,k} = w_k f_k (2 sin theta_k)^{-(m+1/2)} e^{i(nc+m+1/2) theta_k}.
__global__ __launch_bounds__(kDltT) void dlt_fwd_asym_kernel(int q, int L, int lgL, int64_t lines,
                                                            const double* __restrict__ f,
                                                            double* __restrict__ part, const DltDev D) {
    extern __shared__ double2 X[];
    const int j = blockIdx.y;
    const int64_t l = blockIdx.x;
    const int4 B = D.blk[j];
    const double hw = D.bdev[j].y;
    const int n0 = B.x, n1 = B.y, K = B.z, nc = B.w;
    const int nf = n1 - n0;
    int fidx[kDltMaxFreq];
    double sc[kDltMaxFreq], cn[kDltMaxFreq];
    for (int fr = 0; fr < kDltMaxFreq; ++fr) {
        const int i = threadIdx.x + fr * kDltT;
        fidx[fr] = -1;
        cn[fr] = 0.0;
        if (i < nf) {
            const int v = n0 + i - nc;
            fidx[fr] = ((v % L) + L) % L;
            sc[fr] = v / hw;
        }
    }
    double vk[kDltMaxNode];
    int bpos[kDltMaxNode];
    for (int r = 0; r < kDltMaxNode; ++r) {
        const int k = threadIdx.x + r * kDltT;
        vk[r] = 0.0;
        bpos[r] = -1;
        if (k < q && D.nd[k] <= n0) {
            vk[r] = D.wk[k] * f[l * q + k];
            bpos[r] = bitrev(D.qk[k], lgL);
        }
    }
    for (int m = 0; m < kDltM; ++m) {
        double2 T[kDltMaxFreq];
        double pw[kDltMaxFreq];
        for (int fr = 0; fr < kDltMaxFreq; ++fr) {
            T[fr] = make_double2(0.0, 0.0);
            pw[fr] = 1.0;
        }
        // y_k = z_{m,k} (i delta_k hw)^p / p!, from p = 0, advanced by one
        // complex product per Taylor term
        double yr[kDltMaxNode], yi[kDltMaxNode], zd[kDltMaxNode];
        for (int r = 0; r < kDltMaxNode; ++r) {
            yr[r] = yi[r] = zd[r] = 0.0;
            if (bpos[r] < 0) continue;
            const int k = threadIdx.x + r * kDltT;
            const double thk = D.th[k];
            const double amp = vk[r] * std::pow(2.0 * D.sn[k], -(m + 0.5));
            const double ph = (nc + m + 0.5) * thk;
            yr[r] = amp * std::cos(ph);
            yi[r] = amp * std::sin(ph);
            zd[r] = D.dl[k] * hw;
        }
        for (int p = 0; p < K; ++p) {
            for (int t = threadIdx.x; t < L; t += kDltT) X[t] = make_double2(0.0, 0.0);
            __syncthreads();
            // spread y_k to the grid, then y_k *= i z_k / (p + 1)
            for (int r = 0; r < kDltMaxNode; ++r) {
                if (bpos[r] < 0) continue;
                atomicAdd(&X[bpos[r]].x, yr[r]);
                atomicAdd(&X[bpos[r]].y, yi[r]);
                const double c = zd[r] / (p + 1);
                const double nr = -yi[r] * c, ni = yr[r] * c;
                yr[r] = nr;
                yi[r] = ni;
            }
            __syncthreads();
            fft_lds(X, L, lgL, D.tw);
            for (int fr = 0; fr < kDltMaxFreq; ++fr) {
                if (fidx[fr] < 0) continue;
                const double2 G = X[fidx[fr]];
                T[fr].x += pw[fr] * G.x;
                T[fr].y += pw[fr] * G.y;
                pw[fr] *= sc[fr];
            }
            __syncthreads();
        }
        // Re[e^{-i(m+1/2)pi/2} T] = cos((m+1/2)pi/2) Re T + sin((m+1/2)pi/2) Im T
        const double a = (m + 0.5) * 0.5 * M_PI;
        const double ca = std::cos(a), sa = std::sin(a);
        for (int fr = 0; fr < kDltMaxFreq; ++fr) {
            if (fidx[fr] < 0) continue;
            const int n = n0 + threadIdx.x + fr * kDltT;
            cn[fr] += D.ch[(size_t)m * q + n] * (ca * T[fr].x + sa * T[fr].y);
        }
    }
    double* out = part + ((int64_t)j * lines + l) * q;
    for (int n = threadIdx.x; n < q; n += kDltT) out[n] = 0.0;
    __syncthreads();
    for (int fr = 0; fr < kDltMaxFreq; ++fr) {
        if (fidx[fr] < 0) continue;
        const int n = n0 + threadIdx.x + fr * kDltT;
        out[n] = 0.5 * (2 * n + 1) * cn[fr];
    }
}

// ------------------------------------------------------- lines / axes ----
// contiguous rows of the lines along axis `ax` (stride q^ax) of a q^d array, and back
__global__ void gather_lines_kernel(int64_t nq, int q, int64_t s, const double* __restrict__ in,
                                    double* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nq; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = e / q, i = e - l * q;
        const int64_t lo = l % s, hi = l / s;
        out[e] = in[hi * s * q + lo + i * s];
    }
}
__global__ void scatter_lines_kernel(int64_t nq, int q, int64_t s, const double* __restrict__ in,
                                     double* __restrict__ out) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nq; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = e / q, i = e - l * q;
        const int64_t lo = l % s, hi = l / s;
        out[hi * s * q + lo + i * s] = in[e];
    }
}

static int egrid(int64_t n) { return (int)std::min<int64_t>(8192, (n + 255) / 256); }

// 1D transforms of `count` contiguous vectors (forward: FDLT, else BDLT)
static lgp_status dlt_lines(Dlt& D, bool forward, int64_t count, const double* in, double* out, hipStream_t s) {
    const int q = D.q;
    const size_t shm = (size_t)D.L * sizeof(double2);
    double* direct = D.part + (size_t)D.nb * count * q;
    if (!forward) {
        hipLaunchKernelGGL(dlt_bwd_direct_kernel, dim3((unsigned)count), dim3(kDltT), q * 8, s, q, in, direct,
                           (const double*)D.v.xk, (const int*)D.v.nd);
        if (D.nb > 0) {
            (void)hipFuncSetAttribute((const void*)dlt_bwd_asym_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)shm);
            hipLaunchKernelGGL(dlt_bwd_asym_kernel, dim3((unsigned)count, D.nb), dim3(kDltT), shm, s, q, D.L, D.lgL,
                               count, in, D.part, D.v);
        }
    } else {
        hipLaunchKernelGGL(dlt_fwd_direct_kernel, dim3((unsigned)count), dim3(kDltT), 0, s, q, in, direct,
                           (const double*)D.v.xk, (const double*)D.v.wk, (const int*)D.v.nd);
        if (D.nb > 0) {
            (void)hipFuncSetAttribute((const void*)dlt_fwd_asym_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)shm);
            hipLaunchKernelGGL(dlt_fwd_asym_kernel, dim3((unsigned)count, D.nb), dim3(kDltT), shm, s, q, D.L, D.lgL,
                               count, in, D.part, D.v);
        }
    }
    const int64_t total = count * q;
    hipLaunchKernelGGL(dlt_sum_kernel, dim3(egrid(total)), dim3(256), 0, s, total, D.nb, (const double*)direct,
                       (const double*)D.part, out);
    LGP_CHECK_LAUNCH();
    return LGP_OK;
}

// tensor transform of a q^d array along every axis; in and out are not
// the scratch buffers s0..s3 (they may be the same array)
static lgp_status dlt_tensor(Dlt& D, bool forward, const double* in, double* out, hipStream_t s) {
    const int q = D.q;
    const int64_t nq = D.lines_max * q;
    const double* cur = in;
    for (int ax = 0; ax < D.d; ++ax) {
        int64_t st = 1;
        for (int k = 0; k < ax; ++k) st *= q;
        double* dst = (ax == D.d - 1) ? out : (cur == D.s0 ? D.s1 : D.s0);
        if (ax == 0) {
            lgp_status e = dlt_lines(D, forward, D.lines_max, cur, dst, s);
            if (e != LGP_OK) return e;
        } else {
            hipLaunchKernelGGL(gather_lines_kernel, dim3(egrid(nq)), dim3(256), 0, s, nq, q, st, cur, D.s2);
            lgp_status e = dlt_lines(D, forward, D.lines_max, D.s2, D.s3, s);
            if (e != LGP_OK) return e;
            hipLaunchKernelGGL(scatter_lines_kernel, dim3(egrid(nq)), dim3(256), 0, s, nq, q, st, (const double*)D.s3,
                               dst);
        }
        cur = dst;
    }
    LGP_CHECK_LAUNCH();
    return LGP_OK;
}

// --------------------------------------------------- product (Sec. 4.3) ---
// Step 1 for one field: Legendre coefficients c (q^d) of u (n1^d) with, per
// axis, phi_k = L_k - L_{k+2} or, on the derivative axis, phi_k' = -(2k+3) L_{k+1}.
__global__ void phi_to_legendre_kernel(int d, int n1, int q, int deriv, const double* __restrict__ u,
                                       double* __restrict__ c) {
    int64_t nq = q;
    for (int k = 1; k < d; ++k) nq *= q;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nq; e += (int64_t)gridDim.x * blockDim.x) {
        int idx[3] = {0, 0, 0};
        int64_t r = e;
        for (int a = 0; a < d; ++a) {
            idx[a] = (int)(r % q);
            r /= q;
        }
        // sum over the (at most 2 per axis) source indices
        double acc = 0.0;
        const int combos = 1 << d;
        for (int cmb = 0; cmb < combos; ++cmb) {
            double coef = 1.0;
            int64_t src = 0, mul = 1;
            bool ok = true;
            for (int a = 0; a < d && ok; ++a) {
                const int n = idx[a];
                int kk;
                double cf;
                if (a == deriv) {
                    if ((cmb >> a) & 1) { ok = false; break; }
                    kk = n - 1;   // L_{k+1} from phi_k'
                    cf = -(2.0 * kk + 3.0);
                } else if (((cmb >> a) & 1) == 0) {
                    kk = n;       // + L_k
                    cf = 1.0;
                } else {
                    kk = n - 2;   // - L_{k+2}
                    cf = -1.0;
                }
                if (kk < 0 || kk >= n1) { ok = false; break; }
                coef *= cf;
                src += kk * mul;
                mul *= n1;
            }
            if (ok) acc += coef * u[src];
        }
        c[e] = acc;
    }
}

// pointwise: v = a (or b) * v
__global__ void mul_field_kernel(int64_t n, const double* __restrict__ a, double* __restrict__ v) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        v[e] *= a[e];
}

// Step 4 for one field: y[m] (+)= sum over axes of the test-function maps:
// on the derivative axis phi_m' = -(2m+3) L_{m+1}: 2/(2m+3) * -(2m+3) c_{m+1} = -2 c_{m+1};
// elsewhere phi_m = L_m - L_{m+2}: 2/(2m+1) c_m - 2/(2m+5) c_{m+2}.
__global__ void recombine_kernel(int d, int n1, int q, int deriv, const double* __restrict__ c,
                                 double* __restrict__ y, int accumulate) {
    int64_t n = n1;
    for (int k = 1; k < d; ++k) n *= n1;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        int idx[3] = {0, 0, 0};
        int64_t r = e;
        for (int a = 0; a < d; ++a) {
            idx[a] = (int)(r % n1);
            r /= n1;
        }
        double acc = 0.0;
        const int combos = 1 << d;
        for (int cmb = 0; cmb < combos; ++cmb) {
            double coef = 1.0;
            int64_t src = 0, mul = 1;
            bool ok = true;
            for (int a = 0; a < d; ++a) {
                const int m = idx[a];
                int kk;
                double cf;
                if (a == deriv) {
                    if ((cmb >> a) & 1) { ok = false; break; }
                    kk = m + 1;
                    cf = -2.0;
                } else if (((cmb >> a) & 1) == 0) {
                    kk = m;
                    cf = 2.0 / (2 * m + 1);
                } else {
                    kk = m + 2;
                    cf = -2.0 / (2 * m + 5);
                }
                coef *= cf;
                src += kk * mul;
                mul *= q;
            }
            if (ok) acc += coef * c[src];
        }
        y[e] = accumulate ? y[e] + acc : acc;
    }
}

lgp_status matvec_fast(Dlt& D, const double* u, double* y, hipStream_t s) {
    Problem& P = *D.P;
    const int d = P.d, n1 = P.n1, q = P.q;
    const int64_t nq = P.nq, n = P.n;
    // b-term, then the a-term of each direction (a_j in slot j when anisotropic)
    for (int field = -1; field < d; ++field) {
        hipLaunchKernelGGL(phi_to_legendre_kernel, dim3(egrid(nq)), dim3(256), 0, s, d, n1, q, field, u, D.f0);
        lgp_status e = dlt_tensor(D, false, D.f0, D.f1, s);                     // step 2: BDLT
        if (e != LGP_OK) return e;
        const double* coef = field < 0 ? P.b_nodes : P.a_nodes + (P.aniso ? (int64_t)field * nq : 0);
        hipLaunchKernelGGL(mul_field_kernel, dim3(egrid(nq)), dim3(256), 0, s, nq, coef, D.f1);
        e = dlt_tensor(D, true, D.f1, D.f0, s);                                 // step 3: FDLT
        if (e != LGP_OK) return e;
        hipLaunchKernelGGL(recombine_kernel, dim3(egrid(n)), dim3(256), 0, s, d, n1, q, field, (const double*)D.f0, y,
                           field >= 0 ? 1 : 0);                                  // step 4
        LGP_CHECK_LAUNCH();
    }
    return LGP_OK;
}

// ------------------------------------------------------------ handle ------
Dlt* dlt_create(Problem& P, void* buf, size_t bytes, hipStream_t s, lgp_status* st) {
    Dlt* D = new (std::nothrow) Dlt();
    if (!D) {
        *st = LGP_E_NOMEM;
        return nullptr;
    }
    if (plan_dlt(*D, P, buf) > bytes) {
        delete D;
        *st = LGP_E_NOMEM;
        return nullptr;
    }
    *st = upload_dlt(*D, s);
    if (*st != LGP_OK) {
        delete D;
        return nullptr;
    }
    return D;
}

void dlt_destroy(Dlt* D) { delete D; }

lgp_status dlt_apply(Dlt& D, bool forward, int64_t count, const double* in, double* out, hipStream_t s) {
    if (count < 1 || count > D.lines_cap) return LGP_E_ARG;
    return dlt_lines(D, forward, count, in, out, s);
}

int dlt_blocks(const Dlt& D) { return D.nb; }

}  // namespace lgp

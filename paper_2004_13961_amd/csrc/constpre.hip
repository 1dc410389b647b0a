// The constant-coefficient preconditioner of the comparison method PCG-I
// (Sec. 5.2): a and b replaced by their series truncated at t1 = t2 = 0, i.e.
// the constants c_a = a_hat_0 and c_b = b_hat_0 (Sec. 4.1 with T = 0), so
//   K0 = c_a (S (x) M + M (x) S) + c_b M (x) M        (2D; three terms in 3D)
// with the 1D stiffness S = diag(4k + 6) and the pentadiagonal 1D mass M
// (offsets 0 and +-2), both exact for the compact basis (Sec. 2.1, 3). The
// paper solves K0 directly by Shen's fast methods; here it is solved exactly
// by matrix diagonalisation: with E^T S E = I and E^T M E = diag(lam) (the
// generalized eigenvectors of (M, S), from two symmetric tridiagonal
// problems since M couples only indices of equal parity),
//   K0^{-1} r = (E (x) E) diag(1 / (c_a (lam_j + lam_i) + c_b lam_j lam_i)) (E (x) E)^T r,
// i.e. 2d dense contractions with E on the MFMA units and one pointwise
// scaling fused into a contraction epilogue.
#include <cfloat>
#include <cmath>
#include <map>
#include <mutex>
#include <vector>

#include "lgp_internal.h"

namespace lgp {

// Symmetric tridiagonal eigenproblem by the implicit QL iteration with
// Wilkinson-type shifts (the tql2 procedure of Bowdler, Martin, Reinsch and
// Wilkinson, Numer. Math. 11, 1968). d: diagonal (m), e: sub-diagonal
// (m - 1). On return d holds the eigenvalues and z (row-major m x m) the
// orthonormal eigenvectors as columns. False if an eigenvalue needs more
// than 60 sweeps.
static bool tridiagonal_ql(int m, std::vector<double>& d, std::vector<double> e, std::vector<double>& z) {
    z.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) z[(size_t)i * m + i] = 1.0;
    e.resize(m, 0.0);
    e[m - 1] = 0.0;
    for (int l = 0; l < m; ++l) {
        for (int sweeps = 0;; ++sweeps) {
            // the first negligible off-diagonal entry at or after l splits the matrix
            int mm = l;
            while (mm < m - 1 && std::fabs(e[mm]) > DBL_EPSILON * (std::fabs(d[mm]) + std::fabs(d[mm + 1]))) ++mm;
            if (mm == l) break;
            if (sweeps == 60) return false;
            // shift from the leading 2x2 block, then chase the bulge from mm up to l
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[mm] - d[l] + e[l] / (g + std::copysign(r, g));
            double s = 1.0, c = 1.0, p = 0.0;
            bool early = false;
            for (int i = mm - 1; i >= l; --i) {
                const double f = s * e[i];
                const double b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {   // exact split: deflate and restart
                    d[i + 1] -= p;
                    e[mm] = 0.0;
                    early = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                for (int k = 0; k < m; ++k) {   // accumulate the rotation into the eigenvectors
                    double* zk = &z[(size_t)k * m];
                    const double t = zk[i + 1];
                    zk[i + 1] = s * zk[i] + c * t;
                    zk[i] = c * zk[i] - s * t;
                }
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[mm] = 0.0;
        }
    }
    return true;
}

// E (n1 x n1, row k = basis index, column j = eigenpair) and lam for degree N.
struct ConstBasis {
    std::vector<double> E, lam;
    bool ok = false;
};

static std::mutex g_cb_mu;
static std::map<int, ConstBasis> g_cb;

static const ConstBasis& const_basis(int N) {
    {
        std::lock_guard<std::mutex> lk(g_cb_mu);
        auto it = g_cb.find(N);
        if (it != g_cb.end()) return it->second;
    }
    const int n1 = N - 1;
    ConstBasis cb;
    cb.E.assign((size_t)n1 * n1, 0.0);
    cb.lam.assign(n1, 0.0);
    cb.ok = true;
    auto sk = [](int k) { return 4.0 * k + 6.0; };
    auto mdiag = [](int k) { return 2.0 / (2 * k + 1) + 2.0 / (2 * k + 5); };
    auto moff = [](int k) { return -2.0 / (2 * k + 5); };   // M(k, k+2)
    int col = 0;
    for (int par = 0; par < 2; ++par) {
        // indices k = par, par + 2, ...: S^{-1/2} M S^{-1/2} restricted to them is tridiagonal
        const int m = (n1 - par + 1) / 2;
        if (m <= 0) continue;
        std::vector<double> d(m), e(m > 1 ? m - 1 : 1, 0.0), z;
        for (int i = 0; i < m; ++i) {
            const int k = par + 2 * i;
            d[i] = mdiag(k) / sk(k);
            if (i + 1 < m) e[i] = moff(k) / std::sqrt(sk(k) * sk(k + 2));
        }
        if (!tridiagonal_ql(m, d, e, z)) cb.ok = false;
        for (int c = 0; c < m; ++c, ++col) {
            cb.lam[col] = d[c];
            for (int i = 0; i < m; ++i) {
                const int k = par + 2 * i;
                cb.E[(size_t)k * n1 + col] = z[(size_t)i * m + c] / std::sqrt(sk(k));
            }
        }
    }
    std::lock_guard<std::mutex> lk(g_cb_mu);
    return g_cb.emplace(N, std::move(cb)).first->second;
}

size_t const_factor_bytes(const Problem& P) {
    Carver c(nullptr);
    const int64_t n = P.n;
    c.take<double>((size_t)P.n1 * P.n1);
    c.take<double>(P.n1);
    c.take<double>(n);
    c.take<double>(n);
    c.take<double>(n);
    c.take<double>(4 * 256 + 4);
    return c.off + 256;
}

// per-block partial sums of the 1+d weighted fields W*b, W*a_{d-1}, .., W*a_0
// (the FDLT coefficient of index 0 is the weighted mean: c_0 = 2^-d sum W f)
__global__ void cc_partial_kernel(int64_t nq, int nf, const double* __restrict__ wab, double* __restrict__ part) {
    __shared__ double sv[256];
    for (int f = 0; f < nf; ++f) {
        double v = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nq; i += (int64_t)gridDim.x * 256)
            v += wab[(int64_t)f * nq + i];
        sv[threadIdx.x] = v;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sv[threadIdx.x] += sv[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[f * 256 + blockIdx.x] = sv[0];
        __syncthreads();
    }
}

// part[1024 + f] = field f's mean: f = 0 is c_b, f = 1 + (d-1-j) is c_a of direction j
__global__ void cc_final_kernel(int d, double* __restrict__ part) {
    if (threadIdx.x != 0) return;
    const double scale = (d == 1) ? 0.5 : (d == 2) ? 0.25 : 0.125;   // 1 / |Omega|
    for (int f = 0; f <= d; ++f) {
        double v = 0.0;
        for (int i = 0; i < 256; ++i) v += part[f * 256 + i];
        part[1024 + f] = v * scale;
    }
}

// 1 / (sum_j c_j prod_{k != j} lam_k + c_b prod_k lam_k): in the eigenbasis the
// stiffness of direction j becomes 1 and every mass factor its eigenvalue;
// V[l][j][i] (3D) or V[j][i] (2D), i along x
__global__ void cc_inverse_kernel(int d, int n1, int64_t n, const double* __restrict__ lam,
                                  const double* __restrict__ cc, double* __restrict__ inv) {
    const double cb = cc[1024];
    const double cx = cc[1024 + d], cy = d >= 2 ? cc[1024 + d - 1] : 0.0, cz = d == 3 ? cc[1025] : 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e % n1);
        const int j = (int)((e / n1) % n1);
        double den;
        if (d == 2) {
            den = cx * lam[j] + cy * lam[i] + cb * lam[j] * lam[i];
        } else {
            const int l = (int)(e / ((int64_t)n1 * n1));
            den = cx * lam[l] * lam[j] + cy * lam[l] * lam[i] + cz * lam[j] * lam[i] + cb * lam[l] * lam[j] * lam[i];
        }
        inv[e] = 1.0 / den;
    }
}

lgp_status const_factor_build(Factor& F, Problem& P, void* buf, size_t bytes, hipStream_t s) {
    if (bytes < const_factor_bytes(P)) return LGP_E_NOMEM;
    const ConstBasis& cb = const_basis(P.N);
    if (!cb.ok) return LGP_E_UNSUPPORTED;
    F.kind = 1;
    F.P = &P;
    F.d = P.d;
    F.n1 = P.n1;
    F.n = P.n;
    Carver c(buf);
    const int n1 = P.n1;
    F.ccE = c.take<double>((size_t)n1 * n1);
    F.ccLam = c.take<double>(n1);
    F.ccInv = c.take<double>(P.n);
    F.ccT1 = c.take<double>(P.n);
    F.ccT2 = c.take<double>(P.n);
    F.ccPart = c.take<double>(4 * 256 + 4);
    F.bytes = c.off + 256;
    LGP_HIP(hipMemcpyAsync(F.ccE, cb.E.data(), cb.E.size() * 8, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(F.ccLam, cb.lam.data(), cb.lam.size() * 8, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(cc_partial_kernel, dim3(256), dim3(256), 0, s, P.nq, 1 + P.d, (const double*)P.wab, F.ccPart);
    hipLaunchKernelGGL(cc_final_kernel, dim3(1), dim3(64), 0, s, P.d, F.ccPart);
    hipLaunchKernelGGL(cc_inverse_kernel, dim3((unsigned)std::min<int64_t>(4096, (P.n + 255) / 256)), dim3(256), 0,
                       s, P.d, n1, P.n, (const double*)F.ccLam, (const double*)F.ccPart, F.ccInv);
    LGP_CHECK_LAUNCH();
    // the host copies of E and lam are cached; synchronise so the caller may
    // rely on the handle as for the ILU(0) factor
    LGP_HIP(hipStreamSynchronize(s));
    return LGP_OK;
}

lgp_status const_apply(Factor& F, const double* r, double* z, hipStream_t s) {
    if (F.kind != 1) return LGP_E_ARG;
    const int n1 = F.n1;
    const int64_t nn = (int64_t)n1 * n1;
    const double* E = F.ccE;
    double* T1 = F.ccT1;
    double* T2 = F.ccT2;
    lgp_status st;
#define GEMM(...)                                                    \
    do {                                                             \
        GemmArgs g_ = __VA_ARGS__;                                   \
        if ((st = gemm(GEMM_F64, g_, s)) != LGP_OK) return st;       \
    } while (0)
    // GemmArgs: A,sAb,sAi,sAk, B,sBb,sBk,sBj, C,sCb,sCi,sCj, E,sEb,sEi,sEj, M,N,K,batch, accumulate
    if (F.d == 2) {
        // T1[y][i] = sum_x R[y][x] E[x][i]
        GEMM({r, 0, n1, 1, E, 0, n1, 1, T1, 0, n1, 1, nullptr, 0, 0, 0, n1, n1, n1, 1, 0});
        // T2[j][i] = inv[j][i] * sum_y E[y][j] T1[y][i]
        GEMM({E, 0, 1, n1, T1, 0, n1, 1, T2, 0, n1, 1, F.ccInv, 0, n1, 1, n1, n1, n1, 1, 0});
        // T1[j][x] = sum_i T2[j][i] E[x][i]
        GEMM({T2, 0, n1, 1, E, 0, 1, n1, T1, 0, n1, 1, nullptr, 0, 0, 0, n1, n1, n1, 1, 0});
        // Z[y][x] = sum_j E[y][j] T1[j][x]
        GEMM({E, 0, n1, 1, T1, 0, n1, 1, z, 0, n1, 1, nullptr, 0, 0, 0, n1, n1, n1, 1, 0});
    } else {
        const int nn_i = (int)nn;
        // x: T1[zy][i] = sum_x R[zy][x] E[x][i]
        GEMM({r, 0, n1, 1, E, 0, n1, 1, T1, 0, n1, 1, nullptr, 0, 0, 0, nn_i, n1, n1, 1, 0});
        // y: T2[z][j][i] = sum_y E[y][j] T1[z][y][i]   (batch over z)
        GEMM({E, 0, 1, n1, T1, nn, n1, 1, T2, nn, n1, 1, nullptr, 0, 0, 0, n1, n1, n1, n1, 0});
        // z: T1[l][ji] = inv * sum_z E[z][l] T2[z][ji]
        GEMM({E, 0, 1, n1, T2, 0, nn, 1, T1, 0, nn, 1, F.ccInv, 0, nn, 1, n1, nn_i, n1, 1, 0});
        // back along z: T2[z][ji] = sum_l E[z][l] T1[l][ji]
        GEMM({E, 0, n1, 1, T1, 0, nn, 1, T2, 0, nn, 1, nullptr, 0, 0, 0, n1, nn_i, n1, 1, 0});
        // back along y: T1[z][y][i] = sum_j E[y][j] T2[z][j][i]
        GEMM({E, 0, n1, 1, T2, nn, n1, 1, T1, nn, n1, 1, nullptr, 0, 0, 0, n1, n1, n1, n1, 0});
        // back along x: Z[zy][x] = sum_i T1[zy][i] E[x][i]
        GEMM({T1, 0, n1, 1, E, 0, 1, n1, z, 0, n1, 1, nullptr, 0, 0, 0, nn_i, n1, n1, 1, 0});
    }
#undef GEMM
    return LGP_OK;
}

}  // namespace lgp

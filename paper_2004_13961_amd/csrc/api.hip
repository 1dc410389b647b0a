// extern "C" entry points of liblgpcg (declared and documented in
// include/lgpcg.h).
#include <algorithm>
#include <array>
#include <map>
#include <cmath>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "lgp_internal.h"

using namespace lgp;

namespace lgp {
static std::mutex g_guard_mu;
static std::thread::id g_guard_owner;
static int g_guard_depth = 0;

ThreadGuard::ThreadGuard() {
    std::lock_guard<std::mutex> lk(g_guard_mu);
    const std::thread::id me = std::this_thread::get_id();
    ok = (g_guard_depth == 0 || g_guard_owner == me);
    if (ok) {
        g_guard_owner = me;
        ++g_guard_depth;
    }
}
ThreadGuard::~ThreadGuard() {
    if (!ok) return;
    std::lock_guard<std::mutex> lk(g_guard_mu);
    --g_guard_depth;
}
}  // namespace lgp

struct lgp_problem_s {
    Problem P;
};
struct lgp_factor_s {
    Factor F;
};

extern "C" {

int lgp_version(void) { return 100; }

const char* lgp_status_str(lgp_status s) {
    switch (s) {
        case LGP_OK: return "ok";
        case LGP_E_ARG: return "invalid argument";
        case LGP_E_NOMEM: return "buffer too small";
        case LGP_E_COEF: return "coefficient violates a > 0 at a node, or b below the coercivity bound";
        case LGP_E_ILU_PIVOT: return "ILU(0) pivot <= 0 or not finite";
        case LGP_E_NOCONV: return "no convergence within max_iter";
        case LGP_E_BREAKDOWN: return "PCG breakdown (p'Kp <= 0 or r'z <= 0)";
        case LGP_E_HIP: return "HIP runtime error";
        case LGP_E_UNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

int lgp_last_hip_error(void) { return g_last_hip_error; }

lgp_status lgp_gauss_legendre(int N, double* x, double* w) {
    if (N < 1 || !x || !w) return LGP_E_ARG;
    std::vector<double> xv, wv;
    gauss_legendre_host(N, xv, wv);
    for (int i = 0; i <= N; ++i) {
        x[i] = xv[i];
        w[i] = wv[i];
    }
    return LGP_OK;
}

static bool valid_dims(int d, int N) { return d >= 1 && d <= 3 && N >= 2 && N <= (d == 1 ? 65536 : 4096); }

static void init_problem_dims(Problem& P, int d, int N) {
    P.d = d;
    P.N = N;
    P.n1 = N - 1;
    P.q = N + 1;
    P.n = 1;
    P.nq = 1;
    for (int k = 0; k < d; ++k) {
        P.n *= P.n1;
        P.nq *= P.q;
    }
}

size_t lgp_problem_bytes(int d, int N) {
    if (!valid_dims(d, N)) return 0;
    Problem P;
    init_problem_dims(P, d, N);
    return plan_problem(P, nullptr);
}

static lgp_status build_problem(int d, int N, const double* a_nodes, const double* b_nodes, bool aniso, void* buf,
                                size_t buf_bytes, void* stream, lgp_problem* out) {
    if (!out) return LGP_E_ARG;
    *out = nullptr;
    if (!valid_dims(d, N) || !a_nodes || !b_nodes || !buf) return LGP_E_ARG;
    LGP_ONE_THREAD();
    lgp_problem_s* h = new (std::nothrow) lgp_problem_s();
    if (!h) return LGP_E_NOMEM;
    Problem& P = h->P;
    init_problem_dims(P, d, N);
    P.aniso = aniso;
    if (plan_problem(P, buf) > buf_bytes) {
        delete h;
        return LGP_E_NOMEM;
    }
    hipStream_t s = (hipStream_t)stream;
    lgp_status st = build_tables(P, s);
    bool ok = false;
    if (st == LGP_OK) st = setup_nodes(P, a_nodes, b_nodes, s, &ok);
    if (st == LGP_OK && !ok) st = LGP_E_COEF;
    if (st != LGP_OK) {
        delete h;
        return st;
    }
    *out = h;
    return LGP_OK;
}

lgp_status lgp_build_problem(int d, int N, const double* a_nodes, const double* b_nodes, void* buf,
                             size_t buf_bytes, void* stream, lgp_problem* out) {
    return build_problem(d, N, a_nodes, b_nodes, false, buf, buf_bytes, stream, out);
}

lgp_status lgp_build_problem_diag(int d, int N, const double* a_dir, const double* b_nodes, void* buf,
                                  size_t buf_bytes, void* stream, lgp_problem* out) {
    return build_problem(d, N, a_dir, b_nodes, true, buf, buf_bytes, stream, out);
}

void lgp_destroy_problem(lgp_problem p) { delete p; }

lgp_status lgp_load_vector(lgp_problem p, const double* f_nodes, double* F, void* stream) {
    if (!p || !f_nodes || !F) return LGP_E_ARG;
    LGP_ONE_THREAD();
    return load_vector(p->P, f_nodes, F, (hipStream_t)stream);
}

lgp_status lgp_matvec(lgp_problem p, const void* u, void* y, lgp_dtype prec, void* stream) {
    if (!p || !u || !y || u == y) return LGP_E_ARG;
    LGP_ONE_THREAD();
    hipStream_t s = (hipStream_t)stream;
    switch (prec) {
        case LGP_F64: return matvec_f64(p->P, (const double*)u, (double*)y, s);
        case LGP_F32: return matvec_lp(p->P, (const float*)u, (float*)y, GEMM_F32, s);
        case LGP_BF16: return matvec_lp(p->P, (const float*)u, (float*)y, GEMM_BF16, s);
    }
    return LGP_E_ARG;
}

// ---------------------------------------------------------- pattern ------
// NZ(M) as the union, over the non-negligible series terms, of the offset
// boxes each Kronecker term can reach: for an a-term with degrees
// (tx, ty, tz) the direction carrying S^(t) reaches |delta| <= t and the
// others (carrying M^(t)) reach t + 2; a b-term reaches t + 2 everywhere.
// ca holds d series of (T+1)^d coefficients, direction j (x first) at j*(T+1)^d:
// the term with S^(t) in direction j carries a_j's series.
static std::vector<std::array<int, 3>> pattern_offsets(int d, int T, const std::vector<double>& ca,
                                                      const std::vector<double>& cb) {
    const int T1 = T + 1, h = T + 2, W = 2 * h + 1;
    const int Wz = (d == 3) ? W : 1, hz = (d == 3) ? h : 0;
    // membership on the dense box [-h, h]^d
    std::vector<char> in((size_t)Wz * W * W, 0);
    in[((size_t)hz * W + h) * W + h] = 1;
    auto add_box = [&](int rx, int ry, int rz) {
        for (int z = -rz; z <= rz; ++z)
            for (int y = -ry; y <= ry; ++y) {
                char* row = &in[((size_t)(z + hz) * W + (y + h)) * W + h];
                for (int x = -rx; x <= rx; ++x) row[x] = 1;
            }
    };
    size_t tp = 1;
    for (int k = 0; k < d; ++k) tp *= (size_t)T1;
    const double* cax = ca.data();
    const double* cay = (d >= 2) ? ca.data() + tp : nullptr;
    const double* caz = (d == 3) ? ca.data() + 2 * tp : nullptr;
    if (d == 1) {
        // one direction: an a-term carries S^(t) (reach t), a b-term M^(t)
        for (int t = 0; t <= T; ++t) {
            if (cax[t] != 0.0) add_box(t, 0, 0);
            if (cb[t] != 0.0) add_box(t + 2, 0, 0);
        }
    }
    const int tz_max = (d == 3) ? T : 0, ty_max = (d == 1) ? -1 : T;
    for (int tz = 0; tz <= tz_max; ++tz)
        for (int ty = 0; ty <= ty_max; ++ty)
            for (int tx = 0; tx <= T; ++tx) {
                const size_t ci = ((size_t)tz * T1 + ty) * T1 + tx;
                if (cax[ci] != 0.0) add_box(tx, ty + 2, d == 3 ? tz + 2 : 0);
                if (cay[ci] != 0.0) add_box(tx + 2, ty, d == 3 ? tz + 2 : 0);
                if (d == 3 && caz[ci] != 0.0) add_box(tx + 2, ty + 2, tz);
                if (cb[ci] != 0.0) add_box(tx + 2, ty + 2, d == 3 ? tz + 2 : 0);
            }
    // sorted by (z, y, x)
    std::vector<std::array<int, 3>> out;
    for (int z = -hz; z <= hz; ++z)
        for (int y = -h; y <= h; ++y)
            for (int x = -h; x <= h; ++x)
                if (in[((size_t)(z + hz) * W + (y + h)) * W + (x + h)]) out.push_back({x, y, z});
    return out;
}

static int count_pairs(const std::vector<std::array<int, 3>>& lower, int h) {
    const int R = 4 * h + 1;
    std::vector<char> in((size_t)R * R * R, 0);
    auto key = [&](int a, int b, int c) { return ((size_t)(c + 2 * h) * R + (b + 2 * h)) * R + (a + 2 * h); };
    for (auto& o : lower) in[key(o[0], o[1], o[2])] = 1;
    int cnt = 0;
    for (size_t j = 0; j < lower.size(); ++j)
        for (size_t k = 0; k < j; ++k) {
            const int a = lower[k][0] - lower[j][0], b = lower[k][1] - lower[j][1], c = lower[k][2] - lower[j][2];
            if (in[key(a, b, c)]) ++cnt;
        }
    return cnt;
}

static void set_pattern(Factor& F, const std::vector<std::array<int, 3>>& offs) {
    F.noff = (int)offs.size();
    F.offs.assign(3 * offs.size(), 0);
    F.Hx = F.Hy = F.Hz = 0;
    int diag = -1;
    for (size_t k = 0; k < offs.size(); ++k) {
        F.offs[3 * k] = offs[k][0];
        F.offs[3 * k + 1] = offs[k][1];
        F.offs[3 * k + 2] = offs[k][2];
        F.Hx = std::max(F.Hx, std::abs(offs[k][0]));
        F.Hy = std::max(F.Hy, std::abs(offs[k][1]));
        F.Hz = std::max(F.Hz, std::abs(offs[k][2]));
        if (offs[k][0] == 0 && offs[k][1] == 0 && offs[k][2] == 0) diag = (int)k;
    }
    F.nlo = diag;
    std::vector<std::array<int, 3>> lower(offs.begin(), offs.begin() + diag);
    F.npairs = count_pairs(lower, F.h);
}

static void init_factor_dims(Factor& F, const Problem& P, const int* Tdir, int Tb) {
    F.P = const_cast<Problem*>(&P);
    F.d = P.d;
    F.n1 = P.n1;
    F.n = P.n;
    // the (N+1)-point transform defines Legendre coefficients of degree <= N
    // only (Sec. 2.2), so truncations beyond N keep all of them
    F.Ta = 0;
    for (int j = 0; j < 3; ++j) {
        F.Tdir[j] = (j < P.d) ? std::min(Tdir[j], P.N) : 0;
        F.Ta = std::max(F.Ta, F.Tdir[j]);
    }
    F.Tb = std::min(Tb, P.N);
    F.T = std::max(F.Ta, F.Tb);
    F.h = F.T + 2;
    F.nlines = (P.d == 1) ? 1 : (P.d == 2) ? P.n1 : P.n1 * P.n1;
    F.levels = 0;
}

// factor storage: FP64; FP64 and FP32; FP32 only (d = 3)
static bool valid_store(const Problem& P, lgp_dtype store) {
    return store == LGP_F64 || store == LGP_F32 || (store == LGP_F32_ONLY && P.d == 3);
}

static bool valid_truncations(const Problem& P, const int* Tdir, int Tb) {
    if (!Tdir || Tb < 0 || Tb > 24) return false;
    for (int j = 0; j < P.d; ++j)
        if (Tdir[j] < 0 || Tdir[j] > 24) return false;
    return true;
}

size_t lgp_factor_bytes_dir(lgp_problem p, const int* Ta_dir, int Tb, lgp_dtype store) {
    if (!p || !valid_truncations(p->P, Ta_dir, Tb) || !valid_store(p->P, store)) return 0;
    Factor F;
    init_factor_dims(F, p->P, Ta_dir, Tb);
    // upper bound: the full box |delta_k| <= h
    const int T1 = F.T + 1;
    size_t tp = 1;
    for (int k = 0; k < p->P.d; ++k) tp *= (size_t)T1;
    std::vector<double> ones(tp, 1.0), ones_a((size_t)p->P.d * tp, 1.0);
    set_pattern(F, pattern_offsets(p->P.d, F.T, ones_a, ones));
    return plan_factor(F, nullptr, (int)store);
}

size_t lgp_factor_bytes(lgp_problem p, int Ta, int Tb, lgp_dtype store) {
    const int Tdir[3] = {Ta, Ta, Ta};
    return lgp_factor_bytes_dir(p, Tdir, Tb, store);
}

lgp_status lgp_factor_M_dir(lgp_problem p, const int* Ta_dir, int Tb, lgp_dtype store, void* buf, size_t buf_bytes,
                            void* stream, lgp_factor* out) {
    if (!out) return LGP_E_ARG;
    *out = nullptr;
    if (!p || !buf || !valid_truncations(p->P, Ta_dir, Tb) || !valid_store(p->P, store)) return LGP_E_ARG;
    if (buf_bytes < lgp_factor_bytes_dir(p, Ta_dir, Tb, store)) return LGP_E_NOMEM;
    LGP_ONE_THREAD();
    Problem& P = p->P;
    hipStream_t s = (hipStream_t)stream;
    lgp_factor_s* hF = new (std::nothrow) lgp_factor_s();
    if (!hF) return LGP_E_NOMEM;
    Factor& F = hF->F;
    init_factor_dims(F, P, Ta_dir, Tb);
    const int T = F.T, T1 = T + 1, q = P.q, d = P.d;
    size_t tp = 1;
    for (int k = 0; k < d; ++k) tp *= (size_t)T1;
    lgp_status st = LGP_OK;
    // --- truncated Legendre coefficients: FDLT of the nodal values (Sec. 2.2),
    //     indices <= T per direction, as contractions with
    //     FT[t][m] = (2t+1)/2 w_m L_t(x_m)
    std::vector<double> FT((size_t)T1 * q);
    for (int m = 0; m < q; ++m) {
        double l0 = 1.0, l1 = P.x[m];
        for (int t = 0; t <= T; ++t) {
            double lt;
            if (t == 0) lt = 1.0;
            else if (t == 1) lt = P.x[m];
            else {
                const double l2 = ((2 * (t - 1) + 1) * P.x[m] * l1 - (t - 1) * l0) / t;
                l0 = l1;
                l1 = l2;
                lt = l2;
            }
            FT[(size_t)t * q + m] = (2 * t + 1) / 2.0 * P.w[m] * lt;
        }
    }
    const size_t need0 = (d == 1) ? 0 : (d == 2) ? (size_t)q * T1 : (size_t)q * q * T1;   // stage outputs
    const size_t need1 = (d == 3) ? (size_t)q * T1 * T1 : 0;
    if (need0 > P.s0n || need1 > P.s1n || (size_t)T1 * q > P.s3n || tp > P.s2n) {
        factor_release(hF->F);
        delete hF;
        return LGP_E_UNSUPPORTED;
    }
    // one series per stored diffusion field, then b's
    const int nfa = P.aniso ? d : 1;
    std::vector<double> cf((size_t)nfa * tp), cb(tp);
    double* dFT = P.s3;
    if (hipMemcpyAsync(dFT, FT.data(), FT.size() * 8, hipMemcpyHostToDevice, s) != hipSuccess) {
        factor_release(hF->F);
        delete hF;
        return LGP_E_HIP;
    }
    for (int which = 0; which <= nfa && st == LGP_OK; ++which) {
        const double* src = which < nfa ? P.a_nodes + (size_t)which * P.nq : P.b_nodes;
        double* dst = P.s2;   // (T+1)^d result
        if (d == 1) {
            // C (T1) = FT f
            GemmArgs g1 = {dFT, 0, q, 1, src, 0, 1, 1, dst, 0, 1, 1, nullptr, 0, 0, 0, T1, 1, q, 1, 0};
            st = gemm(GEMM_F64, g1, s);
        } else if (d == 2) {
            // X (q x T1) = f (q x q) FT^T ; C (T1 x T1) = FT X
            GemmArgs g1 = {src, 0, q, 1, dFT, 0, 1, q, P.s0, 0, T1, 1, nullptr, 0, 0, 0, q, T1, q, 1, 0};
            GemmArgs g2 = {dFT, 0, q, 1, P.s0, 0, T1, 1, dst, 0, T1, 1, nullptr, 0, 0, 0, T1, T1, q, 1, 0};
            if ((st = gemm(GEMM_F64, g1, s)) == LGP_OK) st = gemm(GEMM_F64, g2, s);
        } else {
            const int qq = q * q;
            // x: X (q^2 x T1) = f FT^T; y: per z, Y (T1 x T1) = FT X[z]; z: C (T1 x T1^2) = FT Y
            GemmArgs g1 = {src, 0, q, 1, dFT, 0, 1, q, P.s0, 0, T1, 1, nullptr, 0, 0, 0, qq, T1, q, 1, 0};
            GemmArgs g2 = {dFT, 0, q, 1, P.s0, (int64_t)q * T1, T1, 1, P.s1, (int64_t)T1 * T1, T1, 1,
                           nullptr, 0, 0, 0, T1, T1, q, q, 0};
            GemmArgs g3 = {dFT, 0, q, 1, P.s1, 0, (int64_t)T1 * T1, 1, dst, 0, (int64_t)T1 * T1, 1,
                           nullptr, 0, 0, 0, T1, T1 * T1, q, 1, 0};
            if ((st = gemm(GEMM_F64, g1, s)) == LGP_OK && (st = gemm(GEMM_F64, g2, s)) == LGP_OK)
                st = gemm(GEMM_F64, g3, s);
        }
        if (st == LGP_OK) {
            double* h = which < nfa ? cf.data() + (size_t)which * tp : cb.data();
            if (hipMemcpyAsync(h, dst, tp * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                st = LGP_E_HIP;
        }
    }
    if (st != LGP_OK) {
        hipStreamSynchronize(s);   // FT must outlive its queued copy
        factor_release(hF->F);
        delete hF;
        return st;
    }
    // the series of a_j (direction j, x first) kept for indices <= T_j, b's
    // for indices <= Tb; terms below 1e-13 of the largest magnitude over all
    // the series dropped
    std::vector<double> ca((size_t)d * tp);
    double mx = 0.0;
    for (int j = 0; j < d; ++j) {
        const double* fj = cf.data() + (size_t)(P.aniso ? j : 0) * tp;
        const int Tj = F.Tdir[j];
        for (size_t ci = 0; ci < tp; ++ci) {
            const int tx = (int)(ci % T1), ty = (int)((ci / T1) % T1), tz = (d == 3) ? (int)(ci / (T1 * T1)) : 0;
            const bool keep = tx <= Tj && ty <= Tj && tz <= Tj;
            ca[(size_t)j * tp + ci] = keep ? fj[ci] : 0.0;
            mx = std::max(mx, std::fabs(ca[(size_t)j * tp + ci]));
        }
    }
    for (size_t ci = 0; ci < tp; ++ci) {
        const int tx = (int)(ci % T1), ty = (int)((ci / T1) % T1), tz = (d == 3) ? (int)(ci / (T1 * T1)) : 0;
        if (tx > F.Tb || ty > F.Tb || tz > F.Tb) cb[ci] = 0.0;
        mx = std::max(mx, std::fabs(cb[ci]));
    }
    for (size_t ci = 0; ci < (size_t)d * tp; ++ci)
        if (std::fabs(ca[ci]) <= 1e-13 * mx) ca[ci] = 0.0;
    for (size_t ci = 0; ci < tp; ++ci)
        if (std::fabs(cb[ci]) <= 1e-13 * mx) cb[ci] = 0.0;
    set_pattern(F, pattern_offsets(d, T, ca, cb));
    if (plan_factor(F, buf, (int)store) > buf_bytes) {
        factor_release(hF->F);
        delete hF;
        return LGP_E_NOMEM;
    }
    if (hipMemcpyAsync(F.coefA, ca.data(), (size_t)d * tp * 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(F.coefB, cb.data(), tp * 8, hipMemcpyHostToDevice, s) != hipSuccess) {
        hipStreamSynchronize(s);   // ca, cb must outlive their queued copies
        factor_release(hF->F);
        delete hF;
        return LGP_E_HIP;
    }
    st = factor_build(F, s);
    if (st == LGP_OK) {
        int flag = 0;
        if (hipMemcpyAsync(&flag, F.flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            st = LGP_E_HIP;
        else if (flag)
            st = LGP_E_ILU_PIVOT;
    }
    if (st != LGP_OK) {
        factor_release(hF->F);
        delete hF;
        return st;
    }
    *out = hF;
    return LGP_OK;
}

lgp_status lgp_factor_M(lgp_problem p, int Ta, int Tb, lgp_dtype store, void* buf, size_t buf_bytes, void* stream,
                        lgp_factor* out) {
    const int Tdir[3] = {Ta, Ta, Ta};
    return lgp_factor_M_dir(p, Tdir, Tb, store, buf, buf_bytes, stream, out);
}

void lgp_destroy_factor(lgp_factor m) {
    if (!m) return;
    factor_release(m->F);
    delete m;
}

// In one dimension K0 = c_a S + c_b M is banded (half-width 2) and equals
// the T = 0 truncation (a^_0, b^_0 are the means of a and b), whose ILU(0)
// on the full band is its exact LDL^T factorisation: O(N) work, where the
// diagonalisation would need a dense eigenbasis.
size_t lgp_factor_const_bytes(lgp_problem p) {
    if (!p) return 0;
    if (p->P.d == 1) return lgp_factor_bytes(p, 0, 0, LGP_F64);
    return const_factor_bytes(p->P);
}

lgp_status lgp_factor_const(lgp_problem p, void* buf, size_t buf_bytes, void* stream, lgp_factor* out) {
    if (!out) return LGP_E_ARG;
    *out = nullptr;
    if (!p || !buf) return LGP_E_ARG;
    if (buf_bytes < lgp_factor_const_bytes(p)) return LGP_E_NOMEM;
    LGP_ONE_THREAD();
    if (p->P.d == 1) return lgp_factor_M(p, 0, 0, LGP_F64, buf, buf_bytes, stream, out);
    lgp_factor_s* hF = new (std::nothrow) lgp_factor_s();
    if (!hF) return LGP_E_NOMEM;
    lgp_status st = const_factor_build(hF->F, p->P, buf, buf_bytes, (hipStream_t)stream);
    if (st != LGP_OK) {
        factor_release(hF->F);
        delete hF;
        return st;
    }
    *out = hF;
    return LGP_OK;
}

lgp_status lgp_ilu_forward(lgp_factor m, const double* r, double* y, void* stream) {
    if (!m || !r || !y || r == y) return LGP_E_ARG;
    if (m->F.kind != 0) return LGP_E_UNSUPPORTED;
    LGP_ONE_THREAD();
    return sweep(m->F, false, r, y, (hipStream_t)stream);
}

lgp_status lgp_ilu_backward(lgp_factor m, const double* y, double* z, void* stream) {
    if (!m || !y || !z || y == z) return LGP_E_ARG;
    if (m->F.kind != 0) return LGP_E_UNSUPPORTED;
    LGP_ONE_THREAD();
    return sweep(m->F, true, y, z, (hipStream_t)stream);
}

lgp_status lgp_ilu_forward_f32(lgp_factor m, const float* r, float* y, void* stream) {
    if (!m || !r || !y || (const void*)r == (const void*)y) return LGP_E_ARG;
    if (m->F.kind != 0 || !m->F.has32) return LGP_E_UNSUPPORTED;
    LGP_ONE_THREAD();
    return sweep32(m->F, false, r, y, (hipStream_t)stream);
}

lgp_status lgp_ilu_backward_f32(lgp_factor m, const float* y, float* z, void* stream) {
    if (!m || !y || !z || (const void*)y == (const void*)z) return LGP_E_ARG;
    if (m->F.kind != 0 || !m->F.has32) return LGP_E_UNSUPPORTED;
    LGP_ONE_THREAD();
    return sweep32(m->F, true, y, z, (hipStream_t)stream);
}

lgp_status lgp_precond_apply(lgp_factor m, const double* r, double* z, void* stream) {
    if (!m || !r || !z || r == z) return LGP_E_ARG;
    LGP_ONE_THREAD();
    if (m->F.kind == 1) return const_apply(m->F, r, z, (hipStream_t)stream);
    lgp_status st = sweep(m->F, false, r, m->F.y_tmp, (hipStream_t)stream);
    if (st != LGP_OK) return st;
    return sweep(m->F, true, m->F.y_tmp, z, (hipStream_t)stream);
}

lgp_status lgp_factor_describe(lgp_factor m, lgp_factor_desc* out) {
    if (!m || !out) return LGP_E_ARG;
    if (m->F.kind != 0) return LGP_E_UNSUPPORTED;
    const Factor& F = m->F;
    out->d = F.d;
    out->N = F.n1 + 1;
    out->n1 = F.n1;
    out->Ta = F.Ta;
    out->Tb = F.Tb;
    out->n = F.n;
    out->noff = F.noff;
    out->n_lower = F.nlo;
    out->offsets = F.offs.data();
    out->L = F.layout == 1 ? F.A64 : F.L;
    out->D = F.Dg;
    out->levels = F.levels;
    out->ld = F.layout == 1 ? (int)F.ldo : F.ldl;
    out->factor_kernel_ms = F.factor_kernel_ms;
    out->factor_kernel = F.factor_kernel;
    out->layout = F.layout;
    out->invD = F.invD;
    out->factor_launches = F.factor_launches;
    out->factor_waits = F.factor_waits;
    return LGP_OK;
}

size_t lgp_solve_workspace_bytes(lgp_problem p, lgp_dtype inner) {
    if (!p) return 0;
    return solve_ws_bytes(p->P.n, inner != LGP_F64);
}

lgp_status lgp_pcg_solve(lgp_problem p, lgp_factor m, const double* F, double* x, const lgp_solve_opts* opts,
                         void* ws, size_t ws_bytes, void* stream, lgp_solve_info* info) {
    if (!p || !m || !F || !x || !ws || !info) return LGP_E_ARG;
    if (m->F.P != &p->P) return LGP_E_ARG;
    LGP_ONE_THREAD();
    lgp_solve_opts o;
    o.rtol = 1e-10;
    o.max_iter = 2000;
    o.inner = LGP_F64;
    o.inner_rtol = 0.0;
    o.max_outer = 60;
    o.check_every = 4;
    if (opts) {
        o = *opts;
        if (!(o.rtol > 0.0)) return LGP_E_ARG;
        if (o.max_iter <= 0) o.max_iter = 2000;
        if (o.max_outer <= 0) o.max_outer = 60;
        if (o.check_every <= 0) o.check_every = 4;
    }
    // an inner solve only has to gain what its operator's precision allows:
    // BF16 products are accurate to about 1e-2, so asking the inner PCG for
    // more makes it stall; FP32 ones to about 1e-6
    if (!(o.inner_rtol > 0.0)) o.inner_rtol = (o.inner == LGP_BF16) ? 1e-1 : 1e-3;
    lgp_status st = pcg_solve_impl(p->P, m->F, F, x, o, ws, ws_bytes, (hipStream_t)stream, info);
    info->status = st;
    return st;
}


// ------------------------------------------------------------ batches ----
struct lgp_batch_s {
    Batch* B;
};

static int nlines_of(const Problem& P) { return P.d == 3 ? P.n1 * P.n1 : (P.d == 2 ? P.n1 : 1); }

static bool opts_from(const lgp_solve_opts* opts, lgp_solve_opts& o) {
    o.rtol = 1e-10;
    o.max_iter = 2000;
    o.inner = LGP_F64;
    o.inner_rtol = 0.0;
    o.max_outer = 60;
    o.check_every = 4;
    if (opts) {
        o = *opts;
        if (!(o.rtol > 0.0)) return false;
        if (o.max_iter <= 0) o.max_iter = 2000;
        if (o.max_outer <= 0) o.max_outer = 60;
        if (o.check_every <= 0) o.check_every = 4;
    }
    return o.inner == LGP_F64;
}

size_t lgp_batch_workspace_bytes(lgp_problem shape, int slots) {
    if (!shape || slots < 1 || slots > 4096) return 0;
    return batch_ws_bytes(shape->P.n, nlines_of(shape->P), slots);
}

lgp_status lgp_batch_create(lgp_problem shape, int slots, void* ws, size_t ws_bytes, void* stream, lgp_batch* out) {
    if (!out) return LGP_E_ARG;
    *out = nullptr;
    if (!shape || !ws || slots < 1 || slots > 4096) return LGP_E_ARG;
    lgp_status st = LGP_OK;
    Batch* B = batch_create(shape->P, slots, ws, ws_bytes, (hipStream_t)stream, &st);
    if (!B) return st;
    lgp_batch_s* h = new (std::nothrow) lgp_batch_s{B};
    if (!h) {
        batch_destroy(B);
        return LGP_E_NOMEM;
    }
    *out = h;
    return LGP_OK;
}

lgp_status lgp_batch_add(lgp_batch b, lgp_problem p, lgp_factor m, const double* F, double* x,
                         const lgp_solve_opts* opts, int* slot) {
    if (!b || !p || !m || !F || !x || !slot) return LGP_E_ARG;
    lgp_solve_opts o;
    if (!opts_from(opts, o)) return opts && opts->inner != LGP_F64 ? LGP_E_UNSUPPORTED : LGP_E_ARG;
    LGP_ONE_THREAD();
    return batch_add(b->B, p->P, m->F, F, x, o, slot);
}

lgp_status lgp_batch_step(lgp_batch b, int iters, int* running) {
    if (!b || iters < 0 || !running) return LGP_E_ARG;
    LGP_ONE_THREAD();
    return batch_step(b->B, iters, running);
}

lgp_status lgp_batch_info(lgp_batch b, int slot, lgp_solve_info* info, int* finished) {
    if (!b || !info || !finished) return LGP_E_ARG;
    return batch_info(b->B, slot, info, finished);
}

lgp_status lgp_batch_remove(lgp_batch b, int slot) {
    if (!b) return LGP_E_ARG;
    return batch_remove(b->B, slot);
}

void lgp_batch_destroy(lgp_batch b) {
    if (!b) return;
    batch_destroy(b->B);
    delete b;
}

lgp_status lgp_pcg_solve_batched(int count, const lgp_problem* p, const lgp_factor* m, const double* const* F,
                                 double* const* x, const lgp_solve_opts* opts, void* ws, size_t ws_bytes,
                                 void* stream, lgp_solve_info* info) {
    if (count < 1 || !p || !m || !F || !x || !ws || !info) return LGP_E_ARG;
    for (int k = 0; k < count; ++k)
        if (!p[k] || !m[k] || !F[k] || !x[k]) return LGP_E_ARG;
    lgp_batch b = nullptr;
    lgp_status st = lgp_batch_create(p[0], count, ws, ws_bytes, stream, &b);
    if (st != LGP_OK) return st;
    std::vector<int> slot(count, -1);
    for (int k = 0; k < count && st == LGP_OK; ++k) st = lgp_batch_add(b, p[k], m[k], F[k], x[k], opts, &slot[k]);
    const int every = (opts && opts->check_every > 0) ? opts->check_every : 4;
    int running = 1;
    while (st == LGP_OK && running > 0) st = lgp_batch_step(b, every, &running);
    lgp_status worst = st;
    for (int k = 0; k < count && st == LGP_OK; ++k) {
        int fin = 0;
        lgp_batch_info(b, slot[k], &info[k], &fin);
        if (info[k].status != LGP_OK && worst == LGP_OK) worst = info[k].status;
    }
    lgp_batch_destroy(b);
    return worst;
}

// ------------------------------------------------- allocation-free solve --
// Workspace of lgp_pcg_solve_noalloc: one file-scope device array, one copy
// per GPU, shared by every call on that GPU.
static __device__ __align__(256) unsigned char scratch[LGP_NOALLOC_SCRATCH_BYTES];

// Device address of this GPU's copy of `scratch`, taken once per device with
// that device current (host code never passes the array's name itself).
static lgp_status noalloc_scratch(void** out) {
    static std::mutex mu;
    static std::map<int, void*> addr;
    int dev = 0;
    LGP_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void* ptr = nullptr;
        LGP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return LGP_E_HIP;
        it = addr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return LGP_OK;
}

size_t lgp_pcg_solve_noalloc_max_bytes(void) { return (size_t)LGP_NOALLOC_SCRATCH_BYTES; }

lgp_status lgp_pcg_solve_noalloc(lgp_problem p, lgp_factor m, const double* F, double* x,
                                 const lgp_solve_opts* opts, void* stream, lgp_solve_info* info) {
    if (!p || !m || !F || !x || !info) return LGP_E_ARG;
    const size_t need = lgp_solve_workspace_bytes(p, opts ? opts->inner : LGP_F64);
    if (need == 0 || need > (size_t)LGP_NOALLOC_SCRATCH_BYTES) {
        info->status = LGP_E_NOMEM;
        return LGP_E_NOMEM;
    }
    void* ws = nullptr;
    {
        LGP_ONE_THREAD();
        lgp_status st = noalloc_scratch(&ws);
        if (st != LGP_OK) return st;
    }
    // the solver sets every workspace entry it reads before reading it, so
    // what an earlier call left in the array does not matter
    return lgp_pcg_solve(p, m, F, x, opts, ws, (size_t)LGP_NOALLOC_SCRATCH_BYTES, stream, info);
}

// ------------------------------------------------- fast transforms -------
struct lgp_dlt_s {
    lgp::Dlt* D;
};

size_t lgp_dlt_bytes(lgp_problem p) {
    if (!p || !lgp::dlt_supported(p->P)) return 0;
    return lgp::dlt_bytes(p->P);
}

lgp_status lgp_dlt_create(lgp_problem p, void* buf, size_t buf_bytes, void* stream, lgp_dlt* out) {
    if (!p || !buf || !out) return LGP_E_ARG;
    if (!lgp::dlt_supported(p->P)) return LGP_E_UNSUPPORTED;
    LGP_ONE_THREAD();
    lgp_dlt_s* h = new (std::nothrow) lgp_dlt_s();
    if (!h) return LGP_E_NOMEM;
    lgp_status st = LGP_OK;
    h->D = lgp::dlt_create(p->P, buf, buf_bytes, (hipStream_t)stream, &st);
    if (!h->D) {
        delete h;
        return st;
    }
    *out = h;
    return LGP_OK;
}

lgp_status lgp_dlt_lines(lgp_dlt h, int forward, int64_t count, const double* in, double* out, void* stream) {
    if (!h || !in || !out) return LGP_E_ARG;
    LGP_ONE_THREAD();
    return lgp::dlt_apply(*h->D, forward != 0, count, in, out, (hipStream_t)stream);
}

lgp_status lgp_matvec_fast(lgp_dlt h, const double* u, double* y, void* stream) {
    if (!h || !u || !y || u == y) return LGP_E_ARG;
    LGP_ONE_THREAD();
    return lgp::matvec_fast(*h->D, u, y, (hipStream_t)stream);
}

int lgp_dlt_blocks(lgp_dlt h) { return h ? lgp::dlt_blocks(*h->D) : 0; }

void lgp_dlt_destroy(lgp_dlt h) {
    if (!h) return;
    lgp::dlt_destroy(h->D);
    delete h;
}

}  // extern "C"

// Internal declarations shared by the HIP translation units of liblgpcg.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <vector>

#include "../../include/lgpcg.h"

namespace lgp {

extern thread_local int g_last_hip_error;

// Size of the device array that serves as the workspace of
// lgp_pcg_solve_noalloc (one copy per GPU).
#define LGP_NOALLOC_SCRATCH_BYTES (64u << 20)

#define LGP_HIP(call)                                                   \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) {                                         \
            ::lgp::g_last_hip_error = (int)e_;                          \
            return LGP_E_HIP;                                           \
        }                                                               \
    } while (0)

#define LGP_CHECK_LAUNCH()                                              \
    do {                                                                \
        hipError_t e_ = hipGetLastError();                              \
        if (e_ != hipSuccess) {                                         \
            ::lgp::g_last_hip_error = (int)e_;                          \
            return LGP_E_HIP;                                           \
        }                                                               \
    } while (0)

// At most one host thread at a time may be inside an entry point that
// enqueues device work; a call from a second thread while another thread is
// inside returns LGP_E_UNSUPPORTED. Nested calls on the owning thread pass.
struct ThreadGuard {
    bool ok;
    ThreadGuard();
    ~ThreadGuard();
    ThreadGuard(const ThreadGuard&) = delete;
    ThreadGuard& operator=(const ThreadGuard&) = delete;
};
#define LGP_ONE_THREAD()                                                \
    ::lgp::ThreadGuard lgp_guard_;                                      \
    if (!lgp_guard_.ok) return LGP_E_UNSUPPORTED

// Bump allocator over a caller-provided device buffer (256-byte aligned
// sub-buffers). Used twice: once with base == nullptr to size, once to carve.
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// ------------------------------------------------------------- GEMM ------
// C[b](i,j) (+)= E[b](i,j) * sum_k A[b](i,k) B[b](k,j), element addresses via
// strides (in elements). E may be null (no epilogue multiply).
enum GemmMode { GEMM_F64 = 0, GEMM_F32 = 1, GEMM_BF16 = 2 };

struct GemmArgs {
    const void* A; int64_t sAb, sAi, sAk;
    const void* B; int64_t sBb, sBk, sBj;
    void* C;       int64_t sCb, sCi, sCj;
    const void* E; int64_t sEb, sEi, sEj;
    int M, N, K, batch;
    int accumulate;
    const int* stop = nullptr;   // device flag: when set, the launch returns at once (PCG has converged)
};

lgp_status gemm(GemmMode mode, const GemmArgs& g, hipStream_t s);

// ----------------------------------------------------------- problem -----
struct Problem {
    int d, N, n1, q;
    int64_t n, nq;            // (N-1)^d, (N+1)^d
    std::vector<double> x, w; // host nodes / weights
    // device tables (FP64)
    double* PDT;    // [n1][2q]  : [Phi^T | D^T]          (PDT[k][m] = Phi[m][k], PDT[k][q+m] = D[m][k])
    double* PhiD;   // [2q][n1]  : [Phi ; D]
    double* DP;     // [2q][n1]  : [D ; Phi]
    double* Wnodes; // [nq] tensor weights
    double* wab;    // [1+d][nq] : W*b, then W*a_j for j = d-1 .. 0 (z, y, x: the
                    //             field of the derivative the stage takes)
    double* a_nodes;// [d][nq] copy of a_j (x first); isotropic: a in slot 0 only
    bool aniso;     // one diffusion field per direction (Example 4)
    double* b_nodes;// [nq]  copy of b
    // FP32 copies for the low-precision matvec
    float* PDT32; float* PhiD32; float* DP32; float* wab32;
    // matvec scratch (sized for the largest stage), FP64 and FP32 views share it
    double* s0; double* s1; double* s2; double* s3;
    size_t s0n, s1n, s2n, s3n;
    int* flag;      // device status flag
    double* cmin;   // [2*256 + 2] per-block minima of a and b, then (min a, min b)
    size_t bytes;
};

size_t plan_problem(Problem& P, void* buf);
lgp_status matvec_f64(Problem& P, const double* u, double* y, hipStream_t s, const int* stop = nullptr);
lgp_status matvec_lp(Problem& P, const float* u, float* y, GemmMode mode, hipStream_t s, const int* stop = nullptr);
lgp_status load_vector(Problem& P, const double* f, double* F, hipStream_t s);

// ------------------------------------------------- fast transforms -------
struct Dlt;
bool dlt_supported(const Problem& P);
size_t dlt_bytes(Problem& P);
Dlt* dlt_create(Problem& P, void* buf, size_t bytes, hipStream_t s, lgp_status* st);
void dlt_destroy(Dlt* D);
lgp_status dlt_apply(Dlt& D, bool forward, int64_t count, const double* in, double* out, hipStream_t s);
lgp_status matvec_fast(Dlt& D, const double* u, double* y, hipStream_t s);
int dlt_blocks(const Dlt& D);

// ------------------------------------------------------------ factor -----
struct Factor {
    Problem* P;
    int d, n1, Ta, Tb, T, h;   // h = reach of the pattern per direction
    int Tdir[3];               // truncation of a_j per direction (all Ta if isotropic)
    int64_t n;
    int noff, nlo;             // pattern size, number of strictly lower offsets
    int ldl;                   // row stride of L / Ut (>= nlo + 1, multiple of 32 doubles)
    std::vector<int> offs;     // host, 3*noff
    int Hx, Hy, Hz;            // max |offset| per direction
    int nlines;                // lines of constant (y,z)
    int levels;
    // device
    double* L;        // [n+1][ldl]: L(i, i+delta_k) at k < nlo, 1/D(i) at nlo; row n is zero
    double* Ut;       // [n][ldl]  backward-sweep operator in reversed order
    double* Dg;       // [n] pivots
    double* invD;     // [n]
    float* L32; float* Ut32; float* invD32;   // optional FP32 copies
    int* d_offs;      // [nlo][4] (dx,dy,dz,linear)
    int* line_order;  // [nlines] line ids in dependency order
    unsigned* prog;   // [2][nlines] progress counters (fwd, bwd)
    unsigned* ticket; // [4]
    int* flag;        // [4] device flags
    double* coefA;    // [d][(T+1)^d] truncated coefficients of a_j (x fastest), j = 0 (x) first
    double* coefB;    // [(T+1)^d]
    double* band;     // [2][T+1][n1][2h+1]  S^(t)(i, i+delta), M^(t)(i, i+delta)
    int* pair_ptr;    // [nlo+1]  CSR over k: rows j > k with offset(k)-offset(j) lower
    int* pair_j;      // [npairs] j index (lower offset index, or nlo for the diagonal)
    int* pair_l;      // [npairs] index of offset(k) - offset(j) in the lower list
    int npairs;
    int maxpairs;     // largest pair list of one lower offset
    int* steps;       // [nlo][4] {j, linear offset, first pair, end pair} in dataflow order
    int* sdxyz;       // [nlo] packed (dx+128) | (dy+128) << 8 | (dz+128) << 16 of each step
    unsigned* pairw;  // [npairs] k*8 | (l*8) << 16 (byte offsets), grouped by step
    int maxlev;       // number of hyperplane levels
    int* lev;         // [maxlev + 1] first ticket of each level, then [maxlev] fill counters
    int* runs;        // [nruns][4] runs of lower offsets with equal (dy, dz): {kb, ke, dx_first, dx_last}
    int nruns;
    float factor_kernel_ms;   // duration of the ILU(0) kernel of the last build (HIP events)
    int factor_kernel;        // 2: dataflow kernel, 1: generic kernel
    int factor_launches;      // launches of that kernel in the last build
    int factor_waits = 0;     // 3D chunked kernel: steps that found a row they read not yet written
    // kind 1: the constant-coefficient operator solved exactly (matrix
    // diagonalisation); only P, d, n1, n and the cc* fields are used
    int kind = 0;
    double* ccE = nullptr;     // [n1][n1] generalized eigenvectors, E^T S E = I, E^T M E = diag(lam)
    double* ccLam = nullptr;   // [n1]
    double* ccInv = nullptr;   // [n1^d] 1 / eigenvalues of the transformed operator
    double* ccT1 = nullptr;    // [n1^d] scratch
    double* ccT2 = nullptr;    // [n1^d] scratch
    double* ccPart = nullptr;  // [4*256 + 4] partial sums per field, then the means (c_b, c_a of z, y, x)
    double* y_tmp;    // [n] intermediate of precond_apply
    bool has32;
    bool has64 = true;        // FP64 factor kept (FP64 solves possible)
    size_t bytes;
    // d = 3: factor stored offset-major, A[k * ldo + i] = L(i, i + delta_k),
    // so that both substitutions read it in contiguous runs of rows; rows
    // are factored in an FP64 window (`ring`) of the rows still needed
    int layout = 0;            // 0: row-major L (and Ut); 1: offset-major A64 / A32
    int64_t ldo = 0;           // row stride of the offset-major arrays (>= n)
    double* A64 = nullptr;     // [nlo][ldo], null when only FP32 is kept
    float* A32 = nullptr;      // [nlo][ldo] FP32 copy for the inner sweeps
    double* ring = nullptr;    // [ring_rows + 1][ldl] FP64 rows; the last one is zero
    int64_t ring_rows = 0;     // rows of the window (ring_planes whole z-planes)
    int ring_planes = 0;
    int fB = 0;                // rows per chunk (waves per workgroup) of the 3D factor, 0: generic kernel
    int nxb = 0;               // chunks per grid line
    int nchunks = 0;
    int* chunk_order = nullptr;   // [nchunks] chunk ids in dependency order
    int* chunk_rank = nullptr;    // [nchunks] position of each chunk in that order
    int* pk = nullptr;            // [npk][4] packets of the steps' pair lists {step, first pair, count, last}
    int npk = 0;
    int sBX = 8;                  // rows per block of the 3D substitutions
    int snxb = 0;                 // blocks per line
    int* blk_order = nullptr;     // [nlines * snxb] substitution blocks in dependency order
    int* own = nullptr;           // [8] offset index of (-m, 0, 0), m = 1..8 (-1 if absent)
    double* fold3 = nullptr;      // folded line coefficients of the 3D path
    // box positions of the chunked 3D kernel (u vectors and window rows)
    int bX = 0, bXY = 0, bP0 = 0, bPD = 0;   // x extent, plane size, diagonal position, 1/D slot
    int ldr = 0;                  // window row length (doubles)
    unsigned* pw16 = nullptr;     // pair positions, two 16-bit byte offsets per word
    int* kofp = nullptr;          // [bP0] lower offset index at each box position, or -1
};

// One slot of a batched substitution: the operator and vectors of one
// request (same grid and pattern as the others of the batch). prog: the
// slot's per-line progress counters (3D kernel), stop: the slot's PCG done flag.
template <typename T>
struct SweepSlot {
    const T* A;
    const T* scale;
    const T* in;
    T* out;
    unsigned* prog;
    const int* stop;
};
// substitutions of nslots requests in one launch (slots: device table);
// ticket: one counter; returns LGP_E_UNSUPPORTED where no batched kernel
// serves the pattern
lgp_status sweep_batch(const Factor& ref, int nslots, const SweepSlot<double>* slots, bool backward,
                       unsigned* ticket, hipStream_t s);
lgp_status sweep3_batch(const Factor& ref, int nslots, const SweepSlot<double>* slots, bool backward,
                        unsigned* ticket, hipStream_t s);
int gemm_tuned_variant(GemmMode mode, const GemmArgs& g);

// storage requested for the factor (lgp_dtype values of the ABI)
enum { STORE_F64 = 0, STORE_F64_F32 = 1, STORE_F32_ONLY = 3 };
size_t plan_factor(Factor& F, void* buf, int store);
size_t plan_factor3(Factor& F, void* buf, int store);
lgp_status factor_build3(Factor& F, hipStream_t s, std::vector<int>& off4, std::vector<int>& st4,
                         std::vector<int>& sd, std::vector<unsigned>& pw, hipEvent_t* ev);
lgp_status sweep3(Factor& F, bool backward, bool lowp, const void* in, void* out, hipStream_t s,
                  const int* stop);
lgp_status factor_build(Factor& F, hipStream_t s);
void factor_release(Factor& F);
size_t const_factor_bytes(const Problem& P);
lgp_status const_factor_build(Factor& F, Problem& P, void* buf, size_t bytes, hipStream_t s);
lgp_status const_apply(Factor& F, const double* r, double* z, hipStream_t s);
lgp_status sweep(Factor& F, bool backward, const double* in, double* out, hipStream_t s,
                 const int* stop = nullptr);
lgp_status sweep32(Factor& F, bool backward, const float* in, float* out, hipStream_t s,
                   const int* stop = nullptr);

// PCG driver
struct Batch;
size_t batch_ws_bytes(int64_t n, int nlines, int cap);
Batch* batch_create(Problem& shape, int cap, void* ws, size_t ws_bytes, hipStream_t s, lgp_status* st);
void batch_destroy(Batch* B);
lgp_status batch_add(Batch* B, Problem& P, Factor& M, const double* F, double* x, const lgp_solve_opts& o, int* slot);
lgp_status batch_step(Batch* B, int iters, int* running);
lgp_status batch_info(Batch* B, int k, lgp_solve_info* info, int* finished);
lgp_status batch_remove(Batch* B, int k);
size_t solve_ws_bytes(int64_t n, bool mixed);
lgp_status pcg_solve_impl(Problem& P, Factor& M, const double* F, double* x, const lgp_solve_opts& o, void* ws,
                          size_t ws_bytes, hipStream_t s, lgp_solve_info* info);
lgp_status build_tables(Problem& P, hipStream_t s);
lgp_status setup_nodes(Problem& P, const double* a, const double* b, hipStream_t s, bool* coef_ok);
// offset of the weighted field of direction j (0 = x) in wab / wab32
inline int64_t wa_offset(const Problem& P, int j) { return (int64_t)(1 + (P.d - 1 - j)) * P.nq; }

// host helpers
void gauss_legendre_host(int N, std::vector<double>& x, std::vector<double>& w);
__host__ __device__ double triple_legendre(int t, int m, int n);   // int L_t L_m L_n over (-1,1)

}  // namespace lgp

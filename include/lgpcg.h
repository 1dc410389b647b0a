/* lgpcg.h - C ABI of the MI355X (gfx950) preconditioned Legendre-Galerkin
 * PCG solver for  -div(a grad u) + b u = f  on (-1,1)^d, u = 0 on the
 * boundary, d = 1, 2 or 3 (Diao, Hu, Ma, arXiv 2004.13961; d = 1 is the
 * setting of the paper's Example 1, solved by the same entry points).
 *
 * Discretisation (paper Sec. 3): unknowns are the coefficients of the compact
 * basis phi_k = L_k - L_{k+2}, k = 0..N-2, in tensor form, x index fastest:
 * a vector has (N-1)^d doubles, entry [kx + (N-1)*(ky + (N-1)*kz)].
 * Coefficients a, b and data f enter as values at the (N+1)^d tensor grid of
 * Legendre-Gauss nodes (roots of L_{N+1}, Sec. 2.2), x fastest, node order
 * ascending (see lgp_gauss_legendre). The operator K = A + B is the one of
 * the fast matrix-vector product of Sec. 4.3: the bilinear form with I_N
 * applied to a grad u and b u, i.e. (N+1)-point Gauss quadrature per
 * direction.
 *
 * Conventions for every entry point:
 *   - Pointers marked "device" are HIP device pointers; the others are host.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream). All
 *     device work is enqueued on it; a call returns after enqueueing unless
 *     its comment says it synchronises.
 *   - The caller allocates every device byte (size queries below) and keeps
 *     it alive until the handle that uses it is destroyed. The library never
 *     allocates device memory. Handles are small host objects owned by the
 *     library and released by the matching destroy call.
 *   - Every function returns an lgp_status; nothing throws across the ABI.
 *     After a non-OK build or factor the handle is not created.
 *   - Calls on one handle must be ordered on a single stream.
 *   - One host thread at a time: an entry point that enqueues device work,
 *     called from a second thread while another thread is inside the
 *     library, returns LGP_E_UNSUPPORTED without enqueueing anything.
 *     Requests that should overlap on the device go through the batched
 *     entry points below, from one thread. (Several request streams driven
 *     from several threads once stopped making progress; the library now
 *     uses only the caller's stream, but the case is not served.)
 */
#ifndef LGPCG_H
#define LGPCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LGP_OK = 0,
    LGP_E_ARG = 1,        /* bad argument: d not in {1,2,3}, N out of range, null pointer, T out of
                             range, or a NaN / infinity in F or in the initial guess of a solve */
    LGP_E_NOMEM = 2,      /* caller buffer smaller than the size query returned */
    LGP_E_COEF = 3,       /* a <= 0 or a non-finite value at a node, or min b <= -(d pi^2/4) min a */
    LGP_E_ILU_PIVOT = 4,  /* ILU(0) pivot <= 0 or non-finite (Alg. 2 assumes existence) */
    LGP_E_NOCONV = 5,     /* max_iter reached before the stop rule of Alg. 1 */
    LGP_E_BREAKDOWN = 6,  /* p'Kp <= 0 or r'z <= 0 in PCG, or a non-finite residual after iterating */
    LGP_E_HIP = 7,        /* a HIP runtime call failed; see lgp_last_hip_error */
    LGP_E_UNSUPPORTED = 8 /* valid request the library does not serve */
} lgp_status;

/* Precisions. LGP_F32_ONLY is a factor storage only (lgp_factor_M, d = 3):
 * the factor is kept in FP32 alone, for mixed-precision solves. */
typedef enum { LGP_F64 = 0, LGP_F32 = 1, LGP_BF16 = 2, LGP_F32_ONLY = 3 } lgp_dtype;

typedef struct lgp_problem_s* lgp_problem;
typedef struct lgp_factor_s* lgp_factor;

/* ----------------------------------------------------------- utilities -- */
int lgp_version(void);
const char* lgp_status_str(lgp_status s);
int lgp_last_hip_error(void);            /* last hipError_t seen, 0 if none */

/* Legendre-Gauss nodes (roots of L_{N+1}, Sec. 2.2) in ascending order and
 * their weights; x and w are host arrays of N+1 doubles. Newton iteration on
 * the three-term recurrence of Sec. 2.1. */
lgp_status lgp_gauss_legendre(int N, double* x, double* w);

/* ------------------------------------------------------------ problem -- */
/* Device bytes needed by lgp_build_problem for (d, N); 0 if (d, N) is out
 * of range (d in 1..3, 2 <= N <= 4096, or N <= 65536 for d = 1). */
size_t lgp_problem_bytes(int d, int N);

/* Build the operator K = A + B of Sec. 3 / Sec. 4.3 from nodal coefficient
 * values a_nodes, b_nodes (device, (N+1)^d doubles each, x fastest). The
 * model problem of Sec. 3 asks a > 0 and b >= 0, but the paper's own test
 * coefficients (Sec. 5.2) take b < 0 near a corner; what the method needs
 * is a coercive form, which holds when min b > -(d pi^2/4) min a (Poincare
 * inequality on (-1,1)^d). The call checks a > 0 and finiteness at every
 * node and that bound, and returns LGP_E_COEF otherwise (it synchronises
 * `stream` for that check). The nodal arrays are copied; buf (device, buf_bytes >=
 * lgp_problem_bytes) holds tables, weighted coefficients and matvec
 * scratch and must outlive the handle. */
lgp_status lgp_build_problem(int d, int N, const double* a_nodes, const double* b_nodes,
                             void* buf, size_t buf_bytes, void* stream, lgp_problem* out);

/* The diagonal anisotropic form of Example 4 (Sec. 5.2):
 *   -sum_j (a_j u_{x_j})_{x_j} + b u = f,  one diffusion field per direction.
 * a_dir (device, d * (N+1)^d doubles) holds a_1 (the x field), then a_2,
 * then a_3, each on the full node grid, x fastest (Example 4's a_j depend on
 * x_j only, but any positive fields are accepted). The bilinear form weights
 * the j-th gradient component by I_N a_j. Checks, errors, buffer (same size
 * as lgp_problem_bytes(d, N)) and ownership as lgp_build_problem; every
 * other entry point accepts the handle. For d = 1 it is lgp_build_problem. */
lgp_status lgp_build_problem_diag(int d, int N, const double* a_dir, const double* b_nodes,
                                  void* buf, size_t buf_bytes, void* stream, lgp_problem* out);
void lgp_destroy_problem(lgp_problem p);

/* Load vector F_k = (I_N f, psi_k) (Sec. 3 with the quadrature of Sec. 4.3):
 * f_nodes device (N+1)^d, F device (N-1)^d. Uses the problem's scratch. */
lgp_status lgp_load_vector(lgp_problem p, const double* f_nodes, double* F, void* stream);

/* y = (A + B) u, the fast matrix-vector product of Sec. 4.3 computed by
 * sum-factorised contractions on the matrix cores. prec = LGP_F64: u, y are
 * double. prec = LGP_F32: u, y are float, contractions in FP32. prec =
 * LGP_BF16: u, y are float, contraction operands rounded to bfloat16 with
 * FP32 accumulation. u and y must not alias. Uses the problem's scratch, so
 * matvecs on one problem must be stream-ordered. */
lgp_status lgp_matvec(lgp_problem p, const void* u, void* y, lgp_dtype prec, void* stream);

/* ------------------------------------------------------ preconditioner -- */
/* Device bytes for the ILU(0) factors of M with truncation degrees Ta (for
 * a) and Tb (for b); store = LGP_F32 adds single-precision copies of the
 * factors for the inner sweeps of the mixed-precision solve; store =
 * LGP_F32_ONLY (d = 3) keeps the single-precision factor alone (the
 * factorisation still runs in FP64, over a window of the rows still being
 * read, at most 24 GiB): such a factor serves mixed-precision solves only,
 * and an FP64 solve with it returns LGP_E_UNSUPPORTED. Returns 0 for a
 * store the dimension does not take. */
size_t lgp_factor_bytes(lgp_problem p, int Ta, int Tb, lgp_dtype store);

/* Preconditioner of Sec. 4.1: a and b replaced by their Legendre series
 * truncated to indices <= Ta (resp. Tb) in each direction (coefficients =
 * the discrete Legendre transform of the nodal values, Sec. 2.2, which
 * defines degrees <= N only: Ta, Tb above N act as N; terms below 1e-13 of
 * the largest are dropped), M assembled exactly (product formula,
 * Lemma LegProduct; Kronecker form of Sec. 4.2), then ILU(0) (Alg. 2) in
 * FP64 on the GPU over NZ(M). Because M and NZ(M) are symmetric the factor
 * is stored as unit-lower L plus pivots D, with U = D L^T. For d = 1, M is
 * banded and NZ(M) is its whole band, so ILU(0) is the exact banded
 * factorisation, and the substitutions are sequential over the rows. Returns
 * LGP_E_ILU_PIVOT if a pivot is <= 0 or non-finite. Synchronises `stream`
 * (pattern selection and the pivot check read device results). */
lgp_status lgp_factor_M(lgp_problem p, int Ta, int Tb, lgp_dtype store,
                        void* buf, size_t buf_bytes, void* stream, lgp_factor* out);

/* Per-direction truncations t_{1j} (Example 4, Sec. 5.2): Ta_dir (host, d
 * ints, each 0..24) truncates the series of a_j (or of the one field a of
 * an isotropic problem in the terms where direction j carries S^(t)) at
 * indices <= Ta_dir[j] per direction; Tb as above. lgp_factor_M(p, Ta, Tb,
 * ...) is this call with Ta_dir = {Ta, Ta, Ta}. Returns LGP_E_ARG for a
 * truncation outside 0..24, otherwise as lgp_factor_M. */
size_t lgp_factor_bytes_dir(lgp_problem p, const int* Ta_dir, int Tb, lgp_dtype store);
lgp_status lgp_factor_M_dir(lgp_problem p, const int* Ta_dir, int Tb, lgp_dtype store,
                            void* buf, size_t buf_bytes, void* stream, lgp_factor* out);
void lgp_destroy_factor(lgp_factor m);

/* The constant-coefficient preconditioner of the comparison method PCG-I
 * (Sec. 5.2): a and b replaced by their series truncated at T = 0 (their
 * weighted means c_a, c_b, Sec. 4.1), i.e.
 *   K0 = c_a (S (x) M + M (x) S) + c_b M (x) M      (2D; three terms in 3D)
 * (for the anisotropic form, c_a (S (x) M) becomes c_{a_1} M (x) S and
 * c_{a_2} S (x) M, kron order y, x: one mean per field)
 * with the exact 1D stiffness S = diag(4k+6) and the pentadiagonal 1D mass M
 * of the compact basis (Sec. 2.1, 3). The paper solves K0 by a fast direct
 * method; here it is inverted exactly by matrix diagonalisation (generalized
 * eigenvectors of (M, S), computed once per N on the host in FP64 and
 * cached; 2d dense contractions per application on the GPU). The handle
 * works with lgp_precond_apply (z = K0^{-1} r) and with lgp_pcg_solve for
 * inner = LGP_F64 (PCG-I); lgp_ilu_forward, lgp_ilu_backward and
 * lgp_factor_describe return LGP_E_UNSUPPORTED for it, and so does
 * lgp_pcg_solve with a low-precision inner solve. Buffer: device bytes from
 * lgp_factor_const_bytes, owned by the caller. Synchronises `stream`.
 * For d = 1, K0 = c_a S + c_b M is banded and equals the T = 0 truncation
 * of lgp_factor_M, so this call returns lgp_factor_M(p, 0, 0, LGP_F64, ...):
 * an exact banded factorisation, an ordinary ILU(0) handle (all of the
 * entry points above accept it). */
size_t lgp_factor_const_bytes(lgp_problem p);
lgp_status lgp_factor_const(lgp_problem p, void* buf, size_t buf_bytes, void* stream, lgp_factor* out);

/* One-step preconditioner application of Sec. 4.2: z = U^{-1} L^{-1} r
 * (forward substitution Alg. 3, then backward substitution Alg. 4); for a
 * handle from lgp_factor_const, z = K0^{-1} r. r, z device (N-1)^d doubles;
 * must not alias. */
lgp_status lgp_precond_apply(lgp_factor m, const double* r, double* z, void* stream);
/* The two halves separately: y = L^{-1} r (Alg. 3) and z = U^{-1} y (Alg. 4). */
lgp_status lgp_ilu_forward(lgp_factor m, const double* r, double* y, void* stream);
lgp_status lgp_ilu_backward(lgp_factor m, const double* y, double* z, void* stream);
/* The same two substitutions in single precision on the FP32 copy of the
 * factor (the inner sweeps of the mixed-precision solve): r, y, z device
 * (N-1)^d floats, must not alias. LGP_E_UNSUPPORTED for a factor without an
 * FP32 copy (store = LGP_F64) or from lgp_factor_const. */
lgp_status lgp_ilu_forward_f32(lgp_factor m, const float* r, float* y, void* stream);
lgp_status lgp_ilu_backward_f32(lgp_factor m, const float* y, float* z, void* stream);

/* Layout of a factor, for inspection. offsets (host, 3*noff ints, filled by
 * the library and valid while the handle lives) lists NZ(M) as (dx,dy,dz) in
 * column order; the first n_lower are the strictly lower ones. L (device)
 * is row-major with row stride ld >= n_lower + 1 (a multiple of 32, so rows
 * start on 256-byte boundaries): L[i*ld + k] = L(i, i + offset_k) for
 * k < n_lower, zero where the column leaves the grid, L[i*ld + n_lower]
 * = 1/U(i,i), and zero after that. D (device, n) holds the pivots U(i,i). */
typedef struct {
    int d, N, n1, Ta, Tb;    /* Ta: the largest per-direction truncation, clamped to N */
    int64_t n;
    int noff, n_lower;
    const int* offsets;
    const double* L;
    const double* D;
    int levels;          /* hyperplane depth of the sweeps */
    int ld;              /* row stride of L in doubles */
    double factor_kernel_ms; /* duration of the ILU(0) kernel of this factorisation,
                                from HIP events on the caller's stream (-1 if unknown) */
    int factor_kernel;   /* which ILU(0) kernel built it: 2 = dataflow kernel (one row per
                            wavefront, pair tables in LDS), 1 = generic level-ordered kernel
                            (for d = 1: the single-wavefront band factorisation),
                            3 = chunked kernel of d = 3 (a workgroup per run of rows of
                            a grid line, FP64 rows in a window).
                            The environment variable LGP_FACTOR_KERNEL=1|2 restricts the
                            2D choice to that kernel where it applies (else the generic one
                            runs); unset or 0 takes 2 where it applies. */
    int layout;          /* 0: L row-major as above. 1 (d = 3): offset-major,
                            L[k*ld + i] = L(i, i + offset_k) with ld >= n; L is NULL
                            when the factor is kept in FP32 only */
    const double* invD;  /* device, n: 1/U(i,i) */
    int factor_launches; /* launches of the ILU(0) kernel in the last build (the 3D kernel runs
                            in several, one per window of z-planes); factor_kernel_ms spans
                            all of them and the small fills between them */
    int factor_waits;    /* kernel 3: steps of the last build that found a row they read not
                            yet written and read it again (0 for the other kernels) */
} lgp_factor_desc;
lgp_status lgp_factor_describe(lgp_factor m, lgp_factor_desc* out);

/* ---------------------------------------------------------------- PCG -- */
typedef struct {
    double rtol;         /* stop when ||r||_2 <= rtol ||F||_2 (Alg. 1); default 1e-10 */
    int max_iter;        /* k_max of Alg. 1; default 2000 */
    lgp_dtype inner;     /* LGP_F64: plain PCG. LGP_F32 / LGP_BF16: FP64 iterative
                            refinement around an inner PCG whose matvec runs in that
                            precision and whose sweeps use FP32 factors */
    double inner_rtol;   /* inner stop rule in mixed mode; <= 0 selects the default:
                            1e-3 for LGP_F32, 1e-1 for LGP_BF16 (a BF16 operator is
                            accurate to about 1e-2, and a tighter inner rule stalls) */
    int max_outer;       /* refinement steps in mixed mode; default 60 */
    int check_every;     /* iterations enqueued between host convergence checks; default 4 */
} lgp_solve_opts;

typedef struct {
    int iters;               /* PCG iterations (summed over inner solves in mixed mode) */
    int outer;               /* refinement steps (mixed) or restarts (FP64) */
    double relres_true;      /* ||F - K x||_2 / ||F||_2 recomputed in FP64 at exit */
    double relres_recursive; /* the recursive residual of the last PCG iteration */
    lgp_status status;
} lgp_solve_info;

/* Device bytes of the PCG workspace for problem p and inner precision. */
size_t lgp_solve_workspace_bytes(lgp_problem p, lgp_dtype inner);

/* Solve (A + B) x = F by PCG (Alg. 1) with the one-step ILU(0)
 * preconditioner. F device (N-1)^d; x device, in: initial guess, out:
 * solution. Scalars stay on the device; the host reads the convergence flag
 * every check_every iterations. After Alg. 1 stops, the true residual is
 * recomputed in FP64; if it exceeds rtol the iteration restarts from x (at
 * most 3 times). Synchronises `stream`; fills *info (host). opts may be
 * NULL for the defaults. */
lgp_status lgp_pcg_solve(lgp_problem p, lgp_factor m, const double* F, double* x,
                         const lgp_solve_opts* opts, void* ws, size_t ws_bytes,
                         void* stream, lgp_solve_info* info);

/* ----------------------------------------------------------- batches -- */
/* Many requests of one grid shape (same d and N) solved together (Alg. 1 on
 * each): every kernel of a PCG iteration covers all running requests in one
 * launch -- the two substitutions of every request in one persistent launch,
 * the vector updates and dot products with one block row per request -- and
 * the iteration is captured once as a HIP graph and replayed while the set
 * of running requests is unchanged (not on the null stream). Each request
 * computes exactly what lgp_pcg_solve computes for it (FP64 PCG with the
 * same restarts), so results equal the single-request ones bit for bit.
 * Requests join and leave between steps (continuous batching): a slot is
 * filled by lgp_batch_add, advanced by lgp_batch_step, read by
 * lgp_batch_info and freed by lgp_batch_remove. Factors of one batch must
 * share the pattern NZ(M) (same truncation and nonzero series terms);
 * lgp_batch_add returns LGP_E_UNSUPPORTED for another pattern (it then
 * needs its own batch) and LGP_E_NOMEM when every slot is taken. Only FP64
 * solves (opts->inner = LGP_F64) are batched. The workspace (device,
 * lgp_batch_workspace_bytes) is owned by the caller; problems, factors, F
 * and x must stay alive while their slot is in use. Calls on one batch are
 * ordered on its stream. */
typedef struct lgp_batch_s* lgp_batch;
size_t lgp_batch_workspace_bytes(lgp_problem shape, int slots);
lgp_status lgp_batch_create(lgp_problem shape, int slots, void* ws, size_t ws_bytes, void* stream,
                            lgp_batch* out);
/* Admit a request: ||F||, the true residual of the initial guess x (device,
 * in: x0, out: solution) and the first scalars, on the batch's stream
 * (synchronises); *slot receives its slot. A request that needs no iteration
 * (F = 0, or x0 already within rtol) or is rejected (non-finite F or x0) is
 * finished at once (see lgp_batch_info). */
lgp_status lgp_batch_add(lgp_batch b, lgp_problem p, lgp_factor m, const double* F, double* x,
                         const lgp_solve_opts* opts, int* slot);
/* `iters` PCG iterations of every running request, then the convergence
 * check of each (true FP64 residual, restart up to 3 times); synchronises.
 * *running: requests still running. */
lgp_status lgp_batch_step(lgp_batch b, int iters, int* running);
lgp_status lgp_batch_info(lgp_batch b, int slot, lgp_solve_info* info, int* finished);
lgp_status lgp_batch_remove(lgp_batch b, int slot);
void lgp_batch_destroy(lgp_batch b);
/* All of the above for `count` requests at once: p, m, F, x host arrays of
 * count handles / device pointers, info host array of count results; ws of
 * lgp_batch_workspace_bytes(p[0], count) bytes. Returns the first non-OK
 * status among the requests (each one's is in info). */
lgp_status lgp_pcg_solve_batched(int count, const lgp_problem* p, const lgp_factor* m, const double* const* F,
                                 double* const* x, const lgp_solve_opts* opts, void* ws, size_t ws_bytes,
                                 void* stream, lgp_solve_info* info);

/* ------------------------------------------- fast Legendre transforms -- */
/* The discrete Legendre transforms of Sec. 2.2 at a problem's N+1
 * Legendre-Gauss nodes, computed in O(N (log N)^2) (the approach of Hale and
 * Townsend that the paper cites: an asymptotic expansion of L_n summed with
 * FFTs where it is accurate to 1e-16, the three-term recurrence elsewhere),
 * and the product of Sec. 4.3 through them (steps 1-4: phi to Legendre
 * coefficients, BDLT, pointwise coefficients, FDLT, recombination onto the
 * test functions). The product equals lgp_matvec in FP64 up to rounding;
 * lgp_matvec keeps the dense per-direction contractions on the matrix
 * cores, which are faster at every N this library serves. Served for
 * N + 1 <= 2048 (LGP_E_UNSUPPORTED above). The handle keeps a pointer to
 * the problem, which must outlive it; its buffer (caller-owned device
 * memory of lgp_dlt_bytes bytes) holds the plan and all scratch, so
 * transforms and products on one handle must be stream-ordered. */
typedef struct lgp_dlt_s* lgp_dlt;
size_t lgp_dlt_bytes(lgp_problem p);
/* Plan on the host, tables uploaded on `stream` (synchronised). */
lgp_status lgp_dlt_create(lgp_problem p, void* buf, size_t buf_bytes, void* stream, lgp_dlt* out);
/* count (1 .. max((N+1)^(d-1), 16)) contiguous vectors of N+1 doubles, in to out
 * (device). forward = 0: BDLT, f_k = sum_n c_n L_n(x_k); forward = 1: FDLT,
 * c_n = (2n+1)/2 sum_k w_k f_k L_n(x_k). */
lgp_status lgp_dlt_lines(lgp_dlt h, int forward, int64_t count, const double* in, double* out, void* stream);
/* y = (A + B) u in FP64 through the fast transforms; u, y device (N-1)^d
 * doubles, must not alias. */
lgp_status lgp_matvec_fast(lgp_dlt h, const double* u, double* y, void* stream);
/* Number of degree blocks summed by the expansion (0: every degree direct). */
int lgp_dlt_blocks(lgp_dlt h);
void lgp_dlt_destroy(lgp_dlt h);

/* ------------------------------------------------ allocation-free solve -- */
/* For callers that cannot allocate device memory at solve time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * lgp_pcg_solve without the workspace argument. The PCG workspace is a
 * device array inside the library, one copy per GPU, of
 * lgp_pcg_solve_noalloc_max_bytes() bytes (64 MiB), held until the process
 * ends. Problems whose workspace (lgp_solve_workspace_bytes) exceeds it are
 * refused with LGP_E_NOMEM: FP64 solves up to about 2.09e6 unknowns, mixed
 * ones up to about 1.19e6. The call itself allocates nothing. Every call on
 * a GPU uses that GPU's one array: calls that overlap in time on one GPU
 * (from any stream) race and must not be issued. Arguments, errors and
 * synchronisation otherwise as lgp_pcg_solve. */
size_t lgp_pcg_solve_noalloc_max_bytes(void);
lgp_status lgp_pcg_solve_noalloc(lgp_problem p, lgp_factor m, const double* F, double* x,
                                 const lgp_solve_opts* opts, void* stream, lgp_solve_info* info);

#ifdef __cplusplus
}
#endif
#endif /* LGPCG_H */

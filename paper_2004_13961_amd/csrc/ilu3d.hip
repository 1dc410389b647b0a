// Three-dimensional preconditioner path: ILU(0) of M (Alg. 2) with the
// factor written offset-major, and the two substitutions of the one-step
// method (Alg. 3, Alg. 4) reading that layout.
//
// Storage. A[k * ldo + i] = L(i, i + delta_k) for the lower offsets delta_k
// (zero where the column leaves the grid). For a run of consecutive rows i
// the forward substitution reads A[k][i..] and the backward one, which needs
// L(i - delta_k, i) = A[k][i - delta_k], reads A[k][i - delta_k ..]: both
// are contiguous, so no transposed copy of the factor is kept. The FP64
// factor may be omitted (FP32 copy only, for the mixed-precision solve):
// the factorisation itself always runs in FP64 on a window of rows, the
// `ring`, which holds each row from its completion until the last row that
// reads it is done.
//
// Factorisation schedule. A chunk is B consecutive rows of one grid line
// (fixed iy, iz); one workgroup of B waves takes a chunk, one wave per row.
// With e = ceil(Hx / B), chunk keys kappa = xb + wy iy + wz iz,
// wy = e + 1, wz = e + wy Hy + 1, decrease along every dependency between
// different chunks (a row i + delta lies at most e chunks away in x), so
// handing out chunks in key order by an atomic ticket means a row only
// waits for rows of chunks taken earlier (resident or finished) or for the
// earlier rows of its own chunk. Consecutive rows of a chunk read largely
// the same rows of L at nearly the same time, from the same L2.
//
// Window. The window holds Z whole z-planes of rows, row (ix, iy, iz) in
// slot ((iz mod Z) n1 + iy) n1 + ix. A launch covers chunks of keys [k0, k1)
// and reads rows of keys down to k0 - reach (reach = e + wy Hy + wz Hz): the
// launches are cut so that all of those rows span at most Z planes, so no
// slot in use is overwritten; the slots a launch writes are filled with the
// sentinel before it. A window row holds L(r, r + delta) at delta's position
// p(delta) = P0 + dz XY + dy X + dx in the lower half of the stencil's
// bounding box (X = 2 Hx + 1, XY = X (2 Hy + 1), P0 = p(0); zero at holes,
// columns outside the grid and up to slot PD), and 1/D(r) at slot PD.
//
// Each row is computed left-looking (reading R1): u_j = M(i, i+d_j) -
// sum over pairs (k, l) with d_k = d_j + d_l of u_k L(i+d_j, i+d_k); then
// L(i, i+d_j) = u_j / D(i+d_j), D(i) = M(i,i) - sum_j u_j L(i, i+d_j). The
// offsets j are taken grid line by grid line, the line taken longest ago
// first and the row's own line last, x ascending within a line, so
// consecutive steps read x-neighbouring rows of the window (a quarter less
// traffic beyond the L2 than an order by hyperplane level). The row's u
// vector sits in LDS at the same box positions, so p(d_k) = p(d_l) + p(d_j)
// - P0, and a pair is named by p(d_l) alone. Pairs at adjacent positions p, p + 1 form a
// duo, which one 16-byte load gathers and one LDS read pairs with u (a pair
// without a neighbour is a duo with a flagged, zeroed second term); a duo is
// the 16-bit value 8 p | flag, two per 32-bit word. The duos of all steps
// form one list (each step padded to rows of 128 with P0, whose window slot
// is zero) cut into packets of two rows; the loads of the next packets are
// in flight while a packet is consumed. A row's entries are published
// together when it is done; a gathered sentinel sends the step to coherent
// re-reads.
//
// Substitution schedule. Blocks of BX consecutive rows of a line; a
// workgroup (256 threads: BX rows x 256/BX offset groups) sums the terms of
// every other line for its rows in parallel, then one thread solves the
// short in-line recurrence (offsets (-m, 0, 0)). Blocks are handed out in
// the key order above (B = BX); a block waits until its own line has done
// the previous block, and the lines (iy-1, iz) and (min(iy+Hy, n1-1), iz-1)
// have done the columns it needs (by induction that covers every other
// line). The backward substitution runs the same kernel on the mirrored
// grid (stream row i' = n-1-i).
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "devutil.h"

namespace lgp {

// ------------------------------------------------------------ helpers ----
struct ChunkKeys {
    int e, wy, wz, reach;
};
static ChunkKeys chunk_keys(int B, int Hx, int Hy, int Hz) {
    ChunkKeys k;
    k.e = (Hx + B - 1) / B;
    if (k.e < 1) k.e = 1;
    k.wy = k.e + 1;
    k.wz = k.e + k.wy * Hy + 1;
    k.reach = k.e + k.wy * Hy + k.wz * Hz;
    return k;
}

constexpr int kRowsPerPacket = 2;   // rows of 64 duo words in a packet of the 3D factor kernel

// The chunked kernel lays out each row's u vector (LDS) and the rows of the
// window by position in the lower half of the stencil's bounding box,
// p(delta) = P0 + dz XY + dy X + dx (X = 2 Hx + 1, XY = X (2 Hy + 1), P0 the
// diagonal), so a pair of the recurrence is named by one 16-bit byte offset:
// the neighbour row's entry p(delta_l) and u at p(delta_l) + (p(delta_j) - P0).
// This needs the box order (z, y, x) to be the order of the columns, i.e. a
// grid wider than twice the reach in x and y; other grids take the generic
// kernel. Returns the rows per chunk (0: generic kernel): a power of two up
// to 8 whose u vectors (P0 + 2 doubles each) fit 150 KB of LDS.
static int factor3_waves(const Factor& F) {
    if (F.n1 <= 2 * std::max(F.Hx, F.Hy) || F.bPD + 1 > 8191) return 0;
    const size_t per = (size_t)(F.bP0 + 2) * 8;
    const int fit = (int)((150u * 1024u) / per);
    int B = 8;   // a power of two (slot arithmetic by shifts)
    while (B > fit) B >>= 1;
    return B;
}

// FP64 window of the chunked kernel: Z whole z-planes of rows, row
// (ix, iy, iz) in slot ((iz mod Z) n1 + iy) n1 + ix; at most 64 GiB, never
// more than the grid; LGP_RING_PLANES lowers it (tests of the windowed path)
static int ring_planes_for(const Factor& F, int64_t ldl) {
    const int64_t plane = (int64_t)F.n1 * F.n1 * ldl * 8;
    int64_t Z = (int64_t)(64ull << 30) / plane;
    if (Z > F.n1) Z = F.n1;
    if (const char* e = std::getenv("LGP_RING_PLANES")) {
        const long long v = std::atoll(e);
        if (v > 0 && v < Z) Z = v;
    }
    return (int)Z;
}

size_t plan_factor3(Factor& F, void* buf, int store) {
    Carver c(buf);
    const int64_t n = F.n;
    const int nlo = F.nlo, T = F.T, h = F.h, n1 = F.n1;
    const int T1 = T + 1, W = 2 * h + 1;
    const int64_t tp = (int64_t)T1 * T1 * T1;
    F.layout = 1;
    F.ldl = ((nlo + 1) + 31) & ~31;
    F.ldo = (n + 63) & ~(int64_t)63;
    F.has64 = (store != STORE_F32_ONLY);
    F.has32 = (store != STORE_F64);
    F.bX = 2 * F.Hx + 1;
    F.bXY = F.bX * (2 * F.Hy + 1);
    F.bP0 = F.Hz * F.bXY + F.Hy * F.bX + F.Hx;
    F.bPD = F.Hz * F.bXY + (F.Hy + 1) * F.bX;
    F.ldr = ((F.bPD + 1) + 15) & ~15;
    F.fB = factor3_waves(F);
    F.nxb = F.fB > 0 ? (n1 + F.fB - 1) / F.fB : 0;
    F.nchunks = F.nxb * F.nlines;
    // the generic kernel needs every row at once: the window is the grid
    const int64_t rowlen = F.fB > 0 ? F.ldr : F.ldl;   // window row: box positions, or row-major
    F.ring_planes = F.fB > 0 ? ring_planes_for(F, rowlen) : n1;
    F.ring_rows = (int64_t)F.ring_planes * n1 * n1;
    F.sBX = 8;
    F.snxb = (n1 + F.sBX - 1) / F.sBX;
    F.L = F.Ut = nullptr;
    F.L32 = F.Ut32 = nullptr;
    F.A64 = F.has64 ? c.take<double>((size_t)nlo * F.ldo) : nullptr;
    F.A32 = F.has32 ? c.take<float>((size_t)nlo * F.ldo) : nullptr;
    F.ring = c.take<double>((size_t)(F.ring_rows + 1) * rowlen);
    F.Dg = c.take<double>(n);
    F.invD = c.take<double>(n);
    F.invD32 = F.has32 ? c.take<float>(n) : nullptr;
    F.d_offs = c.take<int>((size_t)4 * (nlo + 1));
    F.prog = c.take<unsigned>((size_t)F.nlines);
    F.ticket = c.take<unsigned>(4);
    F.flag = c.take<int>(4);
    F.coefA = c.take<double>((size_t)3 * tp);
    F.coefB = c.take<double>(tp);
    F.band = c.take<double>((size_t)2 * T1 * n1 * W);
    F.fold3 = c.take<double>((size_t)F.nlines * W * W * 2 * T1);
    F.steps = c.take<int>((size_t)4 * (nlo + 1));
    F.sdxyz = c.take<int>(nlo + 1);
    F.pairw = c.take<unsigned>((size_t)F.npairs + 64 * 8);
    // duo words of the chunked kernel: two 16-bit duos per word, each step
    // padded to rows of 64 words, then one packet of zero words
    F.pw16 = c.take<unsigned>(F.fB > 0 ? ((size_t)F.npairs + 128 * (size_t)(nlo + 1)) / 2 + 64 * kRowsPerPacket : 1);
    F.kofp = c.take<int>(F.fB > 0 ? (size_t)F.bP0 : 1);
    // packets: fewer than one per 128 pairs of each step, plus one per step
    F.pk = c.take<int>((size_t)4 * ((size_t)F.npairs / 128 + 2 * (size_t)nlo + 2));
    F.chunk_order = c.take<int>(F.nchunks > 0 ? F.nchunks : 1);
    F.blk_order = c.take<int>((size_t)F.nlines * F.snxb);
    F.own = c.take<int>(16);
    // generic-kernel fallback: level order of the rows and per-row done flags
    {
        const int64_t A1 = F.Hx + 1, B1 = (int64_t)(F.Hx + 1) * (F.Hy + 1);
        F.maxlev = (int)((n1 - 1) * (1 + A1 + B1) + 1);
    }
    F.lev = c.take<int>((size_t)2 * F.maxlev + 2);
    F.line_order = c.take<int>(F.fB > 0 ? 1 : n);   // row order of the generic kernel
    F.pair_ptr = c.take<int>((size_t)2 * (nlo + 1));   // pair ranges per offset (chunked) / CSR (generic)
    F.pair_j = c.take<int>(F.fB > 0 ? 1 : std::max(F.npairs, 1));
    F.pair_l = c.take<int>(F.fB > 0 ? 1 : std::max(F.npairs, 1));
    F.y_tmp = c.take<double>(n);   // precond_apply intermediate; generic kernel: done flags
    F.runs = nullptr;
    F.bytes = c.off + 256;
    return F.bytes;
}

// ---------------------------------------------------------- kernels ------
__global__ void reset3_kernel(unsigned* p, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// sentinel into the window slots of the rows of chunks order[t0 .. t1)
__global__ void fill_chunk_rows_kernel(double* __restrict__ ring, const int* __restrict__ order, int t0, int t1,
                                       int B, int nxb, int n1, int Z, int ldl, double v) {
    const int64_t per = (int64_t)B * ldl;
    const int64_t total = (int64_t)(t1 - t0) * per;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int ch = order[t0 + (int)(e / per)];
        const int rem = (int)(e % per);
        const int b = rem / ldl, col = rem - b * ldl;
        const int line = ch / nxb;
        const int ix = (ch - line * nxb) * B + b;
        if (ix >= n1) continue;
        const int iz = line / n1, iy = line - iz * n1;
        ring[(((int64_t)(iz % Z) * n1 + iy) * n1 + ix) * ldl + col] = v;
    }
}

__global__ void fill_rows_kernel(double* __restrict__ ring, int64_t first, int64_t rows, int ldl, double v) {
    const int64_t total = rows * ldl;
    double* p = ring + first * ldl;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

struct F3Args {
    int n1, nlo, ldl, T, h, lgB, nxb, npk;
    int X, XY, P0, PD;       // box positions: x extent, plane size, diagonal, 1/D slot (ldl: window row length)
    int64_t n, ring_rows, ldo;
    int ring_planes;
    int tk_begin, tk_end;
    const int4* pk;          // packets {first word, rows, packed (dx,dy,dz), j | first << 30 | last << 31}
    const int2* jrange;      // [nlo] word range of the step of offset j
    const int4* offs;        // [nlo + 1] (dx, dy, dz, linear) in column order
    const unsigned* pairw;   // duo words: two duos (byte offset 8 p | one-pair flag), low half first
    const int* kofp;         // [P0] lower offset index at each box position, or -1
    const int* chunk_order;
    const double* band;
    const double* fold;
    double* ring;
    double* A64;
    float* A32;
    double* Dg;
    double* invD;
    float* invD32;
    unsigned* ticket;
    int* flag;
};

// ring row of row (rx, line rl = ry + n1 rz): ((rz mod Z) n1 + ry) n1 + rx
__device__ inline int64_t ring_slot(const F3Args& a, int rl, int rx) {
    const int rz = rl / a.n1, ry = rl - rz * a.n1;
    return ((int64_t)(rz % a.ring_planes) * a.n1 + ry) * a.n1 + rx;
}

// two adjacent doubles, at 8-byte alignment (one 16-byte load)
typedef double dbl2u __attribute__((ext_vector_type(2), aligned(8)));

// QW rows of 64 duo words per packet (4 QW duos, up to 8 QW pairs, per
// lane), PP packets in flight, the gathers of PG of them
template <int QW, int PP, int PG>
__global__ __launch_bounds__(512) void ilu3d_factor_kernel(F3Args a) {
    extern __shared__ double smem3[];
    __shared__ int s_chunk, s_rank;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n1 = a.n1, nlo = a.nlo, h = a.h;
    const int W = 2 * h + 1, T1 = a.T + 1, bandT = n1 * W;
    const int B = 1 << a.lgB;
    const int X = a.X, XY = a.XY, P0 = a.P0, PD = a.PD;
    double* u = smem3 + (size_t)wv * (P0 + 2);   // box positions 0 .. P0, then a zero slot
    const char* ub = (const char*)u;
    const int64_t zbase = a.ring_rows * (int64_t)a.ldl;   // the zero row
    // duos past a packet's end: the neighbour row's diagonal slot, which the
    // row publishes as zero together with its entries, second element absent
    const unsigned padh = (unsigned)P0 * 8u | 1u;
    const unsigned padw = padh | (padh << 16);
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            const unsigned tk = atomicAdd(a.ticket, 1u);
            const int t = a.tk_begin + (int)tk;
            s_chunk = (t < a.tk_end) ? a.chunk_order[t] : -1;
            s_rank = t;
        }
        __syncthreads();
        const int chunk = s_chunk;
        if (chunk < 0) break;
        const int line = chunk / a.nxb;
        const int ix = (chunk - line * a.nxb) * B + wv;
        if (ix >= n1) continue;   // wave-uniform
        const int iy = line % n1, iz = line / n1;
        const int64_t i = (int64_t)line * n1 + ix;
        const int64_t myslot = ring_slot(a, line, ix);

        // u: zero, then M(i, i + delta_k) for the lower offsets and the
        // diagonal (Kronecker form of Sec. 4.2 over the folded line
        // coefficients) at their box positions; zero where the column leaves
        // the grid
        for (int p = lane; p <= P0 + 1; p += 64) u[p] = 0.0;
        for (int k = lane; k <= nlo; k += 64) {
            const int4 o = a.offs[k];
            if ((unsigned)(ix + o.x) < (unsigned)n1 && (unsigned)(iy + o.y) < (unsigned)n1 &&
                (unsigned)(iz + o.z) < (unsigned)n1) {
                const double* pS = a.band + ix * W + (o.x + h);
                const double* pF = a.fold + ((int64_t)line * W * W + (int64_t)(o.z + h) * W + (o.y + h)) * 2 * T1;
                double v = 0.0;
                for (int t = 0; t < T1; ++t) v += pS[t * bandT] * pF[t] + pS[(T1 + t) * bandT] * pF[T1 + t];
                u[P0 + o.z * XY + o.y * X + o.x] = v;
            }
        }

        dbl2u g[PP][2 * QW];
        unsigned pw[PP][QW];
        int jj[PP], lastp[PP], us[PP];
        int64_t rb[PP];
        int64_t cur = zbase;   // ring row offset of the step being issued
        int cur_s = 0;         // its shift p(delta_j) - P0, in bytes
        // Packet descriptors: lane t of `win` holds packet w0 + t and is read
        // with readlane (no scalar load in the loop); `nxt` collects packets
        // w0 + 64 .. w0 + 127, one lane per issued packet, from a load made
        // PP packets earlier (pkn). Every packet issues the same loads (past
        // the end: a dead packet), so the wait before a use counts exactly
        // the loads issued after it and never drains the pipeline.
        const int lastpk = a.npk - 1;
        int4 win = a.pk[min(lane, lastpk)];
        int4 nxt = make_int4(0, 0, 0, 0);
        int4 pkn[PP];
#pragma unroll
        for (int b = 0; b < PP; ++b) pkn[b] = a.pk[min(64 + b, lastpk)];
        int w0 = 0;
        auto desc = [&](int b, int p) {
            if (p >= w0 + 64) {   // wave-uniform: next window (already loaded)
                w0 += 64;
                win = nxt;
            }
            const int t = p - w0;
            if (lane == t) nxt = pkn[b];   // packet p + 64
            pkn[b] = a.pk[min(p + 64 + PP, lastpk)];
            return make_int4(__builtin_amdgcn_readlane(win.x, t), __builtin_amdgcn_readlane(win.y, t),
                             __builtin_amdgcn_readlane(win.z, t), __builtin_amdgcn_readlane(win.w, t));
        };
        // Two stages per packet: A loads the descriptor's pair words and fixes
        // the step's row (PT packets ahead), B gathers the row entries the
        // pair words name (PG packets ahead), so neither stage waits on a
        // load issued in the same iteration.
        auto stage_a = [&](int b, int p) {
            const int4 Pd = desc(b, p);
            const bool live = p < a.npk;   // wave-uniform
            const int4 P = live ? Pd : make_int4(0, 0, 0, (int)(nlo + 1));
            if (!live) cur = zbase;
            if (P.w & (1 << 30)) {   // first packet of a step: its row and shift
                const int dx = (P.z & 0xFF) - 128, dy = ((P.z >> 8) & 0xFF) - 128, dz = ((P.z >> 16) & 0xFF) - 128;
                const bool valid = (unsigned)(ix + dx) < (unsigned)n1 && (unsigned)(iy + dy) < (unsigned)n1 &&
                                   (unsigned)(iz + dz) < (unsigned)n1;
                cur = valid ? ring_slot(a, line + dy + dz * n1, ix + dx) * a.ldl : zbase;
                cur_s = (dz * XY + dy * X + dx) * 8;
            }
            rb[b] = cur;
            us[b] = cur_s;
            jj[b] = P.w & 0x3FFFFFFF;
            lastp[b] = (P.w >> 31) & 1;
            // P.y: rows of 64 words (128 duos) the packet holds
#pragma unroll
            for (int q = 0; q < QW; ++q) {
                const unsigned wd0 = a.pairw[P.x + lane + 64 * q];
                pw[b][q] = (q < P.y) ? wd0 : padw;
            }
        };
        // one 16-byte load per duo: the entries at its position and the next
        auto stage_b = [&](int b) {
            const char* rowp = (const char*)(a.ring + rb[b]);
#pragma unroll
            for (int q = 0; q < QW; ++q) {
                g[b][2 * q] = *(const dbl2u*)(rowp + (pw[b][q] & 0xFFFEu));
                g[b][2 * q + 1] = *(const dbl2u*)(rowp + ((pw[b][q] >> 16) & 0xFFFEu));
            }
        };
        // a duo's two terms: u at the position (shifted by p(delta_j) - P0)
        // and the next one, times the gathered pair; the second term is zero
        // when the duo holds one pair (flag bit 0)
        auto duo = [&](double s, const char* us_b, unsigned d, double gx, double gy) {
            const char* up = us_b + (d & 0xFFFEu);
            s = __builtin_fma(*(const double*)up, gx, s);
            return __builtin_fma(*(const double*)(up + 8), (d & 1u) ? 0.0 : gy, s);
        };
        // the whole step again with coherent loads, until none of its values
        // is the sentinel (a computed NaN ends the wait as well)
        auto slow_step = [&](int j, int64_t base, int sh) {
            const int2 R = a.jrange[j];
            for (;;) {
                bool pend = false;
                double sum = 0.0;
                for (int e0 = R.x; e0 < R.y || e0 == R.x; e0 += 64) {
                    const int e = e0 + lane;
                    const unsigned wd = (e < R.y) ? a.pairw[e] : padw;
                    const char* rowp = (const char*)(a.ring + base);
#pragma unroll
                    for (int hf = 0; hf < 2; ++hf) {
                        const unsigned d = hf ? wd >> 16 : wd & 0xFFFFu;
                        const double* gp = (const double*)(rowp + (d & 0xFFFEu));
                        const double gx = ld_coh(gp), gy = ld_coh(gp + 1);
                        pend |= Sentinel<double>::is(gx) || (!(d & 1u) && Sentinel<double>::is(gy));
                        // the same operations in the same order as the packets
                        // below, so a step gives the same bits on either path
                        sum = duo(sum, ub + sh, d, gx, gy);
                    }
                }
                if (!__any(pend)) return wave_total_bcast(sum);
                __builtin_amdgcn_s_sleep(2);
            }
        };
        double acc = 0.0;
        int nslow = 0;
        auto consume = [&](int b) {
            const char* us_b = ub + us[b];   // u shifted by p(delta_j) - P0
#pragma unroll
            for (int q = 0; q < QW; ++q) {
                acc = duo(acc, us_b, pw[b][q] & 0xFFFFu, g[b][2 * q].x, g[b][2 * q].y);
                acc = duo(acc, us_b, pw[b][q] >> 16, g[b][2 * q + 1].x, g[b][2 * q + 1].y);
            }
            if (lastp[b]) {   // wave-uniform
                double tot = wave_total_bcast(acc);
                acc = 0.0;
                if (__builtin_expect(isnan(tot), 0)) {
                    tot = slow_step(jj[b], rb[b], us[b]);
                    ++nslow;
                }
                const int jpos = P0 + us[b] / 8;
                const double mj = u[jpos];
                if (lane == 0) u[jpos] = mj - tot;
            }
        };
#pragma unroll
        for (int b = 0; b < PP; ++b) stage_a(b, b);
#pragma unroll
        for (int b = 0; b < PG; ++b) stage_b(b);
        for (int p0 = 0; p0 < a.npk; p0 += PP) {
#pragma unroll
            for (int b = 0; b < PP; ++b) {
                consume(b);                    // packet p0 + b (dead past the end: adds zeros)
                stage_b((b + PG) % PP);        // packet p0 + b + PG
                stage_a(b, p0 + b + PP);
            }
        }

        // L(i, i + delta) = u(p) / D(i + delta), D(i) = M(i, i) - sum_p u(p) L(i, i + delta);
        // the 1/D of FB positions per lane are loaded together, then checked
        constexpr int FB = 8;
        double piv = 0.0;
        for (int pb = 0; pb < P0; pb += 64 * FB) {
            double dv[FB];
            const double* pd[FB];
#pragma unroll
            for (int r = 0; r < FB; ++r) {
                const int p = pb + lane + 64 * r;
                pd[r] = nullptr;
                dv[r] = 0.0;
                if (p < P0) {
                    const int k = a.kofp[p];
                    if (k >= 0 && u[p] != 0.0) {
                        const int4 o = a.offs[k];
                        if ((unsigned)(ix + o.x) < (unsigned)n1 && (unsigned)(iy + o.y) < (unsigned)n1 &&
                            (unsigned)(iz + o.z) < (unsigned)n1)
                            pd[r] = a.ring + ring_slot(a, line + o.y + o.z * n1, ix + o.x) * a.ldl + PD;
                    }
                }
                if (pd[r]) dv[r] = __hip_atomic_load(pd[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
#pragma unroll
            for (int r = 0; r < FB; ++r) {
                const int p = pb + lane + 64 * r;
                if (p < P0) {
                    if (pd[r]) {
                        while (Sentinel<double>::is(dv[r])) {
                            __builtin_amdgcn_s_sleep(2);
                            dv[r] = ld_coh(pd[r]);
                        }
                    }
                    const double uv = u[p];
                    const double lk = pd[r] ? uv * dv[r] : 0.0;
                    piv += uv * lk;
                    u[p] = lk;
                }
            }
        }
        piv = wave_total_bcast(piv);
        const double Dr = u[P0] - piv;
        const double Dii = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(Dr)),
                                            __builtin_amdgcn_readfirstlane(__double2loint(Dr)));
        if (!(Dii > 0.0) || !isfinite(Dii)) {
            if (lane == 0) atomicOr(a.flag, 1);
        }
        const double iv = 1.0 / Dii;
        // the row at its box positions (zero at holes, columns outside the
        // grid and the slots up to 1/D), then 1/D
        double* rowp = a.ring + myslot * a.ldl;
        for (int p = lane; p < PD; p += 64) st_coh(rowp + p, p < P0 ? Sentinel<double>::clean(u[p]) : 0.0);
        for (int p = lane; p < P0; p += 64) {
            const int k = a.kofp[p];
            if (k >= 0) {
                if (a.A64) a.A64[(int64_t)k * a.ldo + i] = u[p];
                if (a.A32) a.A32[(int64_t)k * a.ldo + i] = (float)u[p];
            }
        }
        if (lane == 0 && nslow) atomicAdd(a.flag + 2, nslow);
        if (lane == 0) {
            st_coh(rowp + PD, Sentinel<double>::clean(iv));
            a.Dg[i] = Dii;
            a.invD[i] = iv;
            if (a.invD32) a.invD32[i] = (float)iv;
        }
    }
}

// generic-kernel output (row-major FP64 rows in the ring, 1/D at n_lower)
// into the offset-major arrays
__global__ void rows_to_offset_major_kernel(int64_t n, int nlo, int ldl, int64_t ldo, const double* __restrict__ R,
                                            double* __restrict__ A64, float* __restrict__ A32,
                                            float* __restrict__ invD32) {
    __shared__ double tile[32][33];
    const int64_t i0 = (int64_t)blockIdx.x * 32;
    const int k0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = i0 + r;
        const int k = k0 + tx;
        tile[r][tx] = (i < n && k < nlo) ? R[i * ldl + k] : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int k = k0 + r;
        const int64_t i = i0 + tx;
        if (k < nlo && i < n) {
            const double v = tile[tx][r];
            if (A64) A64[(int64_t)k * ldo + i] = v;
            if (A32) A32[(int64_t)k * ldo + i] = (float)v;
        }
    }
    if (blockIdx.y == 0 && invD32)
        for (int r = threadIdx.x; r < 32; r += blockDim.x)
            if (i0 + r < n) invD32[i0 + r] = (float)R[(i0 + r) * ldl + nlo];
}

// ------------------------------------------------------- substitutions ---
template <typename T>
struct S3Args {
    int n1, nlo, nother, Hx, Hy, BX, nxb, nblk;
    int offs_in_lds;
    int64_t n, ldo;
    const int4* offs;
    const int* own;        // [16] index of offset (-m, 0, 0), m = 1..16, or -1
    const int* blk_order;
    const T* A;
    const T* scale;        // 1/D for the backward substitution, else null
    const T* in;
    T* out;
    unsigned* prog;
    unsigned* ticket;
    const int* stop;
    const SweepSlot<T>* slots;   // batched: per-request operator, vectors, progress and flag
    int nslots;
};

// out[i'] = in[i'] * scale - sum_k L-term * out[i' + delta_k] in stream
// coordinates (REV: the mirrored grid, i = n-1-i'); the L-term is
// A[k][i] (forward) or A[k][i - delta_k] = A[k][mem(i' + delta_k)] (backward).
// NT threads: BXM rows x NG offset groups; the offset table sits in LDS.
template <typename T, bool REV, int NT>
__global__ __launch_bounds__(NT) void sweep3d_kernel(S3Args<T> a) {
    constexpr int BXM = 8;                    // rows per block (a.BX == 8)
    constexpr int NG = NT / BXM;              // offset groups
    constexpr int MO = 16;                    // in-line offsets (-m, 0, 0), m <= MO
    constexpr int U = 8;                      // terms in flight per thread
    extern __shared__ int4 s_offs_lds[];      // [nother] when it fits LDS
    __shared__ T s_part[NG][BXM];
    __shared__ T s_acc[BXM];
    __shared__ T s_coef[BXM][MO];
    __shared__ T s_prev[MO + BXM];
    __shared__ T s_rhs[BXM];
    __shared__ int s_blk;
    const int tid = threadIdx.x;
    const int r = tid % BXM, grp = tid / BXM;
    const int n1 = a.n1;
    const int64_t n = a.n;
    if (!a.slots && a.stop && *a.stop) return;
    const int ns = a.slots ? a.nslots : 1;
    const int4* s_offs = a.offs_in_lds ? s_offs_lds : a.offs;
    if (a.offs_in_lds)
        for (int k = tid; k < a.nother; k += NT) s_offs_lds[k] = a.offs[k];
    auto mem = [&](int64_t ip) -> int64_t { return REV ? (n - 1 - ip) : ip; };
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            // batched: ticket t is block t / ns (in dependency order) of slot t % ns
            const unsigned tk = atomicAdd(a.ticket, 1u);
            s_blk = (tk < (unsigned)(a.nblk * ns)) ? (int)tk : -1;
        }
        __syncthreads();
        const int bt = s_blk;
        if (bt < 0) break;
        const int blk = a.blk_order[bt / ns];
        const T* A = a.A;
        const T* scale = a.scale;
        const T* in = a.in;
        T* out = a.out;
        unsigned* prog = a.prog;
        if (a.slots) {
            const SweepSlot<T> sl = a.slots[bt % ns];
            if (sl.stop && *sl.stop) continue;   // converged request: skipped (the loop head syncs)
            A = sl.A;
            scale = sl.scale;
            in = sl.in;
            out = sl.out;
            prog = sl.prog;
        }
        const int line = blk / a.nxb;
        const int x0 = (blk - line * a.nxb) * BXM;
        const int iy = line % n1, iz = line / n1;
        // in-line coefficients and the right-hand side: independent of the
        // wait below, so their loads go out first
        if (tid < BXM * MO) {
            const int rr = tid / MO, m = tid % MO;   // coefficient of (-(m+1), 0, 0) for row rr
            const int k = a.own[m];
            const int xx = x0 + rr;
            T c = T(0);
            if (k >= 0 && xx < n1 && xx - (m + 1) >= 0) {
                const int64_t ipr = (int64_t)line * n1 + xx;
                c = A[(int64_t)k * a.ldo + (REV ? mem(ipr - (m + 1)) : mem(ipr))];
            }
            s_coef[rr][m] = c;
        } else if (tid >= BXM * MO + MO && tid < BXM * MO + MO + BXM) {
            const int rr = tid - BXM * MO - MO;
            const int xx = x0 + rr;
            T v = T(0);
            if (xx < n1) {
                const int64_t mm = mem((int64_t)line * n1 + xx);
                v = in[mm];
                if (scale) v *= scale[mm];
            }
            s_rhs[rr] = v;
        }
        // wait: own line up to x0, and the two lines that cover the others
        // (the three counters read together, one round trip per poll)
        if (tid == BXM * MO + MO + BXM) {
            const unsigned needo = (unsigned)min(n1, x0 + BXM + a.Hx);
            const int l2 = iz > 0 ? (iz - 1) * n1 + min(iy + a.Hy, n1 - 1) : line;
            for (;;) {
                const unsigned v0 = x0 > 0 ? ld_coh(&prog[line]) : ~0u;
                const unsigned v1 = iy > 0 ? ld_coh(&prog[line - 1]) : ~0u;
                const unsigned v2 = iz > 0 ? ld_coh(&prog[l2]) : ~0u;
                if (v0 >= (unsigned)x0 && v1 >= needo && v2 >= needo) break;
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        const int ix = x0 + r;
        const bool rowok = ix < n1;
        const int64_t ip = (int64_t)line * n1 + (rowok ? ix : x0);
        const int64_t mip = mem(ip);
        // every value read here is final (the progress counters say so), but
        // a cached line may still hold the sentinel (a NaN): the sum is formed
        // first, and only a NaN sum is formed again with coherent re-reads.
        // Loads are unconditional (a term outside the grid reads this row's
        // own entries) and the term is selected away, so U terms are in flight.
        auto terms = [&](bool coherent) {
            T acc = T(0);
            for (int k0 = grp; k0 < a.nother; k0 += NG * U) {
                T cv[U], vv[U];
                bool okv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int k = k0 + u * NG;
                    const int4 o = s_offs[k < a.nother ? k : 0];
                    const bool ok = k < a.nother && rowok && (unsigned)(ix + o.x) < (unsigned)n1 &&
                                    (unsigned)(iy + o.y) < (unsigned)n1 && (unsigned)(iz + o.z) < (unsigned)n1;
                    okv[u] = ok;
                    const int64_t nb = ok ? mem(ip + o.w) : mip;
                    const int kk = ok ? k : 0;
                    cv[u] = A[(int64_t)kk * a.ldo + (REV ? nb : mip)];
                    vv[u] = coherent ? ld_coh(&out[nb]) : out[nb];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (coherent) {
                        const int k = k0 + u * NG;
                        while (okv[u] && Sentinel<T>::is(vv[u])) {
                            const int4 o = s_offs[k];
                            vv[u] = ld_coh(&out[mem(ip + o.w)]);
                        }
                    }
                    acc += okv[u] ? cv[u] * vv[u] : T(0);
                }
            }
            return acc;
        };
        T acc = terms(false);
        if (__builtin_expect(isnan(acc), 0)) acc = terms(true);
        s_part[grp][r] = acc;
        // the values of the preceding rows of the line (final after the wait)
        if (tid >= BXM * MO && tid < BXM * MO + MO) {
            const int m = tid - BXM * MO;       // row x0 - MO + m
            const int xx = x0 - MO + m;
            T v = T(0);
            if (xx >= 0) v = ld_coh(&out[mem((int64_t)line * n1 + xx)]);
            s_prev[m] = v;
        }
        __syncthreads();
        if (tid < BXM) {
            T sum = T(0);
#pragma unroll 8
            for (int g2 = 0; g2 < NG; ++g2) sum += s_part[g2][tid];
            s_acc[tid] = sum;
        }
        __syncthreads();
        if (tid == 0) {
            T y[MO + BXM];
#pragma unroll
            for (int m = 0; m < MO; ++m) y[m] = s_prev[m];
#pragma unroll
            for (int rr = 0; rr < BXM; ++rr) {
                T v = s_rhs[rr] - s_acc[rr];
#pragma unroll
                for (int m = 0; m < MO; ++m) v -= s_coef[rr][m] * y[MO + rr - (m + 1)];
                y[MO + rr] = v;
            }
#pragma unroll
            for (int rr = 0; rr < BXM; ++rr) s_prev[rr] = y[MO + rr];   // results (reuses the buffer)
        }
        __syncthreads();
        if (tid < BXM && x0 + tid < n1) {
            st_coh(&out[mem((int64_t)line * n1 + x0 + tid)], Sentinel<T>::clean(s_prev[tid]));
            wait_own_stores();
        }
        __syncthreads();
        if (tid == 0) publish(&prog[line], (unsigned)min(n1, x0 + BXM));
    }
}

template <typename T>
__global__ void fill_sentinel3_kernel(int64_t n, T* __restrict__ out, const int* __restrict__ stop) {
    if (stop && *stop) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = Sentinel<T>::value();
}

// ------------------------------------------------------------- host ------
static int persistent_grid3(const void* kernel, int block, size_t shmem, int64_t units) {
    int dev = 0, cus = 256, per = 1;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, block, shmem) != hipSuccess || per < 1) per = 1;
    int64_t g = (int64_t)cus * per;
    if (g > units) g = units;
    if (g < 1) g = 1;
    return (int)g;
}

// order of units (x-block xb of line (iy, iz)) by key xb + wy iy + wz iz
static void key_order(int n1, int nxb, const ChunkKeys& K, std::vector<int>& order, std::vector<int>* keys) {
    const int nlines = n1 * n1;
    const int64_t maxkey = (int64_t)(nxb - 1) + (int64_t)K.wy * (n1 - 1) + (int64_t)K.wz * (n1 - 1) + 1;
    std::vector<int> cnt(maxkey + 1, 0);
    for (int l = 0; l < nlines; ++l) {
        const int64_t base = (int64_t)K.wy * (l % n1) + (int64_t)K.wz * (l / n1);
        for (int xb = 0; xb < nxb; ++xb) cnt[base + xb + 1]++;
    }
    for (int64_t k = 0; k < maxkey; ++k) cnt[k + 1] += cnt[k];
    if (keys) keys->assign(cnt.begin(), cnt.end());   // first rank of each key
    order.assign((size_t)nlines * nxb, 0);
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    for (int l = 0; l < nlines; ++l) {
        const int64_t base = (int64_t)K.wy * (l % n1) + (int64_t)K.wz * (l / n1);
        for (int xb = 0; xb < nxb; ++xb) order[fill[base + xb]++] = l * nxb + xb;
    }
}

// Substitution tables: block order and the in-line offsets (-m, 0, 0).
static lgp_status sweep3_tables(Factor& F, hipStream_t s, std::vector<int>& blk, std::vector<int>& own) {
    const ChunkKeys K = chunk_keys(F.sBX, F.Hx, F.Hy, F.Hz);
    key_order(F.n1, F.snxb, K, blk, nullptr);
    own.assign(16, -1);
    for (int k = 0; k < F.nlo; ++k) {
        const int* o = &F.offs[3 * k];
        if (o[1] == 0 && o[2] == 0 && o[0] < 0 && o[0] >= -16) own[-o[0] - 1] = k;
    }
    // the in-line offsets are the last ones of the lower list (column order)
    int nin = 0;
    for (int k = 0; k < F.nlo; ++k)
        if (F.offs[3 * k + 1] == 0 && F.offs[3 * k + 2] == 0) ++nin;
    for (int k = F.nlo - nin; k < F.nlo; ++k)
        if (F.offs[3 * k + 1] != 0 || F.offs[3 * k + 2] != 0 || F.offs[3 * k] < -16) return LGP_E_UNSUPPORTED;
    LGP_HIP(hipMemcpyAsync(F.blk_order, blk.data(), blk.size() * 4, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(F.own, own.data(), own.size() * 4, hipMemcpyHostToDevice, s));
    return LGP_OK;
}

// ILU(0) of the 3D stencil with the chunked kernel. Preconditions: band
// tables and folded coefficients computed, offsets, steps (dataflow order)
// and pair words uploaded (pairw followed by 64 zero words). Synchronises
// the stream before returning (the host tables go out of scope).
lgp_status factor3_run(Factor& F, hipStream_t s, const std::vector<int>& st4, const std::vector<unsigned>& pw,
                       hipEvent_t* ev) {
    const int n1 = F.n1, nlo = F.nlo, B = F.fB;
    if (B <= 0) return LGP_E_UNSUPPORTED;
    const int nsteps = nlo;
    constexpr int QW = kRowsPerPacket;
    const int X = F.bX, XY = F.bXY, P0 = F.bP0;
    // box position of every lower offset
    std::vector<int> kofp(P0, -1), posk(nlo);
    for (int k = 0; k < nlo; ++k) {
        const int* o = &F.offs[3 * k];
        const int p = P0 + o[2] * XY + o[1] * X + o[0];
        if (p < 0 || p >= P0 || kofp[p] >= 0) return LGP_E_UNSUPPORTED;
        kofp[p] = k;
        posk[k] = p;
    }
    // Step order: grid lines of the offsets from the one taken longest ago
    // (largest key lag -(wy dy + wz dz)) to the row's own line, x ascending
    // within a line. A pair's u_k lies on a line of larger lag, or on the
    // same line at smaller dx, so this is an order of the dependencies
    // (checked below); consecutive steps read x-neighbouring rows, which the
    // chunk's next row reads one step earlier, so more of a row's gathers
    // find the L2 lines its neighbour brought in.
    const ChunkKeys K = chunk_keys(B, F.Hx, F.Hy, F.Hz);
    std::vector<int> ord(nsteps), rank(nlo, -1);
    for (int st = 0; st < nsteps; ++st) ord[st] = st;
    auto lag = [&](int st) {
        const int* o = &F.offs[3 * st4[4 * st]];
        return -(K.wy * o[1] + K.wz * o[2]);
    };
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
        const int lx = lag(x), ly = lag(y);
        return lx != ly ? lx > ly : F.offs[3 * st4[4 * x]] < F.offs[3 * st4[4 * y]];
    });
    for (int st = 0; st < nsteps; ++st) rank[st4[4 * ord[st]]] = st;
    for (int st = 0; st < nsteps; ++st)
        for (int e = st4[4 * ord[st] + 2]; e < st4[4 * ord[st] + 3]; ++e)
            if (rank[(pw[e] & 0xFFFFu) / 8u] >= st) return LGP_E_ARG;   // u_k would not be ready
    // Duo words. The pairs of a step (u_k L(i+delta_j, i+delta_k), delta_k =
    // delta_j + delta_l) are cut into duos: two pairs at adjacent positions
    // p(delta_l) = p and p + 1, or one pair alone (flag bit 0 set); a duo is
    // the 16-bit byte offset 8 p | flag, and one 16-byte load gathers it.
    // Word t of a row of 64 holds duos t and 64 + t of the row's 128, so
    // each of a row's two gathers reads 64 consecutive duos. Each step is
    // padded to whole rows with the diagonal position (flagged). Packets of
    // up to QW rows, step by step in that order:
    // {first word, rows, packed (dx, dy, dz), j | first << 30 | last << 31}
    const unsigned padh = (unsigned)P0 * 8u | 1u;
    std::vector<unsigned> words, duos;
    words.reserve(pw.size() / 2 + 64 * (size_t)nsteps + 64 * QW);
    std::vector<int> pk, jr(2 * (size_t)(nlo + 1), 0);
    for (int sti = 0; sti < nsteps; ++sti) {
        const int st = ord[sti];
        const int j = st4[4 * st], p0 = st4[4 * st + 2], p1 = st4[4 * st + 3];
        const int* o = &F.offs[3 * j];
        const int packed = (o[0] + 128) | ((o[1] + 128) << 8) | ((o[2] + 128) << 16);
        duos.clear();
        for (int e = p0; e < p1;) {
            const unsigned pa = (unsigned)posk[(pw[e] >> 16) / 8u];
            const bool two = e + 1 < p1 && (unsigned)posk[(pw[e + 1] >> 16) / 8u] == pa + 1;
            duos.push_back(pa * 8u | (two ? 0u : 1u));
            e += two ? 2 : 1;
        }
        const int nd = (int)duos.size();
        const int rows = std::max(1, (nd + 127) / 128);
        const int w0 = (int)words.size();
        auto db = [&](int e) { return e < nd ? duos[e] : padh; };
        for (int m = 0; m < rows; ++m)
            for (int t = 0; t < 64; ++t) words.push_back(db(128 * m + t) | (db(128 * m + 64 + t) << 16));
        const int npk = (rows + QW - 1) / QW;
        for (int q = 0; q < npk; ++q) {
            const unsigned fl = (unsigned)j | (q == 0 ? 1u << 30 : 0u) | (q == npk - 1 ? 1u << 31 : 0u);
            pk.insert(pk.end(), {w0 + 64 * QW * q, std::min(QW, rows - QW * q), packed, (int)fl});
        }
        jr[2 * j] = w0;
        jr[2 * j + 1] = w0 + 64 * rows;
    }
    words.insert(words.end(), 64 * QW, 0u);   // the rows a last packet loads past its step
    F.npk = (int)pk.size() / 4;
    if ((size_t)F.npk > (size_t)F.npairs / 128 + 2 * (size_t)nlo + 2) return LGP_E_ARG;   // planner disagrees
    if (words.size() > ((size_t)F.npairs + 128 * (size_t)(nlo + 1)) / 2 + 64 * kRowsPerPacket) return LGP_E_ARG;
    LGP_HIP(hipMemcpyAsync(F.pw16, words.data(), words.size() * 4, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(F.kofp, kofp.data(), kofp.size() * 4, hipMemcpyHostToDevice, s));
    // chunk order and ranks
    std::vector<int> order, keystart;
    key_order(n1, F.nxb, K, order, &keystart);
    std::vector<int> blk, own;
    lgp_status st0 = sweep3_tables(F, s, blk, own);
    if (st0 != LGP_OK) return st0;
    LGP_HIP(hipMemcpyAsync(F.pk, pk.data(), pk.size() * 4, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(F.chunk_order, order.data(), order.size() * 4, hipMemcpyHostToDevice, s));
    LGP_HIP(hipMemcpyAsync(F.pair_ptr, jr.data(), jr.size() * 4, hipMemcpyHostToDevice, s));
    // launches: keys [k0, k1) such that the rows of keys [k0 - reach, k1)
    // (all a launch writes or reads) span at most Z z-planes, so no two of
    // them share a window slot
    const int nkeys = (int)keystart.size() - 1;
    const int Z = F.ring_planes;
    std::vector<int> zlo(nkeys, INT32_MAX), zhi(nkeys, -1);
    for (int k = 0; k < nkeys; ++k)
        for (int t = keystart[k]; t < keystart[k + 1]; ++t) {
            const int iz = (order[t] / F.nxb) / n1;
            zlo[k] = std::min(zlo[k], iz);
            zhi[k] = std::max(zhi[k], iz);
        }
    auto span = [&](int klo, int khi) {   // z-planes of the rows of keys [klo, khi)
        int lo = INT32_MAX, hi = -1;
        for (int k = klo; k < khi; ++k) {
            lo = std::min(lo, zlo[k]);
            hi = std::max(hi, zhi[k]);
        }
        return hi < lo ? 0 : hi - lo + 1;
    };
    std::vector<std::pair<int, int>> launches;
    for (int k0 = 0; k0 < nkeys;) {
        const int lo = std::max(0, k0 - K.reach);
        int k1 = k0 + 1;
        if (span(lo, k1) > Z) return LGP_E_UNSUPPORTED;   // window smaller than the reach
        while (k1 < nkeys && span(lo, k1 + 1) <= Z) ++k1;
        launches.push_back({keystart[k0], keystart[k1]});
        k0 = k1;
    }
    // zero row, then per launch: sentinel into its slots, reset the ticket, run
    const int64_t R = F.ring_rows;
    hipLaunchKernelGGL(fill_rows_kernel, dim3(64), dim3(256), 0, s, F.ring, R, (int64_t)1, F.ldr, 0.0);
    LGP_HIP(hipMemsetAsync(F.flag, 0, 16, s));
    F3Args a;
    a.n1 = n1;
    a.nlo = nlo;
    a.ldl = F.ldr;   // window row length
    a.X = X;
    a.XY = XY;
    a.P0 = P0;
    a.PD = F.bPD;
    a.kofp = F.kofp;
    a.T = F.T;
    a.h = F.h;
    a.lgB = 0;
    while ((1 << a.lgB) < B) ++a.lgB;
    a.nxb = F.nxb;
    a.npk = F.npk;
    a.n = F.n;
    a.ring_rows = R;
    a.ring_planes = Z;
    a.ldo = F.ldo;
    a.pk = (const int4*)F.pk;
    a.jrange = (const int2*)F.pair_ptr;
    a.offs = (const int4*)F.d_offs;
    a.pairw = F.pw16;
    a.chunk_order = F.chunk_order;
    a.band = F.band;
    a.fold = F.fold3;
    a.ring = F.ring;
    a.A64 = F.A64;
    a.A32 = F.A32;
    a.Dg = F.Dg;
    a.invD = F.invD;
    a.invD32 = F.invD32;
    a.ticket = F.ticket;
    a.flag = F.flag;
    // two rows per packet, six packets in flight, the gathers of four (of
    // the depths that fit two waves per SIMD, the fastest measured)
    auto kf = ilu3d_factor_kernel<kRowsPerPacket, 6, 4>;
    const size_t shmem = (size_t)B * (P0 + 2) * 8;
    (void)hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (ev) (void)hipEventRecord(ev[0], s);
    for (auto& L : launches) {
        double sen;
        {
            const uint64_t bits = 0x7FF40000DEADBEEFull;   // the sentinel's bit pattern
            memcpy(&sen, &bits, 8);
        }
        hipLaunchKernelGGL(fill_chunk_rows_kernel, dim3(4096), dim3(256), 0, s, F.ring, (const int*)F.chunk_order,
                           L.first, L.second, B, F.nxb, n1, Z, F.ldr, sen);
        hipLaunchKernelGGL(reset3_kernel, dim3(1), dim3(64), 0, s, F.ticket, 4);
        a.tk_begin = L.first;
        a.tk_end = L.second;
        const int grid = persistent_grid3((const void*)kf, 64 * B, shmem, L.second - L.first);
        hipLaunchKernelGGL(kf, dim3(grid), dim3(64 * B), shmem, s, a);
        LGP_CHECK_LAUNCH();
    }
    if (ev) (void)hipEventRecord(ev[1], s);
    F.factor_kernel = 3;
    F.factor_launches = (int)launches.size();
    int fl[4] = {0, 0, 0, 0};
    LGP_HIP(hipMemcpyAsync(fl, F.flag, 16, hipMemcpyDeviceToHost, s));
    LGP_HIP(hipStreamSynchronize(s));
    F.factor_waits = fl[2];
    return LGP_OK;
}

// After the generic kernel has written row-major FP64 rows into the ring
// (ring_rows = n): offset-major arrays, FP32 pivots, substitution tables.
// Synchronises the stream before returning.
lgp_status factor3_generic_finish(Factor& F, hipStream_t s) {
    std::vector<int> blk, own;
    lgp_status st0 = sweep3_tables(F, s, blk, own);
    if (st0 != LGP_OK) return st0;
    const dim3 grid((unsigned)((F.n + 31) / 32), (unsigned)((F.nlo + 31) / 32));
    hipLaunchKernelGGL(rows_to_offset_major_kernel, grid, dim3(256), 0, s, F.n, F.nlo, F.ldl, F.ldo,
                       (const double*)F.ring, F.A64, F.A32, F.invD32);
    LGP_CHECK_LAUNCH();
    LGP_HIP(hipStreamSynchronize(s));
    return LGP_OK;
}

template <typename T>
static lgp_status sweep3_t(Factor& F, bool backward, const T* A, const T* scale, const T* in, T* out,
                           hipStream_t s, const int* stop) {
    if (!A) return LGP_E_UNSUPPORTED;
    const int64_t n = F.n;
    hipLaunchKernelGGL(reset3_kernel, dim3(std::min(1024, (F.nlines + 255) / 256 + 1)), dim3(256), 0, s, F.prog,
                       F.nlines);
    hipLaunchKernelGGL(reset3_kernel, dim3(1), dim3(64), 0, s, F.ticket + 2, 1);
    hipLaunchKernelGGL(fill_sentinel3_kernel<T>, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256),
                       0, s, n, out, stop);
    int nin = 0;
    for (int k = 0; k < F.nlo; ++k)
        if (F.offs[3 * k + 1] == 0 && F.offs[3 * k + 2] == 0) ++nin;
    S3Args<T> a;
    a.n1 = F.n1;
    a.nlo = F.nlo;
    a.nother = F.nlo - nin;
    a.Hx = F.Hx;
    a.Hy = F.Hy;
    a.BX = F.sBX;
    a.nxb = F.snxb;
    a.nblk = F.nlines * F.snxb;
    a.n = n;
    a.ldo = F.ldo;
    a.offs = (const int4*)F.d_offs;
    a.own = F.own;
    a.blk_order = F.blk_order;
    a.A = A;
    a.scale = scale;
    a.in = in;
    a.out = out;
    a.prog = F.prog;
    a.ticket = F.ticket + 2;
    a.stop = stop;
    a.slots = nullptr;
    a.nslots = 0;
    constexpr int NT = 512;
    auto kf = backward ? sweep3d_kernel<T, true, NT> : sweep3d_kernel<T, false, NT>;
    size_t shmem = (size_t)std::max(1, a.nother) * sizeof(int4);
    a.offs_in_lds = shmem <= 96 * 1024;
    if (!a.offs_in_lds) shmem = 16;
    (void)hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    const int grid = persistent_grid3((const void*)kf, NT, shmem, a.nblk);
    hipLaunchKernelGGL(kf, dim3(grid), dim3(NT), shmem, s, a);
    LGP_CHECK_LAUNCH();
    return LGP_OK;
}

template <typename T>
__global__ void fill_sentinel3_slots_kernel(int64_t n, int nlines, const SweepSlot<T>* __restrict__ slots) {
    const SweepSlot<T> sl = slots[blockIdx.y];
    if (sl.stop && *sl.stop) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        sl.out[i] = Sentinel<T>::value();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nlines; i += (int64_t)gridDim.x * blockDim.x)
        sl.prog[i] = 0u;
}

lgp_status sweep3_batch(const Factor& F, int nslots, const SweepSlot<double>* slots, bool backward, unsigned* ticket,
                        hipStream_t s) {
    using T = double;
    if (!F.A64) return LGP_E_UNSUPPORTED;
    const int64_t n = F.n;
    hipLaunchKernelGGL(reset3_kernel, dim3(1), dim3(64), 0, s, ticket, 1);
    hipLaunchKernelGGL(fill_sentinel3_slots_kernel<T>,
                       dim3((unsigned)std::min<int64_t>(2048, (n + 255) / 256), nslots), dim3(256), 0, s, n,
                       F.nlines, slots);
    int nin = 0;
    for (int k = 0; k < F.nlo; ++k)
        if (F.offs[3 * k + 1] == 0 && F.offs[3 * k + 2] == 0) ++nin;
    S3Args<T> a;
    a.n1 = F.n1;
    a.nlo = F.nlo;
    a.nother = F.nlo - nin;
    a.Hx = F.Hx;
    a.Hy = F.Hy;
    a.BX = F.sBX;
    a.nxb = F.snxb;
    a.nblk = F.nlines * F.snxb;
    a.n = n;
    a.ldo = F.ldo;
    a.offs = (const int4*)F.d_offs;
    a.own = F.own;
    a.blk_order = F.blk_order;
    a.A = nullptr;
    a.scale = nullptr;
    a.in = nullptr;
    a.out = nullptr;
    a.prog = nullptr;
    a.ticket = ticket;
    a.stop = nullptr;
    a.slots = slots;
    a.nslots = nslots;
    constexpr int NT = 512;
    auto kf = backward ? sweep3d_kernel<T, true, NT> : sweep3d_kernel<T, false, NT>;
    size_t shmem = (size_t)std::max(1, a.nother) * sizeof(int4);
    a.offs_in_lds = shmem <= 96 * 1024;
    if (!a.offs_in_lds) shmem = 16;
    set_dyn_shmem((const void*)kf, shmem, s);
    const int grid = persistent_grid3((const void*)kf, NT, shmem, (int64_t)a.nblk * nslots);
    hipLaunchKernelGGL(kf, dim3(grid), dim3(NT), shmem, s, a);
    LGP_CHECK_LAUNCH();
    return LGP_OK;
}

lgp_status sweep3(Factor& F, bool backward, bool lowp, const void* in, void* out, hipStream_t s, const int* stop) {
    if (lowp) {
        if (!F.A32) return LGP_E_UNSUPPORTED;
        return sweep3_t<float>(F, backward, F.A32, backward ? F.invD32 : nullptr, (const float*)in, (float*)out, s,
                               stop);
    }
    if (!F.A64) return LGP_E_UNSUPPORTED;
    return sweep3_t<double>(F, backward, F.A64, backward ? F.invD : nullptr, (const double*)in, (double*)out, s,
                            stop);
}

}  // namespace lgp

// SVD of the small projected matrix B (N x N, FP64) of the BLWS step, whose
// singular values are the Ritz values (Algorithm 3 with Theorem 1).
//
// 1. Golub-Kahan bidiagonalisation B = Q_L Bd Q_R^T. Up to N = 224 in ONE
//    workgroup, B held in registers: a 32 x 16 thread grid, thread (tr, tc)
//    owning rows tr + 32a and columns tc + 16c. Up to N = 1024 the first
//    N - 224 steps run across ceil(N / 32) co-resident workgroups holding
//    32-column slabs, with one device-wide barrier per step, and the trailing
//    224 x 224 matrix they leave goes to the one-workgroup kernel. Each step
//    is a left and a right Householder reflection; their vectors are written
//    to global memory for the back-transformation.
// 2. Singular values of Bd by multisection with Sturm counts of B^T B - x^2 I,
//    taken by the differential stationary qd transform on the squared
//    bidiagonal entries (exact for entries perturbed in their last places):
//    one workgroup per value, 256 counts per multisection step.
// 3. Singular vectors from the Golub-Kahan tridiagonal T (size 2N, eigenvector
//    (v0, u0, v1, u1, ...), so u and v come out paired): a twisted
//    factorisation of T - sigma I for a value isolated to 1e-6 relative,
//    inverse iteration otherwise (close, repeated or zero values), in the
//    same workgroup that found the value.
// 4. Back-transformation through the stored reflectors, in blocks of 16
//    (compact WY form, matrix cores up to N = 512, one wavefront per column
//    beyond). With a second stream (the solves) and N <= 512, Q_L and Q_R
//    are formed from the identity there while steps 2 and 3 run, and the
//    back-transformation is two products with them.
#include "blws_common.h"

namespace blws {
namespace {

constexpr int GK_MAXN = 224;   // one-workgroup bidiagonalisation
constexpr int SVD_MAXN = 1024;  // cooperative bidiagonalisation and the later stages

// Start vectors of the inverse iteration: SplitMix64 (Steele, Lea & Flood
// 2014) outputs mapped to [-1, 1), distinct per value so that vectors of a
// multiple singular value start independent.
__device__ __forceinline__ double start_pm1(uint64_t counter)
{
    uint64_t z = 0x5DEECE66DULL + (counter + 1ULL) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}
// Sums across lanes, all on the VALU. Within a row of 16 lanes the partial
// sums move by DPP row rotations; across rows by the gfx950 permlane swaps:
// v_permlane16_swap on (x, x) yields (x0, x0, x2, x2) and (x1, x1, x3, x3)
// for rows x0..x3, v_permlane32_swap yields (lo, lo) and (hi, hi) for the
// two halves, so that adding the pair gives every lane the same bits.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x)
{
    const unsigned long long u = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(u & 0xffffffffu), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double join_words(unsigned lo, unsigned hi)
{
    return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}
// a + b with a from the even and b from the odd 16-lane row of each pair,
// given in every lane of both rows
__device__ __forceinline__ double rows_pair_sum(double x)
{
    const unsigned long long u = __double_as_longlong(x);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false);
    const auto hi =
        __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
    return join_words(lo[0], hi[0]) + join_words(lo[1], hi[1]);
}
// lower-half value + upper-half value, in every lane
__device__ __forceinline__ double halves_sum(double x)
{
    const unsigned long long u = __double_as_longlong(x);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, false, false);
    const auto hi =
        __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
    return join_words(lo[0], hi[0]) + join_words(lo[1], hi[1]);
}
// row_ror:n is DPP control 0x120 + n
__device__ __forceinline__ double row_sum16(double x)
{
    x += dpp_move<0x128>(x);
    x += dpp_move<0x124>(x);
    x += dpp_move<0x122>(x);
    x += dpp_move<0x121>(x);
    return x;
}
__device__ __forceinline__ double half_sum32(double x)  // over the 32 lanes of a half-wavefront
{
    return rows_pair_sum(row_sum16(x));
}
__device__ __forceinline__ double wave_sum64(double x)
{
    return halves_sum(rows_pair_sum(row_sum16(x)));
}

// Householder reflector H = I - tau v v^T with v_0 = 1 mapping (alpha, x)
// to (beta, 0): from alpha and s2 = |x|^2; v = (1, x * scale). With
// nrm = sqrt(alpha^2 + s2) and beta = -sign(alpha) nrm:
//   tau = (beta - alpha) / beta = 1 + |alpha| / nrm,
//   scale = 1 / (alpha - beta) = sign(alpha) / (|alpha| + nrm),
// from r = 1 / nrm (hardware estimate, two Newton steps r <- r (3 - a r^2) / 2)
// and one reciprocal (estimate, two Newton steps): a shorter dependence chain
// than a square root and two divisions. Every thread runs the same sequence,
// so all of them hold the same bits.
__device__ __forceinline__ void house(double alpha, double s2, double& tau, double& beta,
                                      double& scale)
{
    tau = 0.0;
    beta = alpha;
    scale = 0.0;
    if (s2 > 0.0) {
        const double a2 = fma(alpha, alpha, s2);
        double r = __builtin_amdgcn_rsq(a2);
        const double h = 0.5 * a2;
        r = r * fma(-h * r, r, 1.5);
        r = r * fma(-h * r, r, 1.5);
        const double nrm = a2 * r;
        const double aa = fabs(alpha);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = fma(aa, r, 1.0);
        const double den = aa + nrm;
        double q = __builtin_amdgcn_rcp(den);
        q = fma(q, fma(-den, q, 1.0), q);
        q = fma(q, fma(-den, q, 1.0), q);
        scale = alpha >= 0.0 ? q : -q;
    }
}

// Sums over the 32 lanes of a half-wavefront of four values v[0..3] at once:
// lane l (16-lane row position c = l % 16) ends with the sum of v[2 b3 + b2],
// b3, b2 the bits 3 and 2 of c. Reduce-scatter over the first two levels
// (DPP row rotation by 8 pairs c with c ^ 8, the half-row mirror pairs c with
// 7 - c across bit 2; each lane keeps the half its bit selects and adds the
// partner's copy of it), then sums within quads (xor 2, xor 1) and across the
// two rows (permlane16 swap): about half the instructions of four full sums.
__device__ __forceinline__ double quad_col_sum(const double (&v)[4])
{
    const int c = threadIdx.x & 15;
    const bool b3 = (c & 8) != 0, b2 = (c & 4) != 0;
    double k0 = b3 ? v[2] : v[0], k1 = b3 ? v[3] : v[1];
    const double s0 = b3 ? v[0] : v[2], s1 = b3 ? v[1] : v[3];
    k0 += dpp_move<0x128>(s0);  // row_ror:8
    k1 += dpp_move<0x128>(s1);
    double r = (b2 ? k1 : k0) + dpp_move<0x141>(b2 ? k0 : k1);  // row_half_mirror
    r += dpp_move<0x4E>(r);                                    // quad_perm [2,3,0,1]
    r += dpp_move<0xB1>(r);                                    // quad_perm [1,0,3,2]
    return rows_pair_sum(r);
}

constexpr int GK_LD = GK_MAXN + 1;  // padded LDS row of the partial sums

struct GkShared {
    double part[8 * GK_LD];  // per-wavefront partial products B x (right reflection)
    double xc[GK_MAXN];      // the current column (rows >= k): the next left reflection
    double cp[GK_MAXN];      // column k + 1 after the left reflection of step k
    double zs[GK_MAXN];      // B v of the right reflection (without tau), rows > k
    double sx[16 * 16];      // row k beyond k + 1, per half-wavefront: its own columns only
    double srk[16 * 16];     // row k before the left reflection, per half-wavefront
    double sw[16 * 16];      // weights of the left update, per half-wavefront
    double pn[8];            // per-wavefront partial sums of squares of row k
    double ax;               // B[k][k + 1] after the left reflection
};

// Row stores of the reflectors go through buffer resources: the per-lane
// part of the address is then a 32-bit offset, and no 64-bit per-lane pointer
// is held in registers beside the matrix tile. Stores beyond n elements are
// dropped by the hardware range check.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(double* p, int n)
{
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, n * 8, 0x00020000);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, int idx, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, idx * 8, 0, 0);
}

struct GkOut {
    int N;
    int ldv;  // row stride of VL and VR (N, or that of a larger matrix whose trailing part this is)
    double *d, *e, *VL, *tauL, *VR, *tauR;
};

// Steps k of column block KC (16 KC <= k < 16 KC + 16) of the one-workgroup
// bidiagonalisation; row group KC / 2 and column group KC are compile-time,
// so groups wholly above or left of the active trailing matrix cost nothing.
// Per step two barriers:
//  - left reflection of column k (from xc, every wavefront forms it itself):
//    the column products q_j = sum_{i > k} xc_i B_ij are summed over the 32
//    row-lanes of a half-wavefront while the norm is formed, and combined with
//    row k (read across lanes) once the scale is known;
//  - right reflection of row k: its entries are known in every lane after the
//    left update; each wavefront publishes its share of |x|^2 and of B x, the
//    owner of column k + 1 publishes that column (barrier 1); thread i forms
//    z_i = (B v)_i and the next column (barrier 2), and every thread applies
//    the rank-1 update to its part.
template <int NPR, int KC>
__device__ __forceinline__ void gk_block(GkShared& sh, const GkOut& o,
                                         double (&Br)[NPR][2 * NPR])
{
    constexpr int NPC = 2 * NPR;
    if constexpr (KC < NPC) {
        constexpr int KA = KC / 2;
        const int N = o.N;
        const int tid = threadIdx.x, lane = tid & 63, tr = tid & 31, tc = tid >> 5;
        const int ldv = o.ldv;
        const int nv = (N - 1) * ldv + N;  // the reflector rows' extent
        const __amdgpu_buffer_rsrc_t rVL = buf_rsrc(o.VL, nv), rVR = buf_rsrc(o.VR, nv);
        const int kend = min(16 * KC + 16, N);
        for (int k = 16 * KC; k < kend; ++k) {
            // Lane tests against step k. Here 16 KC <= k < 16 KC + 16, so
            // only column groups KC, KC + 1 and row group KA can straddle the
            // boundary; the tests are written so (once the loops over c and
            // a are unrolled) the others fold to constants and no per-column
            // index is kept in a register.
            const int kr = k - 16 * KC;  // 0 .. 15
            const int kq = k - 32 * KA;  // 0 .. 31
            auto row_gt = [&](int a) { return a == KA ? tr > kq : true; };          // i > k
            auto row_eq = [&](int a) { return a == KA && tr == kq; };              // i == k
            auto col_gt = [&](int c) { return c == KC ? tc > kr : true; };         // j > k
            auto col_ge2 = [&](int c) {                                           // j >= k + 2
                return c == KC ? tc >= kr + 2 : (c == KC + 1 ? tc >= kr - 14 : true);
            };
            auto col_eq1 = [&](int c) {                                           // j == k + 1
                return c == KC ? tc == kr + 1 : (c == KC + 1 && tc == kr - 15);
            };
            // ---- left reflection of column k
            const double alphaL = sh.xc[k];
            double s2a = 0.0, s2b = 0.0;
            {
                int i = k + 1 + lane;
                for (; i + 64 < N; i += 128) {
                    const double u0 = sh.xc[i], u1 = sh.xc[i + 64];
                    s2a += u0 * u0;
                    s2b += u1 * u1;
                }
                if (i < N) s2a += sh.xc[i] * sh.xc[i];
            }
            // the reflector needs only column k
            double tauLk, betaL, scaleL;
            house(alphaL, wave_sum64(s2a + s2b), tauLk, betaL, scaleL);
            // the owner of row k in each half-wavefront hands its entries to the
            // lanes that finish the column sums, through the half-wavefront's
            // own LDS row (read back by the same wavefront, in order)
            if (tr == (k & 31)) {
#pragma unroll
                for (int c = KC; c < NPC; ++c) sh.srk[tc * 16 + c] = Br[KA][c];
            }
            double xa[NPR];
#pragma unroll
            for (int a = KA; a < NPR; ++a)  // rows > k (xc is zero beyond N)
                xa[a] = row_gt(a) ? sh.xc[tr + 32 * a] : 0.0;
            // Column sums q_j = sum_{i > k} xc_i B_ij, four columns at a time;
            // lane 4 u of the first row then holds q for column g + u and forms
            // that column's weight w_j = tau (B_kj + scale q_j) of the left
            // update (zero for j <= k), row k after the update (x_j, kept for
            // j >= k + 2) and, for j = k + 1, the right reflector's alpha.
#pragma unroll
            for (int g = KC; g < NPC; g += 4) {
                double v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int c = g + u < NPC ? g + u : NPC - 1;
                    double p = 0.0;
#pragma unroll
                    for (int a = KA; a < NPR; ++a) p += xa[a] * Br[a][c];
                    v[u] = g + u < NPC ? p : 0.0;
                }
                const double q4 = quad_col_sum(v);
                const int l16 = tr & 15;
                const int c = g + (l16 >> 2);
                if (tr < 16 && (l16 & 3) == 0 && c < NPC) {
                    const double rk = sh.srk[tc * 16 + c];  // B[k][j]
                    const double wj = col_gt(c) ? tauLk * (rk + scaleL * q4) : 0.0;
                    const double xk = rk - wj;
                    sh.sw[tc * 16 + c] = wj;
                    sh.sx[tc * 16 + c] = col_ge2(c) ? xk : 0.0;
                    if (col_eq1(c)) sh.ax = xk;
                }
            }
            if (tid > k && tid < N) buf_st(rVL, k * ldv + tid, sh.xc[tid] * scaleL);
            if (tid == k) {
                o.VL[(size_t)k * ldv + k] = 1.0;
                o.tauL[k] = tauLk;
                o.d[k] = betaL;
            }
            // left update B <- B - v w^T over rows > k (row k: v = 1)
#pragma unroll
            for (int a = KA; a < NPR; ++a) xa[a] = row_eq(a) ? 1.0 : xa[a] * scaleL;
#pragma unroll
            for (int c = KC; c < NPC; ++c) {  // column j = tc + 16 c; zero beyond N
                const double wj = sh.sw[tc * 16 + c];
#pragma unroll
                for (int a = KA; a < NPR; ++a) Br[a][c] -= xa[a] * wj;
            }
            if (k + 1 >= N) break;
            // ---- right reflection of row k: partial sums, column k + 1
            // (sx is private to the half-wavefront: written and read back by
            // the same wavefront, in order)
            {
                if (tc == ((k + 1) & 15)) {
                    const bool next = (k & 15) == 15;
#pragma unroll
                    for (int a = KA; a < NPR; ++a) {
                        double v = Br[a][KC];
                        if constexpr (KC + 1 < NPC)
                            if (next) v = Br[a][KC + 1];
                        if (row_gt(a)) sh.cp[tr + 32 * a] = v;
                    }
                }
                // row k's entries are read as they are used (not held in
                // registers beside the tile)
                double acc[NPR];
#pragma unroll
                for (int a = KA; a < NPR; ++a) acc[a] = 0.0;
                double pa = 0.0, pb = 0.0;
#pragma unroll
                for (int c = KC; c < NPC; ++c) {
                    const double x = sh.sx[tc * 16 + c];
                    if ((c - KC) & 1)
                        pb += x * x;
                    else
                        pa += x * x;
#pragma unroll
                    for (int a = KA; a < NPR; ++a) acc[a] += Br[a][c] * x;
                }
                const double pnh = halves_sum(pa + pb);
                if (lane == 0) sh.pn[tid >> 6] = pnh;
#pragma unroll
                for (int a = KA; a < NPR; ++a) {
                    const double t = halves_sum(acc[a]);
                    if (lane < 32) sh.part[(tid >> 6) * GK_LD + tr + 32 * a] = t;
                }
            }
            __syncthreads();
            double tauRk, betaR, scaleR;
            {
                double s2 = 0.0;
#pragma unroll
                for (int w = 0; w < 8; ++w) s2 += sh.pn[w];
                house(sh.ax, s2, tauRk, betaR, scaleR);
            }
            if (tr < NPC - KC) {  // lane tr stores column tc + 16 (KC + tr) of row k
                const int j = tc + 16 * (KC + tr);
                if (j >= k + 2 && j < N) buf_st(rVR, k * ldv + j, sh.sx[tc * 16 + KC + tr] * scaleR);
            }
            if (tid == 0) {
                o.VR[(size_t)k * ldv + k + 1] = 1.0;
                o.tauR[k] = tauRk;
                o.e[k] = betaR;
            }
            if (tid > k && tid < N) {
                double s0 = 0.0, s1 = 0.0;
#pragma unroll
                for (int w = 0; w < 8; w += 2) {
                    s0 += sh.part[w * GK_LD + tid];
                    s1 += sh.part[(w + 1) * GK_LD + tid];
                }
                const double c0 = sh.cp[tid];
                const double z = c0 + scaleR * (s0 + s1);
                sh.zs[tid] = z;
                sh.xc[tid] = c0 - tauRk * z;
            }
            __syncthreads();
            // ---- right update: rows > k, columns > k
            {
                double zr[NPR];
#pragma unroll
                for (int a = KA; a < NPR; ++a)  // zs is zero beyond N
                    zr[a] = row_gt(a) ? tauRk * sh.zs[tr + 32 * a] : 0.0;
#pragma unroll
                for (int c = KC; c < NPC; ++c) {
                    const double vj =
                        col_eq1(c) ? 1.0 : sh.sx[tc * 16 + c] * scaleR;
#pragma unroll
                    for (int a = KA; a < NPR; ++a) Br[a][c] -= zr[a] * vj;
                }
            }
        }
        gk_block<NPR, KC + 1>(sh, o, Br);
    }
}

// One-workgroup bidiagonalisation for N <= 32 NPR (NPR <= 7): thread
// (tr, tc) of the 32 x 16 grid owns rows tr + 32a (a < NPR) and columns
// tc + 16c (c < 2 NPR), 7 x 14 doubles at N = 224. Reflector k is row k of
// VL / VR with stride ldv (N; larger when B is the trailing part of a bigger
// matrix whose first steps the cooperative kernel took).
template <int NPR>
__global__ __launch_bounds__(512) void gk_bidiag_kernel(int N, const double* __restrict__ B,
                                                        int ldb, double* __restrict__ dout,
                                                        double* __restrict__ eout,
                                                        double* __restrict__ VL,
                                                        double* __restrict__ tauL,
                                                        double* __restrict__ VR,
                                                        double* __restrict__ tauR, int ldv)
{
    constexpr int NPC = 2 * NPR;
    __shared__ GkShared sh;
    const int tid = threadIdx.x;
    const int tr = tid & 31, tc = tid >> 5;

    double Br[NPR][NPC];
#pragma unroll
    for (int a = 0; a < NPR; ++a)
#pragma unroll
        for (int c = 0; c < NPC; ++c) {
            const int i = tr + 32 * a, j = tc + 16 * c;
            Br[a][c] = (i < N && j < N) ? B[(size_t)i * ldb + j] : 0.0;
        }
    if (tid < GK_MAXN) {  // beyond N these stay zero
        sh.xc[tid] = tid < N ? B[(size_t)tid * ldb] : 0.0;
        sh.zs[tid] = 0.0;
    }
    __syncthreads();
    const GkOut o{N, ldv, dout, eout, VL, tauL, VR, tauR};
    gk_block<NPR, 0>(sh, o, Br);
}

// ---------------------------------------------------------------------------
// Cooperative Golub-Kahan bidiagonalisation for GK_MAXN < N <= SVD_MAXN.
//
// P = ceil(N / 32) workgroups, all resident at once (cooperative launch).
// Workgroup p holds columns 32p .. 32p + 31 of B in registers: thread (g, c)
// of a 16 x 32 grid owns column 32p + c and rows g + 16q (q < NQ). Per step k:
//  - every workgroup forms the left reflector of column k on its own, from
//    the column as published in the previous step, and applies it to its
//    columns (no barrier needed);
//  - for the right reflector of row k (x = row k beyond the superdiagonal)
//    each workgroup publishes the sum of squares of its part of x and its
//    part of sum_j B[i][j] x_j, and the owner of column k + 1 publishes that
//    column; after ONE device-wide barrier every workgroup forms the
//    reflector, z = B v and the next column from these in a fixed order
//    (so all workgroups hold bit-identical copies) and updates its columns.
// The barrier waits are bounded: on a timeout the error flag is set and every
// workgroup leaves the kernel.
// ---------------------------------------------------------------------------
constexpr unsigned CO_SPIN_LIMIT = 1u << 22;

// A compiler barrier right after a batch of loads keeps them issued together
// (otherwise they are folded into loads at their use, each waited on in turn).
__device__ __forceinline__ void loads_issued() { asm volatile("" ::: "memory"); }

struct CoopBuf {
    double* colpub;  // 2 x N: column k + 1 before the right update
    double* nrm;     // 2 x P: partial sums of squares of row k
    double* part;    // 2 x P x N: partial products B x
    unsigned* ctr;   // barrier arrivals (zero at launch)
    int* err;        // set on a barrier timeout
};

// The partials are exchanged with plain stores and loads: the barrier's
// agent-scope release (after the stores) and acquire (before the loads) make
// them visible across the XCDs, and plain loads can all be in flight at once.
__device__ __forceinline__ double ld_agent(const double* p) { return *p; }
__device__ __forceinline__ void st_agent(double* p, double v) { *p = v; }

// Device-wide barrier among the co-resident workgroups. Every wavefront
// first waits for its own stores to complete (so they sit in this XCD's L2);
// after the workgroup barrier one thread makes them visible at agent scope
// (release: L2 write-back), arrives, polls the counter with relaxed loads
// (bounded), and invalidates the local caches once (acquire) before the
// workgroup continues.
__device__ bool coop_barrier(unsigned* ctr, unsigned target, int* err, int* ok_lds)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        unsigned spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                ++spins > CO_SPIN_LIMIT) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *ok_lds = ok;
    }
    __syncthreads();
    return *ok_lds != 0;
}

// Butterfly transpose-reduction over the 32 lanes of a half-wavefront: lane
// c holds v[0..32); on return v[0] of lane c is the sum over the 32 lanes of
// their v[c]. Each level pairs lane c with c ^ s; the lane keeps the half of
// its remaining values whose index bit matches its own lane bit and adds the
// partner's copy of that half (31 shuffles in all, the adds independent).
template <int S>
__device__ __forceinline__ void transpose_level(double (&v)[32], bool hi)
{
#pragma unroll
    for (int j = 0; j < S; ++j) {
        const double keep = hi ? v[j + S] : v[j];
        const double send = hi ? v[j] : v[j + S];
        v[j] = keep + __shfl_xor(send, S, 64);
    }
}

// Level 16 by v_permlane16_swap on (v[j], v[j + 16]): the even row of each
// pair ends with (own v[j], partner's v[j]), the odd row with (partner's
// v[j + 16], own v[j + 16]).
__device__ __forceinline__ void transpose_level16(double (&v)[32])
{
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const unsigned long long a = __double_as_longlong(v[j]), b = __double_as_longlong(v[j + 16]);
        const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)a, (unsigned)b, false, false);
        const auto hi =
            __builtin_amdgcn_permlane16_swap((unsigned)(a >> 32), (unsigned)(b >> 32), false, false);
        v[j] = join_words(lo[0], hi[0]) + join_words(lo[1], hi[1]);
    }
}

__device__ __forceinline__ void transpose_sum32(double (&v)[32], int c)
{
    transpose_level16(v);
    transpose_level<8>(v, (c & 8) != 0);
    transpose_level<4>(v, (c & 4) != 0);
    transpose_level<2>(v, (c & 2) != 0);
    transpose_level<1>(v, (c & 1) != 0);
}

// Steps 0 .. kstop - 1 only when kstop < N: the trailing matrix
// B[kstop:, kstop:] after them is written to Tout (leading dimension
// N - kstop), whose bidiagonalisation gives the remaining steps.
template <int NQ>
__global__ __launch_bounds__(512) void gk_bidiag_coop_kernel(
    int N, const double* __restrict__ B, int ldb, double* __restrict__ dout,
    double* __restrict__ eout, double* __restrict__ VL, double* __restrict__ tauL,
    double* __restrict__ VR, double* __restrict__ tauR, CoopBuf cb, int kstop,
    double* __restrict__ Tout)
{
    __shared__ double xcol[SVD_MAXN];  // column k, then the left vector
    __shared__ double zs[SVD_MAXN];    // z = B v of the right reflector
    __shared__ double red[16][33];
    __shared__ double red0[16][33];
    __shared__ double wcol[32];
    __shared__ double rowk[32];
    __shared__ double sc[4];
    __shared__ int okl;
    const int P = gridDim.x, p = blockIdx.x;
    const int tid = threadIdx.x, c = tid & 31, g = tid >> 5, lane = tid & 63, wave = tid >> 6;
    const int j = 32 * p + c;
    const bool jv = j < N;

    double a[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = g + 16 * q;
        a[q] = (i < N && jv) ? B[(size_t)i * ldb + j] : 0.0;
    }
    for (int i = tid; i < N; i += 512) xcol[i] = B[(size_t)i * ldb];
    __syncthreads();

    for (int k = 0; k < kstop; ++k) {
        // ---- left reflector of column k (rows k..N-1), formed by every
        // wavefront of every workgroup from the published column (the same
        // loads and the same order everywhere: the same bits). The column
        // products are taken unscaled, sum_{i > k} x_i B[i][j] and row k's own
        // entry apart, while the norm is formed:
        //   w_j = tau (B[k][j] + scale sum_{i > k} x_i B[i][j]).
        double tl, sl;
        {
            const double alpha = xcol[k];
            double s2a = 0.0, s2b = 0.0;
            {
                int i = k + 1 + lane;
                for (; i + 64 < N; i += 128) {
                    const double u0 = xcol[i], u1 = xcol[i + 64];
                    s2a += u0 * u0;
                    s2b += u1 * u1;
                }
                if (i < N) s2a += xcol[i] * xcol[i];
            }
            // the column entries are read 16 row groups at a time, all loads
            // of a batch issued before any is used; rows outside k < i < N
            // are masked by a select (xcol beyond N is never written)
            double pw[4] = {0.0, 0.0, 0.0, 0.0}, p0 = 0.0;
#pragma unroll
            for (int q0 = 0; q0 < NQ; q0 += 16) {
                if (16 * q0 + 255 < k) continue;  // uniform
                double xq[16];
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (q0 + u < NQ) xq[u] = xcol[g + 16 * (q0 + u)];
                loads_issued();
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int q = q0 + u;
                    if (q >= NQ) break;
                    const int i = g + 16 * q;
                    pw[q & 3] += (i > k && i < N) ? xq[u] * a[q] : 0.0;
                    if (i == k) p0 = a[q];
                }
            }
            red[g][c] = (pw[0] + pw[1]) + (pw[2] + pw[3]);
            red0[g][c] = p0;
            double beta;
            house(alpha, wave_sum64(s2a + s2b), tl, beta, sl);
            if (p == 0) {
                for (int i = k + 1 + tid; i < N; i += 512) VL[(size_t)k * N + i] = xcol[i] * sl;
                if (tid == 0) {
                    VL[(size_t)k * N + k] = 1.0;
                    tauL[k] = tl;
                    dout[k] = beta;
                }
            }
        }
        __syncthreads();
        if (tl != 0.0) {
            if (tid < 32) {
                double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0, r0 = 0.0;
#pragma unroll
                for (int gg = 0; gg < 16; gg += 4) {
                    w0 += red[gg][tid];
                    w1 += red[gg + 1][tid];
                    w2 += red[gg + 2][tid];
                    w3 += red[gg + 3][tid];
                }
#pragma unroll
                for (int gg = 0; gg < 16; ++gg) r0 += red0[gg][tid];  // one nonzero term
                wcol[tid] = tl * fma(sl, (w0 + w1) + (w2 + w3), r0);
            }
            __syncthreads();
            const double wj = (jv && j > k) ? wcol[c] : 0.0;
#pragma unroll
            for (int q0 = 0; q0 < NQ; q0 += 16) {
                if (16 * q0 + 255 < k) continue;  // uniform
                double xq[16];
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (q0 + u < NQ) xq[u] = xcol[g + 16 * (q0 + u)];
                loads_issued();
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int q = q0 + u;
                    if (q >= NQ) break;
                    const int i = g + 16 * q;
                    const double vi = (i == k) ? 1.0 : xq[u] * sl;
                    a[q] = (i >= k && i < N) ? a[q] - vi * wj : a[q];
                }
            }
        }
        if (k + 1 >= N) break;

        // ---- right reflector of row k: this workgroup's partials
        const int slot = k & 1;
        if (g == (k & 15)) {
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                if (q == (k >> 4)) v = a[q];
            rowk[c] = jv ? v : 0.0;
        }
        __syncthreads();
        {
            // partial (B x)_i over this slab's columns, rows i = g + 16 q: the
            // products of the 32 column-lanes summed by a transpose-reduction,
            // after which lane c holds row g + 16 (q0 + c)
            const double xj = (jv && j >= k + 2) ? rowk[c] : 0.0;
            double* prow = cb.part + ((size_t)slot * P + p) * N;
#pragma unroll
            for (int q0 = 0; q0 < NQ; q0 += 32) {
                double v[32];
#pragma unroll
                for (int u = 0; u < 32; ++u) v[u] = (q0 + u < NQ) ? a[q0 + u < NQ ? q0 + u : 0] * xj : 0.0;
                transpose_sum32(v, c);
                const int i = g + 16 * (q0 + c);
                if (q0 + c < NQ && i >= k + 1 && i < N) st_agent(prow + i, v[0]);
            }
        }
        if (tid < 64) {  // this slab's part of |x|^2, summed over the 32 column lanes
            const double rv = (c == tid && jv && j >= k + 2) ? rowk[c] : 0.0;
            const double s2 = half_sum32(rv * rv);
            if (tid == 0) st_agent(cb.nrm + slot * P + p, s2);
        }
        if (p == ((k + 1) >> 5) && c == ((k + 1) & 31)) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int i = g + 16 * q;
                if (i >= k && i < N) st_agent(cb.colpub + (size_t)slot * N + i, a[q]);
            }
        }
        if (!coop_barrier(cb.ctr, (unsigned)(k + 1) * (unsigned)P, cb.err, &okl)) return;

        // ---- the reflector, z = B v and the next column, from the partials;
        // every thread loads the norms with its partials and forms the
        // reflector itself (same loads, same order: the same bits everywhere)
        // Up to N = 512 (P <= 16) all of this step's exchange this thread
        // needs (alpha, the P norms, row k + 1 + tid's P partials and column
        // entry) is loaded at once, from clamped addresses, before any is
        // used: one memory round trip instead of one per load. The sums run in
        // the fixed order q = 0 .. P - 1 either way.
        constexpr int PB = NQ <= 32 ? (NQ + 1) / 2 : 1;
        const int i0 = k + 1 + tid;
        const int ic = i0 < N ? i0 : N - 1;
        double nb[PB], pb[PB], cp0 = 0.0;
        if constexpr (NQ <= 32) {
#pragma unroll
            for (int q = 0; q < PB; ++q) {
                const int qc = q < P ? q : P - 1;
                nb[q] = ld_agent(cb.nrm + slot * P + qc);
                pb[q] = ld_agent(cb.part + ((size_t)slot * P + qc) * N + ic);
            }
            cp0 = ld_agent(cb.colpub + (size_t)slot * N + ic);
        }
        double tq, scl;
        {
            const double alpha = ld_agent(cb.colpub + (size_t)slot * N + k);
            loads_issued();
            double s2 = 0.0;
            if constexpr (NQ <= 32) {
#pragma unroll
                for (int q = 0; q < PB; ++q)
                    if (q < P) s2 += nb[q];
            } else {
                for (int q = 0; q < P; ++q) s2 += ld_agent(cb.nrm + slot * P + q);
            }
            double tau, beta, scale;
            house(alpha, s2, tau, beta, scale);
            tq = tau;
            scl = scale;
            if (p == 0 && tid == 0) {
                tauR[k] = tau;
                eout[k] = beta;
            }
        }
        int ibeg = k + 1 + tid;
        if constexpr (NQ <= 32) {
            if (i0 < N) {
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < PB; ++q)
                    if (q < P) acc += pb[q];
                const double z = cp0 + scl * acc;
                zs[i0] = z;
                xcol[i0] = cp0 - tq * z;
            }
            ibeg += 512;
        }
        for (int i = ibeg; i < N; i += 512) {
            double acc = 0.0;
            for (int q = 0; q < P; ++q) acc += ld_agent(cb.part + ((size_t)slot * P + q) * N + i);
            const double cp = ld_agent(cb.colpub + (size_t)slot * N + i);
            const double z = cp + scl * acc;
            zs[i] = z;
            xcol[i] = cp - tq * z;
        }
        if (g == 0 && jv && j >= k + 1) VR[(size_t)k * N + j] = (j == k + 1) ? 1.0 : rowk[c] * scl;
        __syncthreads();
        if (tq != 0.0) {
            const double vj = (jv && j >= k + 1) ? ((j == k + 1) ? 1.0 : rowk[c] * scl) : 0.0;
#pragma unroll
            for (int q0 = 0; q0 < NQ; q0 += 16) {
                if (16 * q0 + 255 < k + 1) continue;  // uniform
                double zq[16];
#pragma unroll
                for (int u = 0; u < 16; ++u)
                    if (q0 + u < NQ) zq[u] = zs[g + 16 * (q0 + u)];
                loads_issued();
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int q = q0 + u;
                    if (q >= NQ) break;
                    const int i = g + 16 * q;
                    a[q] = (i >= k + 1 && i < N) ? a[q] - tq * zq[u] * vj : a[q];
                }
            }
        }
        __syncthreads();  // rowk, zs and sc are rewritten in the next step
    }
    if (kstop < N && jv && j >= kstop) {
        const int nt = N - kstop;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = g + 16 * q;
            if (i >= kstop && i < N) Tout[(size_t)(i - kstop) * nt + (j - kstop)] = a[q];
        }
    }
}

// The recurrences below read their operands from LDS in blocks of eight,
// alternating between two register sets: the loads of one block are issued
// before the previous block is computed (loads_issued keeps them there).

// Number of singular values of the upper bidiagonal B = (d, e) below sqrt(tau),
// by the differential stationary qd transform of B^T B - tau I = L D L^T
// carried on the squared entries q_i = d_i^2, ee_i = e_i^2 (B^T B is never
// formed): from s_0 = -tau,
//   D_i = q_i + s_i,    s_{i+1} = ee_i s_i / D_i - tau,
// and by Sylvester's law of inertia the number of negative D_i is the number
// of eigenvalues of B^T B below tau. The transform is exact for entries
// perturbed by a few units in the last place, so the count carries the
// relative accuracy of the bidiagonal's values, at half the length of the
// Sturm sequence of the Golub-Kahan tridiagonal. 1 / D is the hardware
// estimate (relative error ~5e-8) refined by one Newton step (~2e-15), which
// again perturbs ee_i in the 15th digit only.
// Without GUARD a pivot D = 0 (or one whose quotient overflows) turns s into
// a NaN or an infinity that reaches the end of the chain; the caller then
// counts again with GUARD, which replaces |D| < pivmin by -pivmin. (The
// recurrence is a chain of dependent operations; the guard would lengthen it.)
template <bool GUARD>
__device__ __forceinline__ void qd_block(const double2 (&c)[8], double& s, int& neg, double tau,
                                         double pivmin)
{
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        double D = c[u].x + s;
        if (GUARD) D = fabs(D) < pivmin ? -pivmin : D;
        neg += D < 0.0;
        double r = __builtin_amdgcn_rcp(D);
        r = fma(r, fma(-D, r, 1.0), r);
        s = fma(c[u].y * s, r, -tau);
    }
}

// qe holds (q_i, ee_i) for i < N with ee_{N-1} = 0, then at least 23 pad
// pairs (4, 0) that are never counted (the entries are scaled below 1, so
// tau < 1 and 4 - tau > 0). The chain ends with s = -tau unless a pivot
// broke it.
template <bool GUARD>
__device__ __forceinline__ int count_below(int N, const double2* __restrict__ qe, double tau,
                                           double pivmin, double& s_end)
{
    int neg = 0;
    double s = -tau;
    double2 a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = qe[u];
    for (int i0 = 0; i0 < N; i0 += 16) {
#pragma unroll
        for (int u = 0; u < 8; ++u) b[u] = qe[i0 + 8 + u];
        loads_issued();
        qd_block<GUARD>(a, s, neg, tau, pivmin);
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = qe[i0 + 16 + u];
        loads_issued();
        qd_block<GUARD>(b, s, neg, tau, pivmin);
    }
    s_end = s;
    return neg;
}

// One inverse-iteration factor row: the multiplier of L, and U's row divided
// by its diagonal.
struct InvFac {
    double dl, rdd, bdu, bdu2;
};

// One step of the LU factorisation with partial pivoting of the tridiagonal
// T - s I (zero diagonal, off-diagonals f): rows j and j + 1 of the active
// part are (.. ddj duj 0 ..) and (.. dlj -s dun ..). The pivot is the larger
// of ddj, dlj; a pivot below `tiny` in magnitude is taken as +-tiny. A row
// interchange gives U a second superdiagonal. The quotient uses the hardware
// reciprocal refined by one Newton step; the stored 1 / u_jj by two.
// Beyond the last row (dlj = dun = 0) a step stores 1 / u_jj of the last row
// and zero multipliers, and leaves ddj = -s.
__device__ __forceinline__ void lu_step(double& ddj, double& duj, double dlj, double dun,
                                        double s, double tiny, InvFac& o, unsigned char& sw)
{
    const bool swp = fabs(ddj) < fabs(dlj);
    const double piv = swp ? dlj : ddj;
    const double oth = swp ? ddj : dlj;
    const double pc = fabs(piv) < tiny ? (piv < 0.0 ? -tiny : tiny) : piv;
    double r = __builtin_amdgcn_rcp(pc);
    r = fma(r, fma(-pc, r, 1.0), r);
    const double fact = oth * r;
    const double odu = swp ? -s : duj;
    const double odu2 = swp ? dun : 0.0;
    const double ndd = swp ? fma(fact, s, duj) : fma(-fact, duj, -s);
    duj = swp ? -fact * dun : dun;
    ddj = ndd;
    const double rd = fma(r, fma(-pc, r, 1.0), r);
    o.dl = fact;
    o.rdd = rd;
    o.bdu = odu * rd;
    o.bdu2 = odu2 * rd;
    sw = swp;
}

// The factorisation's dependence chain alone: the multiplier is formed both
// ways, dlj / ddj from a reciprocal of ddj on the chain and ddj / dlj from
// the reciprocal rl of dlj taken beforehand, and the pivot test only selects
// between them. The step stores the multiplier and the incoming (ddj, duj);
// U's row divided by its (guarded) diagonal is formed afterwards for all rows
// at once (tgk_solve_kernel). For nonzero pivots this gives lu_step's factors
// except that a pivot below `tiny` is used as it is in the multiplier.
__device__ __forceinline__ void lu_chain_step(double& ddj, double& duj, double dlj, double rl,
                                              double dun, double s, InvFac& o, unsigned char& sw)
{
    const bool swp = fabs(ddj) < fabs(dlj);
    double r = __builtin_amdgcn_rcp(ddj);
    r = fma(r, fma(-ddj, r, 1.0), r);
    const double fact = swp ? ddj * rl : dlj * r;
    o.dl = fact;
    o.rdd = ddj;  // replaced by 1 / u_jj
    o.bdu = duj;  // replaced by u_j,j+1 / u_jj
    sw = swp;
    const double ndd = swp ? fma(fact, s, duj) : fma(-fact, duj, -s);
    duj = swp ? -fact * dun : dun;
    ddj = ndd;
}

template <int B0>
__device__ __forceinline__ void lu_chain_block(double& ddj, double& duj, const double (&fw)[9],
                                               const double (&rl)[8], double s, InvFac* fac,
                                               unsigned char* swp)
{
#pragma unroll
    for (int u = 0; u < 8; ++u)
        lu_chain_step(ddj, duj, fw[u], rl[u], fw[u + 1], s, fac[B0 + u], swp[B0 + u]);
}

template <int B0>
__device__ __forceinline__ void lu_block(double& ddj, double& duj, const double (&fw)[9], double s,
                                         double tiny, InvFac* fac, unsigned char* swp)
{
#pragma unroll
    for (int u = 0; u < 8; ++u) lu_step(ddj, duj, fw[u], fw[u + 1], s, tiny, fac[B0 + u], swp[B0 + u]);
}

// Forward substitution with L (row interchanges as recorded), z_j carried;
// zn holds z_{j+1} before it is overwritten, scaled by `inv` on use.
__device__ __forceinline__ void fwd_block(double& zj, const double (&zn)[8], const double (&l)[8],
                                          const unsigned char (&sw)[8], double inv, double* z)
{
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const double znx = zn[u] * inv;
        const double out = sw[u] ? znx : zj;
        const double oth = sw[u] ? zj : znx;
        z[u] = out;
        zj = fma(-l[u], out, oth);
    }
}

// Back substitution, rows j, j - 1, ..., j - 7 with z_{j+1}, z_{j+2} carried:
// z_j = z_j / u_jj - (u_j,j+1 / u_jj) z_{j+1} - (u_j,j+2 / u_jj) z_{j+2}.
__device__ __forceinline__ void bwd_block(double& z1, double& z2, const InvFac (&c)[8],
                                          const double (&zc)[8], double* z)
{
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        const double z0 = fma(-c[u].bdu, z1, fma(-c[u].bdu2, z2, zc[u] * c[u].rdd));
        z[-u] = z0;
        z2 = z1;
        z1 = z0;
    }
}

// Eight steps of the factorisation T - ss I = L D L^T of a tridiagonal with
// zero diagonal and off-diagonals g (top-down, or bottom-up on the reversed
// off-diagonals): the pivot x_j is stored, m_j = g_j / x_j, and
// x_{j+1} = -ss - m_j g_j. A pivot below pivmin in magnitude is taken as
// -pivmin (IEEE arithmetic then carries the huge multiplier through).
__device__ __forceinline__ void twist_block(double& x, const double (&g)[8], double ss,
                                            double pivmin, double* X, double* M)
{
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        X[u] = x;
        const double xc = fabs(x) < pivmin ? -pivmin : x;
        double r = __builtin_amdgcn_rcp(xc);
        r = fma(r, fma(-xc, r, 1.0), r);
        const double m = g[u] * r;
        M[u] = m;
        x = fma(-m, g[u], -ss);
    }
}

// Singular value sigma_t (the t-th largest) of the bidiagonal (d, e) and its
// left and right singular vectors, one workgroup per value.
//  - Values: multisection on [0, Gershgorin bound] with BS_PTS Sturm counts
//    per step (count_below), to relative precision 2u (absolute u ||B|| near
//    zero). The entries are first scaled by a power of two to below 1.
//  - Vectors: inverse iteration on the Golub-Kahan tridiagonal T (zero
//    diagonal, off-diagonals (d_0, e_0, d_1, e_1, ...)) at +sigma_t: the LU
//    factorisation of T - sigma I, then two solves from the counter-based
//    start vector, rescaled to max |z| = 1 in between. The eigenvector
//    z = (v_0, u_0, v_1, u_1, ...) splits into the right and left singular
//    vectors, each normalised.
// The factorisation and the solves are recurrences run by one thread in
// blocks of eight steps. Blocks run past the ends of the n = 2N rows into
// padding (zero off-diagonals above, an offset of TG_OFF rows below); n is
// even, so the factorisation's blocks always include its step n - 1, which
// stores the last 1 / u_jj.
constexpr int BS_PTS = 256;
constexpr int TG_PAD = 24;
constexpr int TG_OFF = 24;
constexpr int TG_TW = TG_OFF + 2 * SVD_MAXN + TG_PAD;
struct TgkShared {
    union {
        double2 qe[SVD_MAXN + TG_PAD];                     // multisection
        InvFac fac[TG_OFF + 2 * SVD_MAXN + TG_PAD];        // LU factors, row j at TG_OFF + j
        struct {                                           // twisted factorisation:
            double X0[TG_TW], M0[TG_TW];                   //  top-down pivots, multipliers
            double X1[TG_TW], M1[TG_TW];                   //  bottom-up, in reversed order
        } tw;
    };
    double f[2 * SVD_MAXN + TG_PAD];                       // scaled off-diagonals, zero beyond
    double rl[2 * SVD_MAXN + TG_PAD];                      // their reciprocals
    double z[TG_OFF + 2 * SVD_MAXN + TG_PAD];              // row j at TG_OFF + j
    unsigned char swp[TG_OFF + 2 * SVD_MAXN + TG_PAD];
    int cnt[BS_PTS];
    double red[BS_PTS / 64];
    int best;
    int twr;      // twist index
    double twg;   // |gamma| at the twist
};

__global__ __launch_bounds__(BS_PTS) void tgk_solve_kernel(int N, const double* __restrict__ d,
                                                           const double* __restrict__ e,
                                                           double* __restrict__ sig,
                                                           double* __restrict__ ubd,
                                                           double* __restrict__ vbd, int ldv)
{
    __shared__ TgkShared sh;
    const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const int n = 2 * N;
    // Gershgorin bound of T: max_j |f_{j-1}| + |f_j|
    double gb = 0.0;
    for (int j = tid; j < n; j += BS_PTS) {
        const double l = j > 0 ? fabs(((j - 1) & 1) ? e[(j - 1) >> 1] : d[(j - 1) >> 1]) : 0.0;
        const double r = j < n - 1 ? fabs((j & 1) ? e[j >> 1] : d[j >> 1]) : 0.0;
        gb = fmax(gb, l + r);
    }
    for (int off = 32; off > 0; off >>= 1) gb = fmax(gb, __shfl_xor(gb, off, 64));
    if (lane == 0) sh.red[tid >> 6] = gb;
    __syncthreads();
    double bound = 0.0;
#pragma unroll
    for (int w = 0; w < BS_PTS / 64; ++w) bound = fmax(bound, sh.red[w]);
    if (!(bound > 0.0)) {  // B = 0: the value and the vectors are zero
        if (tid == 0) sig[t] = 0.0;
        for (int i = tid; i < N; i += BS_PTS) {
            ubd[(size_t)i * ldv + t] = 0.0;
            vbd[(size_t)i * ldv + t] = 0.0;
        }
        return;
    }
    int ex;
    frexp(bound, &ex);
    const double sc = ldexp(1.0, -ex);  // bound * sc in [0.5, 1)
    const double bs = bound * sc;
    for (int j = tid; j < N + TG_PAD; j += BS_PTS) {
        double2 v = make_double2(4.0, 0.0);
        if (j < N) {
            const double dj = d[j] * sc, ej = j < N - 1 ? e[j] * sc : 0.0;
            v = make_double2(dj * dj, ej * ej);
        }
        sh.qe[j] = v;
    }
    for (int j = tid; j < n + TG_PAD; j += BS_PTS)
        sh.f[j] = j < n - 1 ? ((j & 1) ? e[j >> 1] : d[j >> 1]) * sc : 0.0;
    __syncthreads();
    constexpr double U = 0x1.0p-52;
    constexpr double PIVMIN = 0x1.0p-1000;
    double lo = 0.0, hi = bs * (1.0 + 4.0 * U) + 0x1.0p-1000;
    // invariant: #{sigma >= lo} >= t + 1 (lo = 0 counts every value), #{sigma >= hi} <= t
    for (int step = 0; step < 16; ++step) {
        if (hi - lo <= 2.0 * U * hi || hi - lo <= U * bs) break;
        const double x = lo + (hi - lo) * (double)(tid + 1) / (double)(BS_PTS + 1);
        double s_end;
        int neg = count_below<false>(N, sh.qe, x * x, PIVMIN, s_end);
        if (!(fabs(s_end) <= 4.0))  // a zero pivot broke the chain
            neg = count_below<true>(N, sh.qe, x * x, PIVMIN, s_end);
        sh.cnt[tid] = N - neg;
        if (tid == 0) sh.best = -1;
        __syncthreads();
        // the last point still holding >= t + 1 values
        if (sh.cnt[tid] >= t + 1) atomicMax(&sh.best, tid);
        __syncthreads();
        const int best = sh.best;
        const double nlo = best >= 0 ? lo + (hi - lo) * (double)(best + 1) / (double)(BS_PTS + 1) : lo;
        const double nhi = best < BS_PTS - 1
                               ? lo + (hi - lo) * (double)(best + 2) / (double)(BS_PTS + 1)
                               : hi;
        lo = nlo;
        hi = nhi;
        __syncthreads();
    }
    // a value the bracket cannot separate from zero is reported as zero
    const bool zero = lo == 0.0 && hi <= 8.0 * U * bs;
    const double ss = zero ? 0.0 : 0.5 * (lo + hi);  // sigma_t, scaled
    if (tid == 0) sig[t] = ss / sc;

    // ---- eigenvector of T at +ss (qe is read once more, by the isolation test)
    double* const z = sh.z + TG_OFF;
    InvFac* const fac = sh.fac + TG_OFF;
    unsigned char* const swp = sh.swp + TG_OFF;
    // First by a twisted factorisation: T - ss I = L D L^T (top-down) and
    // U P U^T (bottom-up), run at once by lanes 0 and 1; at the twist index r
    // minimising |gamma_k| = |d_k + p_k + ss|, z_r = 1, z_k = -l_k z_{k+1}
    // above and z_{k+1} = -u_k z_k below (again two lanes at once). Then
    // (T - ss I) z = gamma_r e_r: the vector is accepted when |gamma_r| is
    // within 64 n u ||T|| of ||z|| (and every entry finite); otherwise inverse
    // iteration below computes it. The twisted form is used only for a value
    // isolated to 1e-6 relative (one value in [ss (1 - 1e-6), ss (1 + 1e-6)]
    // widened by 1e-12 ||T||, counted by lanes 0 and 1): the vectors of close
    // or repeated values come from inverse iteration's distinct start vectors.
    if (tid < 2) {
        const double xb = tid == 0 ? ss * (1.0 - 1e-6) - 1e-12 * bs : ss * (1.0 + 1e-6) + 1e-12 * bs;
        int ge = N;  // #{sigma >= xb}
        if (xb > 0.0) {
            double s_end;
            int neg = count_below<false>(N, sh.qe, xb * xb, PIVMIN, s_end);
            if (!(fabs(s_end) <= 4.0)) neg = count_below<true>(N, sh.qe, xb * xb, PIVMIN, s_end);
            ge = N - neg;
        }
        sh.cnt[tid] = ge;
    }
    __syncthreads();
    const bool isolated = ss > 0.0 && sh.cnt[0] - sh.cnt[1] == 1;
    __syncthreads();  // cnt is reused
    bool twisted_ok = false;
    if (isolated) {  // uniform
    for (int j = tid; j < n + TG_PAD; j += BS_PTS)  // rl holds f reversed for now
        sh.rl[j] = j < n - 1 ? sh.f[n - 2 - j] : 0.0;
    __syncthreads();
    if (tid < 2) {
        const double* g = tid == 0 ? sh.f : sh.rl;
        double* X = tid == 0 ? sh.tw.X0 : sh.tw.X1;
        double* M = tid == 0 ? sh.tw.M0 : sh.tw.M1;
        double x = -ss;
        double ga[8], gb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) ga[u] = g[u];
        for (int j0 = 0; j0 < n - 1; j0 += 16) {  // steps beyond n - 2 run on zeros
#pragma unroll
            for (int u = 0; u < 8; ++u) gb[u] = g[j0 + 8 + u];
            loads_issued();
            twist_block(x, ga, ss, PIVMIN, X + j0, M + j0);
#pragma unroll
            for (int u = 0; u < 8; ++u) ga[u] = g[j0 + 16 + u];
            loads_issued();
            twist_block(x, gb, ss, PIVMIN, X + j0 + 8, M + j0 + 8);
        }
    }
    __syncthreads();
    {
        double gm = INFINITY;
        int gk = n;
        for (int k = tid; k < n; k += BS_PTS) {
            const double gv = fabs(sh.tw.X0[k] + sh.tw.X1[n - 1 - k] + ss);
            if (gv < gm) {
                gm = gv;
                gk = k;
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double og = __shfl_xor(gm, off, 64);
            const int ok = __shfl_xor(gk, off, 64);
            if (og < gm || (og == gm && ok < gk)) {
                gm = og;
                gk = ok;
            }
        }
        if (lane == 0) {
            sh.red[tid >> 6] = gm;
            sh.cnt[tid >> 6] = gk;
        }
        __syncthreads();
        if (tid == 0) {
            double bg = sh.red[0];
            int bk = sh.cnt[0];
            for (int w = 1; w < BS_PTS / 64; ++w)
                if (sh.red[w] < bg || (sh.red[w] == bg && sh.cnt[w] < bk)) {
                    bg = sh.red[w];
                    bk = sh.cnt[w];
                }
            sh.twr = bk < n ? bk : 0;
            sh.twg = bg;
        }
        __syncthreads();
    }
    const int r = sh.twr;
    if (tid < 2) {
        // lane 0: z_k = -l_k z_{k+1}, k = r - 1 .. 0; lane 1: z_{k+1} = -u_k z_k,
        // k = r .. n - 2 (u_k is M1[n - 2 - k]); multipliers read eight ahead
        const int len = tid == 0 ? r : n - 1 - r;
        const int len_max = r > n - 1 - r ? r : n - 1 - r;
        const double* src = tid == 0 ? sh.tw.M0 + (r - 1) : sh.tw.M1 + (n - 2 - r);
        const int step = tid == 0 ? -1 : 1;
        double* dst = z + r + step;
        if (tid == 0) z[r] = 1.0;
        double zp = 1.0;
        auto mul_at = [&](int q) { return q < len ? src[-q] : 0.0; };
        double ma[8], mb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) ma[u] = mul_at(u);
        for (int q0 = 0; q0 < len_max; q0 += 16) {
#pragma unroll
            for (int u = 0; u < 8; ++u) mb[u] = mul_at(q0 + 8 + u);
            loads_issued();
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q0 + u < len) {
                    zp = -ma[u] * zp;
                    dst[step * (q0 + u)] = zp;
                }
#pragma unroll
            for (int u = 0; u < 8; ++u) ma[u] = mul_at(q0 + 16 + u);
            loads_issued();
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (q0 + 8 + u < len) {
                    zp = -mb[u] * zp;
                    dst[step * (q0 + 8 + u)] = zp;
                }
        }
    }
    __syncthreads();
    {
        double zz = 0.0;
        bool fin = true;
        for (int k = tid; k < n; k += BS_PTS) {
            const double v = z[k];
            fin = fin && fabs(v) <= 1e150;
            zz += v * v;
        }
        for (int off = 32; off > 0; off >>= 1) zz += __shfl_xor(zz, off, 64);
        const int allfin = __syncthreads_and(fin ? 1 : 0);
        if (lane == 0) sh.red[tid >> 6] = zz;
        __syncthreads();
        double tot = 0.0;
#pragma unroll
        for (int w = 0; w < BS_PTS / 64; ++w) tot += sh.red[w];
        const double tol = 64.0 * n * U * bs;
        twisted_ok = allfin && sh.twg <= tol * sqrt(tot);
        __syncthreads();  // red is reused
    }
    }  // twisted factorisation
    if (!twisted_ok) {
    // ---- inverse iteration at +ss on the scaled T
    for (int j = tid - TG_OFF; j < n + TG_PAD; j += BS_PTS)
        z[j] = (j >= 0 && j < n) ? start_pm1((uint64_t)t * 4096ULL + (uint64_t)j) : 0.0;
    __syncthreads();
    for (int j = tid; j < n + TG_PAD; j += BS_PTS) {  // 1 / f_j (infinite for f_j = 0, then unused)
        const double fj = sh.f[j];
        double r = __builtin_amdgcn_rcp(fj);
        r = fma(r, fma(-fj, r, 1.0), r);
        sh.rl[j] = fma(r, fma(-fj, r, 1.0), r);
    }
    __syncthreads();
    const double tiny = bs * U + 1e-300;
    if (tid == 0) {
        double ddj = -ss, duj = sh.f[0];
        double fa[9], fb[9], ra[8], rb[8];
#pragma unroll
        for (int u = 0; u < 9; ++u) fa[u] = sh.f[u];
#pragma unroll
        for (int u = 0; u < 8; ++u) ra[u] = sh.rl[u];
        for (int j0 = 0; j0 < n - 1; j0 += 16) {
#pragma unroll
            for (int u = 0; u < 9; ++u) fb[u] = sh.f[j0 + 8 + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) rb[u] = sh.rl[j0 + 8 + u];
            loads_issued();
            lu_chain_block<0>(ddj, duj, fa, ra, ss, fac + j0, swp + j0);
#pragma unroll
            for (int u = 0; u < 9; ++u) fa[u] = sh.f[j0 + 16 + u];
#pragma unroll
            for (int u = 0; u < 8; ++u) ra[u] = sh.rl[j0 + 16 + u];
            loads_issued();
            lu_chain_block<8>(ddj, duj, fb, rb, ss, fac + j0, swp + j0);
        }
    }
    __syncthreads();
    // U's rows divided by the guarded diagonal; a multiplier that is not a
    // number of magnitude <= 1 (a zero or underflowing pivot in a row below
    // n - 1) sends the factorisation to the guarded form
    int bad = 0;
    for (int j = tid; j < n; j += BS_PTS) {
        const InvFac o = fac[j];
        const bool sw = swp[j];
        const double piv = sw ? sh.f[j] : o.rdd;
        const double pc = fabs(piv) < tiny ? (piv < 0.0 ? -tiny : tiny) : piv;
        const double rd = 1.0 / pc;
        const double odu = sw ? -ss : o.bdu;
        const double odu2 = sw ? sh.f[j + 1] : 0.0;
        fac[j].rdd = rd;
        fac[j].bdu = odu * rd;
        fac[j].bdu2 = odu2 * rd;
        if (j < n - 1 && !(fabs(o.dl) <= 1.0000001)) bad = 1;
    }
    if (__syncthreads_or(bad) && tid == 0) {
        double ddj = -ss, duj = sh.f[0];
        for (int j0 = 0; j0 < n - 1; j0 += 8) {
            double fw[9];
#pragma unroll
            for (int u = 0; u < 9; ++u) fw[u] = sh.f[j0 + u];
            lu_block<0>(ddj, duj, fw, ss, tiny, fac + j0, swp + j0);
        }
    }
    for (int it = 0; it < 2; ++it) {
        __syncthreads();
        double inv = 1.0;
        if (it > 0) {  // the previous solve's scale, 1 / max |z|
            double m = 0.0;
            for (int j = tid; j < n; j += BS_PTS) m = fmax(m, fabs(z[j]));
            for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
            if (lane == 0) sh.red[tid >> 6] = m;
            __syncthreads();
            m = 0.0;
#pragma unroll
            for (int w = 0; w < BS_PTS / 64; ++w) m = fmax(m, sh.red[w]);
            inv = m > 0.0 ? 1.0 / m : 0.0;
        }
        if (tid == 0) {
            // forward: z_j for j = 0 .. n - 2; the step at n - 1 (no
            // interchange, zero multiplier) stores the carried value as z_{n-1}
            double zj = z[0] * inv;
            {
                double za[8], la[8], zb[8], lb[8];
                unsigned char sa[8], sb[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    za[u] = z[u + 1];
                    la[u] = fac[u].dl;
                    sa[u] = swp[u];
                }
                for (int j0 = 0; j0 < n - 1; j0 += 16) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        zb[u] = z[j0 + 9 + u];
                        lb[u] = fac[j0 + 8 + u].dl;
                        sb[u] = swp[j0 + 8 + u];
                    }
                    loads_issued();
                    fwd_block(zj, za, la, sa, inv, z + j0);
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        za[u] = z[j0 + 17 + u];
                        la[u] = fac[j0 + 16 + u].dl;
                        sa[u] = swp[j0 + 16 + u];
                    }
                    loads_issued();
                    fwd_block(zj, zb, lb, sb, inv, z + j0 + 8);
                }
            }
            // back substitution from row n - 1 down; rows below 0 land in the
            // offset and are ignored
            double z1 = z[n - 1] * fac[n - 1].rdd, z2 = 0.0;
            z[n - 1] = z1;
            {
                InvFac ca[8], cb[8];
                double ya[8], yb[8];
                int k0 = n - 2;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    ca[u] = fac[k0 - u];
                    ya[u] = z[k0 - u];
                }
                for (; k0 >= 0; k0 -= 16) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        cb[u] = fac[k0 - 8 - u];
                        yb[u] = z[k0 - 8 - u];
                    }
                    loads_issued();
                    bwd_block(z1, z2, ca, ya, z + k0);
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        ca[u] = fac[k0 - 16 - u];
                        ya[u] = z[k0 - 16 - u];
                    }
                    loads_issued();
                    bwd_block(z1, z2, cb, yb, z + k0 - 8);
                }
            }
        }
    }
    }  // inverse iteration
    __syncthreads();
    // split and normalise each half to unit length
    double nu = 0.0, nv = 0.0;
    for (int i = tid; i < N; i += BS_PTS) {
        nv += z[2 * i] * z[2 * i];
        nu += z[2 * i + 1] * z[2 * i + 1];
    }
    for (int off = 32; off > 0; off >>= 1) {
        nu += __shfl_xor(nu, off, 64);
        nv += __shfl_xor(nv, off, 64);
    }
    if (lane == 0) sh.red[tid >> 6] = nu;
    __syncthreads();
    double su = 0.0;
#pragma unroll
    for (int w = 0; w < BS_PTS / 64; ++w) su += sh.red[w];
    __syncthreads();
    if (lane == 0) sh.red[tid >> 6] = nv;
    __syncthreads();
    double sv = 0.0;
#pragma unroll
    for (int w = 0; w < BS_PTS / 64; ++w) sv += sh.red[w];
    const double ru = su > 0.0 ? 1.0 / sqrt(su) : 0.0;
    const double rv = sv > 0.0 ? 1.0 / sqrt(sv) : 0.0;
    for (int i = tid; i < N; i += BS_PTS) {
        vbd[(size_t)i * ldv + t] = z[2 * i] * rv;
        ubd[(size_t)i * ldv + t] = z[2 * i + 1] * ru;
    }
}

// Back-transformation of the bidiagonal's singular vectors.
//   UB(:, t) <- H_0 ... H_{N-1} UB(:, t)   (left reflectors: row k of VL, unit at k)
//   VB(:, t) <- G_0 ... G_{N-2} VB(:, t)   (right reflectors: row k of VR, unit at k + 1)
// Blocks of WY_RB consecutive reflectors are applied, last block first, in the
// compact WY form H_k0 ... H_k1 = I - Y T Y^T (T upper triangular). The T of
// every block is built once by wy_t_kernel (one workgroup per block, from
// Y^T Y and the tau's); backtransform_kernel then applies the blocks with one
// wavefront per column, so a column needs WY_RB independent dot products per
// block instead of WY_RB dependent ones.
constexpr int WY_RB = 16;

// grid.x = block index over both sides (left blocks first); 256 threads.
__global__ __launch_bounds__(256) void wy_t_kernel(int N, const double* __restrict__ VL,
                                                   const double* __restrict__ tL,
                                                   const double* __restrict__ VR,
                                                   const double* __restrict__ tR,
                                                   double* __restrict__ Tout)
{
    __shared__ double Y[WY_RB][SVD_MAXN];
    __shared__ double YtY[WY_RB][WY_RB + 1];
    __shared__ double Tm[WY_RB][WY_RB + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblkL = (N + WY_RB - 1) / WY_RB;
    const bool left = (int)blockIdx.x < nblkL;
    const int blk = left ? blockIdx.x : blockIdx.x - nblkL;
    const double* Vh = left ? VL : VR;
    const double* tau = left ? tL : tR;
    const int nref = left ? N : N - 1, off = left ? 0 : 1;
    const int k0 = blk * WY_RB;
    const int cnt = (nref - k0) < WY_RB ? (nref - k0) : WY_RB;
    for (int q = 0; q < WY_RB; ++q)
        for (int i = tid; i < N; i += 256)
            Y[q][i] = (q < cnt && i >= k0 + q + off) ? Vh[(size_t)(k0 + q) * N + i] : 0.0;
    __syncthreads();
    // Y^T Y: pair (p, q), p < q, on wavefront (pair index % 4), lanes over i
    for (int base = wave * 8; base < WY_RB * WY_RB; base += 32) {
        double s[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int pq = base + u, p = pq / WY_RB, q = pq % WY_RB;
            double a = 0.0;
            if (p < q)
                for (int i = lane; i < N; i += 64) a += Y[p][i] * Y[q][i];
            s[u] = a;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] = wave_sum64(s[u]);
        if (lane == 0)
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int pq = base + u, p = pq / WY_RB, q = pq % WY_RB;
                if (p < q) YtY[p][q] = s[u];
            }
    }
    __syncthreads();
    // T (forward, columnwise): T[q][q] = tau_q, T[0:q, q] = -tau_q T[0:q, 0:q] Y^T y_q
    if (wave == 0) {
        for (int q = 0; q < WY_RB; ++q) {
            const double tq = q < cnt ? tau[k0 + q] : 0.0;
            double v = 0.0;
            if (lane < q) {
#pragma unroll
                for (int r = 0; r < WY_RB; ++r)
                    if (r >= lane && r < q) v += Tm[lane][r] * YtY[r][q];
                v *= -tq;
            }
            if (lane < WY_RB) Tm[lane][q] = lane < q ? v : (lane == q ? tq : 0.0);
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_wave_barrier();
        }
        for (int e = lane; e < WY_RB * WY_RB; e += 64)
            Tout[(size_t)blockIdx.x * WY_RB * WY_RB + e] = Tm[e / WY_RB][e % WY_RB];
    }
}

// grid (ceil(nv / 4), 2): blockIdx.y = 0 applies the left blocks to UB,
// 1 the right blocks to VB (the two sides are independent); one wavefront
// per column, the Y block of each step shared in LDS. The next step's Y block
// and T factor are loaded into registers while the current one is applied.
template <int MAXN, int R>
__global__ __launch_bounds__(256) void backtransform_kernel(
    int N, int nv, const double* __restrict__ VL, const double* __restrict__ VR,
    const double* __restrict__ Tall, double* __restrict__ UB, double* __restrict__ VB, int ld,
    int roff)
{
    __shared__ double Y[WY_RB][MAXN];
    __shared__ double Tm[WY_RB][WY_RB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = blockIdx.x * 4 + wave;
    const int side = blockIdx.y;
    const double* Vh = side == 0 ? VL : VR;
    double* X = side == 0 ? UB : VB;
    const int off = side == 0 ? 0 : roff;  // right reflector k starts at column k + roff
    const int nref = N - off;
    const int nblkL = (N + WY_RB - 1) / WY_RB;
    const int nsteps = (nref + WY_RB - 1) / WY_RB;
    double xr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = lane + 64 * r;
        xr[r] = (col < nv && i < N) ? X[(size_t)i * ld + col] : 0.0;
    }
    // steps: this side's blocks, last block first
    constexpr int PFN = MAXN <= 512 ? WY_RB * ((MAXN + 255) / 256) : 1;
    double pf[PFN];
    double tpf = 0.0;
    auto y_elem = [&](int blk, int q, int i) -> double {
        const int k0 = blk * WY_RB;
        const int cnt = (nref - k0) < WY_RB ? (nref - k0) : WY_RB;
        return (q < cnt && i < N && i >= k0 + q + off) ? Vh[(size_t)(k0 + q) * N + i] : 0.0;
    };
    auto t_index = [&](int blk) { return side == 0 ? blk : nblkL + blk; };
    auto prefetch = [&](int st) {
        const int blk = nsteps - 1 - st;
        if constexpr (MAXN <= 512) {
#pragma unroll
            for (int q = 0; q < WY_RB; ++q)
#pragma unroll
                for (int u = 0; u < PFN / WY_RB; ++u)
                    pf[q * (PFN / WY_RB) + u] = y_elem(blk, q, tid + 256 * u);
        }
        tpf = Tall[(size_t)t_index(blk) * WY_RB * WY_RB + tid];
    };
    prefetch(0);
    for (int st = 0; st < nsteps; ++st) {
        const int blk = nsteps - 1 - st;
        __syncthreads();  // the previous step's reads of Y and Tm are done
        if constexpr (MAXN <= 512) {
#pragma unroll
            for (int q = 0; q < WY_RB; ++q)
#pragma unroll
                for (int u = 0; u < PFN / WY_RB; ++u) {
                    const int i = tid + 256 * u;
                    if (i < MAXN) Y[q][i] = pf[q * (PFN / WY_RB) + u];
                }
        } else {
            for (int q = 0; q < WY_RB; ++q)
                for (int i = tid; i < N; i += 256) Y[q][i] = y_elem(blk, q, i);
        }
        Tm[tid >> 4][tid & 15] = tpf;
        __syncthreads();
        if (st + 1 < nsteps) prefetch(st + 1);
        // x <- x - Y (T (Y^T x))
        double yx[WY_RB];
#pragma unroll
        for (int q = 0; q < WY_RB; ++q) {
            double sm = 0.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = lane + 64 * r;
                if (i < N) sm += Y[q][i] * xr[r];
            }
            yx[q] = sm;
        }
#pragma unroll
        for (int q = 0; q < WY_RB; ++q) yx[q] = wave_sum64(yx[q]);
        double wv[WY_RB];
#pragma unroll
        for (int p = 0; p < WY_RB; ++p) {
            double sm = 0.0;
#pragma unroll
            for (int q = 0; q < WY_RB; ++q)
                if (q >= p) sm += Tm[p][q] * yx[q];
            wv[p] = sm;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = lane + 64 * r;
            if (i < N) {
                double sm = 0.0;
#pragma unroll
                for (int p = 0; p < WY_RB; ++p) sm += Y[p][i] * wv[p];
                xr[r] -= sm;
            }
        }
    }
    if (col < nv) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = lane + 64 * r;
            if (i < N) X[(size_t)i * ld + col] = xr[r];
        }
    }
}

// The same back-transformation with matrix cores for N <= MAXN: grid
// (ceil(nv / 16), 2), workgroup (c, side) holds columns 16 c .. 16 c + 15 of
// UB (side 0) or VB (side 1) in LDS and applies that side's blocks, last
// first: W = Y^T X by MFMA with the rows split over the four wavefronts (the
// partial products summed in LDS in wavefront order), W <- T W, then
// X <- X - Y W by MFMA over 16-row tiles. The next block's Y is loaded into
// registers while the current one is applied. MAXN = 256 (70 KB of LDS) or
// 512 (151 KB, for 256 < N <= 512).
constexpr int BT_MAXN = 512;
typedef double d4 __attribute__((ext_vector_type(4)));
template <int MAXN>
__global__ __launch_bounds__(256) void backtransform_mfma_kernel(
    int N, int nv, const double* __restrict__ VL, const double* __restrict__ VR,
    const double* __restrict__ Tall, double* __restrict__ UB, double* __restrict__ VB, int ld,
    int roff)
{
    __shared__ double Xs[MAXN][17];
    __shared__ double Ys[MAXN][17];
    __shared__ double Wp[4][16][17];
    __shared__ double Ws[16][17];
    __shared__ double WT[16][17];
    __shared__ double Tm[16][17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int side = blockIdx.y, c0 = 16 * blockIdx.x;
    const double* Vh = side == 0 ? VL : VR;
    double* X = side == 0 ? UB : VB;
    const int off = side == 0 ? 0 : roff;  // right reflector k starts at column k + roff
    const int nref = N - off;
    const int nblkL = (N + WY_RB - 1) / WY_RB;
    const int nsteps = (nref + WY_RB - 1) / WY_RB;
    for (int e = tid; e < N * 16; e += 256) {
        const int i = e >> 4, q = e & 15;
        Xs[i][q] = c0 + q < nv ? X[(size_t)i * ld + c0 + q] : 0.0;
    }
    // the Y block of a step as 16 x N (row q = reflector k0 + q), read along
    // the reflector rows; at most MAXN * 16 / 256 values per thread
    constexpr int PY = MAXN * 16 / 256;
    double py[PY];
    double pt = 0.0;
    auto prefetch = [&](int st) {
        const int blk = nsteps - 1 - st, k0 = blk * WY_RB;
        const int cnt = (nref - k0) < WY_RB ? (nref - k0) : WY_RB;
        if constexpr (MAXN > 256) {
            // launched for N > 256 only: element e + 256 is at most one
            // reflector row further on
            int q = tid / N, i = tid - q * N;
#pragma unroll
            for (int u = 0; u < PY; ++u) {
                const int e = tid + 256 * u;
                py[u] = (e < 16 * N && q < cnt && i >= k0 + q + off) ? Vh[(size_t)(k0 + q) * N + i]
                                                                      : 0.0;
                i += 256;
                if (i >= N) {
                    i -= N;
                    ++q;
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < PY; ++u) {
                const int e = tid + 256 * u, q = e / N, i = e - q * N;
                py[u] = (e < 16 * N && q < cnt && i >= k0 + q + off) ? Vh[(size_t)(k0 + q) * N + i]
                                                                      : 0.0;
            }
        }
        pt = Tall[(size_t)(side == 0 ? blk : nblkL + blk) * WY_RB * WY_RB + tid];
    };
    prefetch(0);
    for (int st = 0; st < nsteps; ++st) {
        const int k0 = (nsteps - 1 - st) * WY_RB;
        __syncthreads();  // the previous step is done with Ys, Tm, WT and Xs
#pragma unroll
        for (int u = 0; u < PY; ++u) {
            const int e = tid + 256 * u, q = e / N, i = e - q * N;
            if (e < 16 * N) Ys[i][q] = py[u];
        }
        Tm[tid >> 4][tid & 15] = pt;
        __syncthreads();
        if (st + 1 < nsteps) prefetch(st + 1);
        // W = Y^T X over rows >= k0, four rows per MFMA step, interleaved by wavefront
        {
            d4 acc = d4{0.0, 0.0, 0.0, 0.0};
            for (int kb = k0 + 4 * wave; kb < N; kb += 16) {
                const int i = kb + (lane >> 4);
                const double a = i < N ? Ys[i][lane & 15] : 0.0;
                const double b = i < N ? Xs[i][lane & 15] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) Wp[wave][(lane >> 4) + 4 * r][lane & 15] = acc[r];
        }
        __syncthreads();
        {
            const int q = tid >> 4, col = tid & 15;
            Ws[q][col] = ((Wp[0][q][col] + Wp[1][q][col]) + Wp[2][q][col]) + Wp[3][q][col];
        }
        __syncthreads();
        {
            const int p = tid >> 4, col = tid & 15;
            double sm = 0.0;
#pragma unroll
            for (int q = 0; q < WY_RB; ++q)
                if (q >= p) sm += Tm[p][q] * Ws[q][col];
            WT[p][col] = sm;
        }
        __syncthreads();
        // X <- X - Y (T W) over 16-row tiles from k0 (rows above k0 + q + off
        // have Y = 0)
        for (int rt = k0 / 16 + wave; 16 * rt < N; rt += 4) {
            d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int i = 16 * rt + (lane & 15);
                const double a = i < N ? Ys[i][4 * kk + (lane >> 4)] : 0.0;
                const double b = WT[4 * kk + (lane >> 4)][lane & 15];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * rt + (lane >> 4) + 4 * r;
                if (row < N) Xs[row][lane & 15] -= acc[r];
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < N * 16; e += 256) {
        const int i = e >> 4, q = e & 15;
        if (c0 + q < nv) X[(size_t)i * ld + c0 + q] = Xs[i][q];
    }
}

// The matrix-core back-transformation for N <= BT_MAXN, the smaller LDS
// form up to 256 (two workgroups per CU).
void backtransform_mfma(int N, int nv, const double* VL, const double* VR, const double* Tall,
                        double* UB, double* VB, int ld, int roff, hipStream_t s)
{
    const dim3 grid((nv + 15) / 16, 2);
    if (N <= 256)
        hipLaunchKernelGGL((backtransform_mfma_kernel<256>), grid, dim3(256), 0, s, N, nv, VL, VR,
                           Tall, UB, VB, ld, roff);
    else
        hipLaunchKernelGGL((backtransform_mfma_kernel<BT_MAXN>), grid, dim3(256), 0, s, N, nv, VL,
                           VR, Tall, UB, VB, ld, roff);
}

// QL = QR = I (N x N)
__global__ void eye2_kernel(int N, double* __restrict__ QL, double* __restrict__ QR)
{
    const size_t total = (size_t)N * N;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const double v = (e / N == e % N) ? 1.0 : 0.0;
        QL[e] = v;
        QR[e] = v;
    }
}

// Sign convention of the singular pairs: the first largest-magnitude entry of
// the left vector positive (u and v of a pair flip together). One wavefront
// per column.
__global__ __launch_bounds__(256) void sign_fix_kernel(int N, int nv, double* __restrict__ UB,
                                                       double* __restrict__ VB, int ld)
{
    const int lane = threadIdx.x & 63;
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (col >= nv) return;  // uniform per wavefront
    double vmax = -1.0, xv = 0.0;
    int imax = 0;
    for (int i = lane; i < N; i += 64) {
        const double x = UB[(size_t)i * ld + col];
        if (fabs(x) > vmax) {
            vmax = fabs(x);
            imax = i;
            xv = x;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(vmax, o, 64);
        const int oi = __shfl_xor(imax, o, 64);
        const double ox = __shfl_xor(xv, o, 64);
        if (ov > vmax || (ov == vmax && oi < imax)) {
            vmax = ov;
            imax = oi;
            xv = ox;
        }
    }
    if (xv < 0.0) {
        for (int i = lane; i < N; i += 64) {
            UB[(size_t)i * ld + col] = -UB[(size_t)i * ld + col];
            VB[(size_t)i * ld + col] = -VB[(size_t)i * ld + col];
        }
    }
}

}  // namespace

bool small_svd_gk_supported(int N) { return N >= 2 && N <= SVD_MAXN; }

size_t small_svd_gk_scratch_elems(int N)
{
    // d, e, tauL, tauR, the reflector vectors VL, VR, for the cooperative
    // bidiagonalisation the published column, partials and barrier counter,
    // the T factors, and beyond GK_MAXN the trailing GK_MAXN x GK_MAXN matrix
    // the cooperative steps hand to the one-workgroup kernel
    // (up to BT_MAXN also Q_L, Q_R, the bidiagonal's vectors and the
    // partials of the products that apply Q_L, Q_R to them)
    const size_t P = (N + 31) / 32;
    const size_t nblk = (N + WY_RB - 1) / WY_RB + (N - 1 + WY_RB - 1) / WY_RB;
    return 4 * (size_t)N + 2 * (size_t)N * N + 2 * (size_t)N + 2 * P + 2 * P * N + 8 +
           nblk * WY_RB * WY_RB + (N > GK_MAXN ? (size_t)GK_MAXN * GK_MAXN : 0) +
           (N <= BT_MAXN ? 4 * (size_t)N * N + gemm_partial_elems(N, N, N) + 1 : 0);
}

// Outputs: S[0..nv), UB, VB (N x N, ld N) with their first nv columns set.
void small_svd_gk(Timer* tm, int N, int nv, const double* B, int ldb, double* UB, double* S,
                  double* VB, double* scratch, int* err, hipStream_t s, hipStream_t s2,
                  hipEvent_t ev_a, hipEvent_t ev_b)
{
    BLWS_REQUIRE(small_svd_gk_supported(N) && nv >= 1 && nv <= N, BLWS_EUNSUPPORTED,
                 "small_svd_gk: size out of range");
    double* d = scratch;
    double* e = d + N;
    double* tL = e + N;
    double* tR = tL + N;
    double* VL = tR + N;
    double* VR = VL + (size_t)N * N;
    static const char* const coop_fam[8] = {"gk_bidiag_coop_q20", "gk_bidiag_coop_q24",
                                            "gk_bidiag_coop_q28", "gk_bidiag_coop_q32",
                                            "gk_bidiag_coop_q40", "gk_bidiag_coop_q48",
                                            "gk_bidiag_coop_q56", "gk_bidiag_coop_q64"};
    static const char* const one_fam[7] = {"gk_bidiag_p1", "gk_bidiag_p2", "gk_bidiag_p3",
                                           "gk_bidiag_p4", "gk_bidiag_p5", "gk_bidiag_p6",
                                           "gk_bidiag_p7"};
    // bidiagonalisation flops: 4 N^3 - 4 N^3 / 3 (Householder, both sides)
    const double bd_flops = 8.0 / 3.0 * N * (double)N * N;
    if (N > GK_MAXN) {
        // The first N - GK_MAXN steps across ceil(N / 32) co-resident
        // workgroups; the trailing GK_MAXN x GK_MAXN matrix they leave is
        // then bidiagonalised by the one-workgroup kernel (its steps cost a
        // workgroup barrier, not a device-wide one), writing its reflectors
        // into the trailing part of VL and VR.
        const int kstop = N - GK_MAXN;
        const int nblk_t = (N + WY_RB - 1) / WY_RB + (N - 1 + WY_RB - 1) / WY_RB;
        const int Pt = (N + 31) / 32;
        double* Tt = VR + (size_t)N * N + 2 * (size_t)N + 2 * (size_t)Pt + 2 * (size_t)Pt * N + 8 +
                     (size_t)nblk_t * WY_RB * WY_RB;
        {
        const int NQc = (N + 15) / 16;
        const int qi = NQc <= 20 ? 0 : NQc <= 24 ? 1 : NQc <= 28 ? 2 : NQc <= 32 ? 3
                     : NQc <= 40 ? 4 : NQc <= 48 ? 5 : NQc <= 56 ? 6 : 7;
        TimedLaunch tl(tm, coop_fam[qi], s, bd_flops, 16.0 * N * N);
        const int P = (N + 31) / 32;
        CoopBuf cb;
        cb.colpub = VR + (size_t)N * N;
        cb.nrm = cb.colpub + 2 * (size_t)N;
        cb.part = cb.nrm + 2 * (size_t)P;
        cb.ctr = (unsigned*)(cb.part + 2 * (size_t)P * N);
        cb.err = err;
        zero_bytes(cb.ctr, sizeof(unsigned), s);
        void* args[] = {(void*)&N,  (void*)&B,  (void*)&ldb, (void*)&d,     (void*)&e,
                        (void*)&VL, (void*)&tL, (void*)&VR,  (void*)&tR,    (void*)&cb,
                        (void*)&kstop, (void*)&Tt};
        const void* fn = nullptr;
        const int NQ = (N + 15) / 16;
        if (NQ <= 20) fn = (const void*)gk_bidiag_coop_kernel<20>;
        else if (NQ <= 24) fn = (const void*)gk_bidiag_coop_kernel<24>;
        else if (NQ <= 28) fn = (const void*)gk_bidiag_coop_kernel<28>;
        else if (NQ <= 32) fn = (const void*)gk_bidiag_coop_kernel<32>;
        else if (NQ <= 40) fn = (const void*)gk_bidiag_coop_kernel<40>;
        else if (NQ <= 48) fn = (const void*)gk_bidiag_coop_kernel<48>;
        else if (NQ <= 56) fn = (const void*)gk_bidiag_coop_kernel<56>;
        else fn = (const void*)gk_bidiag_coop_kernel<64>;
        HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(P), dim3(512), args, 0, s));
        }
        {
            const int nt = GK_MAXN;
            TimedLaunch tl(tm, one_fam[6], s, 8.0 / 3.0 * nt * (double)nt * nt, 16.0 * nt * nt);
            const size_t off = (size_t)kstop * N + kstop;
            hipLaunchKernelGGL((gk_bidiag_kernel<7>), dim3(1), dim3(512), 0, s, nt, Tt, nt,
                               d + kstop, e + kstop, VL + off, tL + kstop, VR + off, tR + kstop, N);
        }
    } else {
        const int NP = (N + 31) / 32;
        TimedLaunch tl(tm, one_fam[NP - 1], s, bd_flops, 16.0 * N * N);
#define BLWS_GK_CASE(P)                                                                      \
    case P:                                                                                  \
        hipLaunchKernelGGL((gk_bidiag_kernel<P>), dim3(1), dim3(512), 0, s, N, B, ldb, d, e, VL, \
                           tL, VR, tR, N);                                                   \
        break;
        switch (NP) {
            BLWS_GK_CASE(1)
            BLWS_GK_CASE(2)
            BLWS_GK_CASE(3)
            BLWS_GK_CASE(4)
            BLWS_GK_CASE(5)
            BLWS_GK_CASE(6)
            default:
                BLWS_GK_CASE(7)
        }
#undef BLWS_GK_CASE
    }
    // The T factors of the reflector blocks need only the reflectors: with a
    // second stream they are built there while the values and vectors of the
    // bidiagonal are found.
    const int nblk = (N + WY_RB - 1) / WY_RB + (N - 1 + WY_RB - 1) / WY_RB;
    double* Tall = VR + (size_t)N * N + 2 * (size_t)N + 2 * (size_t)((N + 31) / 32) +
                   2 * (size_t)((N + 31) / 32) * N + 8;
    const bool two = s2 != nullptr && ev_a != nullptr && ev_b != nullptr;
    if (two && N <= BT_MAXN) {
        // Q_L = H_0 .. H_{N-1} and Q_R formed on the second stream (the
        // reflectors applied to the identity) while the values and the
        // bidiagonal's vectors are found; the back-transformation is then
        // two products UB = Q_L Ubd, VB = Q_R Vbd instead of a chain of
        // reflector blocks after the vectors.
        double* QL = Tall + (size_t)nblk * WY_RB * WY_RB +
                     (N > GK_MAXN ? (size_t)GK_MAXN * GK_MAXN : 0);
        double* QR = QL + (size_t)N * N;
        double* Ubd = QR + (size_t)N * N;
        double* Vbd = Ubd + (size_t)N * N;
        double* gpart = Vbd + (size_t)N * N;
        const size_t gpe = gemm_partial_elems(N, N, N);
        HIP_TRY(hipEventRecord(ev_a, s));
        HIP_TRY(hipStreamWaitEvent(s2, ev_a, 0));
        {
            TimedLaunch tl(tm, "wy_t", s2, 0.0, 0.0);
            hipLaunchKernelGGL(wy_t_kernel, dim3(nblk), dim3(256), 0, s2, N, VL, tL, VR, tR, Tall);
        }
        {
            TimedLaunch tl(tm, "gk_form_q", s2, 8.0 * N * (double)N * N, 0.0);
            hipLaunchKernelGGL(eye2_kernel, dim3((N * N + 255) / 256), dim3(256), 0, s2, N, QL, QR);
            backtransform_mfma(N, N, VL, VR, Tall, QL, QR, N, 1, s2);
        }
        HIP_TRY(hipEventRecord(ev_b, s2));
        {
            TimedLaunch tl(tm, "tgk_solve", s, 0.0, 0.0);
            hipLaunchKernelGGL(tgk_solve_kernel, dim3(nv), dim3(BS_PTS), 0, s, N, d, e, S, Ubd, Vbd,
                               N);
        }
        HIP_TRY(hipStreamWaitEvent(s, ev_b, 0));
        {
            TimedLaunch tl(tm, "gk_backtransform", s, 4.0 * N * (double)N * nv, 0.0);
            gemm<double, double, double>(tm, "gemm_ts", false, N, nv, N, 1.0, QL, N, Ubd, N, 0.0,
                                         (const double*)nullptr, 0, UB, N, gpart, gpe, s);
            gemm<double, double, double>(tm, "gemm_ts", false, N, nv, N, 1.0, QR, N, Vbd, N, 0.0,
                                         (const double*)nullptr, 0, VB, N, gpart, gpe, s);
            hipLaunchKernelGGL(sign_fix_kernel, dim3((nv + 3) / 4), dim3(256), 0, s, N, nv, UB, VB,
                               N);
        }
        return;
    }
    if (two) {
        HIP_TRY(hipEventRecord(ev_a, s));
        HIP_TRY(hipStreamWaitEvent(s2, ev_a, 0));
        TimedLaunch tl(tm, "wy_t", s2, 0.0, 0.0);
        hipLaunchKernelGGL(wy_t_kernel, dim3(nblk), dim3(256), 0, s2, N, VL, tL, VR, tR, Tall);
        HIP_TRY(hipEventRecord(ev_b, s2));
    }
    {
        TimedLaunch tl(tm, "tgk_solve", s, 0.0, 0.0);
        hipLaunchKernelGGL(tgk_solve_kernel, dim3(nv), dim3(BS_PTS), 0, s, N, d, e, S, UB, VB, N);
    }
    if (two) {
        HIP_TRY(hipStreamWaitEvent(s, ev_b, 0));
    } else {
        TimedLaunch tl(tm, "wy_t", s, 0.0, 0.0);
        hipLaunchKernelGGL(wy_t_kernel, dim3(nblk), dim3(256), 0, s, N, VL, tL, VR, tR, Tall);
    }
    {
        TimedLaunch tl(tm, "gk_backtransform", s, 4.0 * N * (double)N * nv, 0.0);
        const int blocks = (nv + 3) / 4;
        if (N <= BT_MAXN)
            backtransform_mfma(N, nv, VL, VR, Tall, UB, VB, N, 1, s);
        else
            hipLaunchKernelGGL((backtransform_kernel<SVD_MAXN, 16>), dim3(blocks, 2), dim3(256), 0,
                               s, N, nv, VL, VR, Tall, UB, VB, N, 1);
        hipLaunchKernelGGL(sign_fix_kernel, dim3(blocks), dim3(256), 0, s, N, nv, UB, VB, N);
    }
}

}  // namespace blws

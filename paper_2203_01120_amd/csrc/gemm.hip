// Complex FP64 contractions on the matrix cores (v_mfma_f64_16x16x4f64).
//
// Two shapes cover the nonlocal pseudopotential term and the projector onto
// the empty manifold of every (side, k) block:
//   k_gemm_cn:     C[m][n] = sum_k conj(A[m][k]) B[n][k]   (small C, long K;
//                  split over K, partials summed by k_reduce_parts)
//   k_gemm_update: Y[n][k] = os * (Y[n][k] + cs * sum_m C[m][n] A[m][k])
//                  (long output rows, short inner dimension)
// Nonlocal term (Eq. H0_k_plus_q, V_NL with the 2x2 spin D matrix):
//   B = beta^dag x,  W_i = sum_j D_ij B_j,  phi += beta W.
// Projector (Eqs. P_minus_q2 / P_plus_q2):
//   S = O^dag phi,  phi <- sg (phi - O S), sg = -1 on the lower row of L.
// Complex products use four real MFMAs (re*re, im*im, re*im, im*re).
//
// Lane layout of the 16x16x4 MFMAs for wave lane l (measured on gfx950):
// A[l%16][l/16], B[l/16][l%16]; accumulator element v holds
//   FP64 (v_mfma_f64_16x16x4f64): D[4*v + l/16][l%16]
//   FP32 (v_mfma_f32_16x16x4f32): D[4*(l/16) + v][l%16]
// The FP32 variants (single-precision bulk path) round the FP64 operands to
// FP32 on load and accumulate in FP32; partial sums and outputs stay FP64.
#include "tm_internal.h"

namespace tml {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline v4d mfma(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma(float a, float b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }

template <class R>
struct MF;
template <>
struct MF<double> {
    using V = v4d;
    // output row of accumulator element v for lane group kk = l / 16
    __device__ static int row(int v, int kk) { return 4 * v + kk; }
};
template <>
struct MF<float> {
    using V = v4f;
    __device__ static int row(int v, int kk) { return 4 * kk + v; }
};

// Batches of several right-hand sides: batch b uses the A of b % amod (its
// side and k point); B, C, Y and the partials are per b.
struct GemmCN {
    const double2* const* A_tab;  // per batch b % amod (or null -> A_base + b*a_bstride)
    int amod;
    const double2* A_base;
    long long a_bstride;
    int lda;
    const double2* B_base;        // per batch B_base + b*b_bstride
    long long b_bstride;
    int ldb;
    int M, Nn, K, kchunk, ksplit, nt;
    double2* part;                // [b][ks][M][Nn]
};

__device__ double2 g_zero2;  // zero-initialised, never written
// a complex value as a native vector, and a pointer to one in global memory
// (operands reached through pointer tables would otherwise be read with flat
// loads, which make every wait a wait for all loads, LDS included)
typedef double __attribute__((ext_vector_type(2))) DVec2;
typedef const DVec2 __attribute__((address_space(1))) GlobalD2;

// *p as a global-memory load
__device__ __forceinline__ double2 gload(const double2* p) {
    const DVec2 v = *(const GlobalD2*)p;
    return cmk(v.x, v.y);
}

template <class R>
__global__ void __launch_bounds__(64) k_gemm_cn(GemmCN g) {
    const int b = blockIdx.z, ks = blockIdx.y;
    const int tile = blockIdx.x;
    const int m0 = (tile / g.nt) * 16, n0 = (tile % g.nt) * 16;
    const int l = threadIdx.x, i = l & 15, kk = l >> 4;
    const double2* A = g.A_tab ? g.A_tab[b % g.amod] : g.A_base + (long long)b * g.a_bstride;
    const double2* B = g.B_base + (long long)b * g.b_bstride;
    const int kbeg = ks * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);
    typename MF<R>::V cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
    const bool arow = (m0 + i) < g.M, brow = (n0 + i) < g.Nn;
    const double2* Ap = A + (long long)(m0 + i) * g.lda;
    const double2* Bp = B + (long long)(n0 + i) * g.ldb;
    // KU steps' loads in flight together (global loads, an element outside
    // the operands read from a zero); the products run in step order
    constexpr int KU = 4;
    for (int k = kbeg; k < kend; k += 4 * KU) {
        double2 a[KU], bv[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int kx = k + 4 * u + kk;
            a[u] = gload((arow && kx < kend) ? Ap + kx : &g_zero2);
            bv[u] = gload((brow && kx < kend) ? Bp + kx : &g_zero2);
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            if (k + 4 * u < kend) {
                const R ax = (R)a[u].x, ay = (R)a[u].y, bx = (R)bv[u].x, by = (R)bv[u].y;
                cr = mfma(ax, bx, cr);
                cr = mfma(ay, by, cr);
                ci = mfma(ax, by, ci);
                ci = mfma(-ay, bx, ci);
            }
        }
    }
    double2* out = g.part + ((long long)b * g.ksplit + ks) * g.M * g.Nn;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        int m = m0 + MF<R>::row(v, kk), n = n0 + i;
        if (m < g.M && n < g.Nn) out[(long long)m * g.Nn + n] = cmk((double)cr[v], (double)ci[v]);
    }
}

// Small contractions (a few output tiles, K of at most kSmallK): one block
// per (tile, batch); its waves take interleaved K slices of 4 and their
// 16 x 16 accumulators are added in wave order through LDS, so the result
// goes straight to `out` with no partial buffer and no second launch.
constexpr int kSmallWaves = 16;
constexpr int kSmallK = 4096;

template <class R>
__global__ void __launch_bounds__(64 * kSmallWaves) k_gemm_cn_small(GemmCN g, double2* out) {
    __shared__ double2 red[kSmallWaves][256];
    const int b = blockIdx.y, tile = blockIdx.x;
    const int m0 = (tile / g.nt) * 16, n0 = (tile % g.nt) * 16;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, i = l & 15, kk = l >> 4;
    const double2* A = g.A_tab ? g.A_tab[b % g.amod] : g.A_base + (long long)b * g.a_bstride;
    const double2* B = g.B_base + (long long)b * g.b_bstride;
    typename MF<R>::V cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
    const bool arow = (m0 + i) < g.M, brow = (n0 + i) < g.Nn;
    const double2* Ap = A + (long long)(m0 + i) * g.lda;
    const double2* Bp = B + (long long)(n0 + i) * g.ldb;
    // KU slices a wave's loads are in flight together
    constexpr int KU = 4, KS = 4 * kSmallWaves;
    for (int k0 = 4 * w; k0 < g.K; k0 += KU * KS) {
        double2 a[KU], bv[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int kx = k0 + u * KS + kk;
            a[u] = gload((arow && kx < g.K) ? Ap + kx : &g_zero2);
            bv[u] = gload((brow && kx < g.K) ? Bp + kx : &g_zero2);
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const R ax = (R)a[u].x, ay = (R)a[u].y, bx = (R)bv[u].x, by = (R)bv[u].y;
            cr = mfma(ax, bx, cr);
            cr = mfma(ay, by, cr);
            ci = mfma(ax, by, ci);
            ci = mfma(-ay, bx, ci);
        }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) red[w][MF<R>::row(v, kk) * 16 + i] = cmk((double)cr[v], (double)ci[v]);
    __syncthreads();
    if (threadIdx.x < 256) {
        const int m = m0 + threadIdx.x / 16, n = n0 + (threadIdx.x & 15);
        double2 sum = red[0][threadIdx.x];
#pragma unroll
        for (int v = 1; v < kSmallWaves; ++v) sum = cadd(sum, red[v][threadIdx.x]);
        if (m < g.M && n < g.Nn) out[((long long)b * g.M + m) * g.Nn + n] = sum;
    }
}

// The same contraction with both operands of a K-chunk staged in LDS: one
// block per (batch, K split) computes every 16x16 output tile from LDS (waves
// take tiles in turn), so each operand element is read from memory once
// instead of once per output tile.  The next chunk's loads are issued before
// the current chunk's products, so memory latency hides behind the MFMAs.
// Needs M, Nn <= 16 * kMaxTiles1D.
constexpr int kCnThreads = 512;
constexpr int kCnChunk = 16;          // K values per LDS chunk
constexpr int kMaxTiles1D = 14;       // M, Nn up to 224
constexpr int kCnTilesPerWave = 7;    // (mt * nt) / 8 waves, at most
constexpr int kCnMaxTilesSum = 16;   // mt + nt, at most
constexpr int kCnStage = kCnMaxTilesSum * 16 * kCnChunk / kCnThreads;  // staged elements per thread

template <class R>
struct LdsC {
    R re, im;
};

template <class R>
__global__ void __launch_bounds__(kCnThreads) k_gemm_cn_lds(GemmCN g, int mt) {
    extern __shared__ double lds_raw[];
    constexpr int LS = kCnChunk + 1;  // padded row
    const int Mp = mt * 16, Np = g.nt * 16;
    LdsC<R>* As = reinterpret_cast<LdsC<R>*>(lds_raw);
    LdsC<R>* Bs = As + Mp * LS;
    const int b = blockIdx.y, ks = blockIdx.x;
    const double2* A = g.A_tab ? g.A_tab[b % g.amod] : g.A_base + (long long)b * g.a_bstride;
    const double2* B = g.B_base + (long long)b * g.b_bstride;
    const int kbeg = ks * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, i = l & 15, kk = l >> 4;
    const int ntiles = mt * g.nt;
    typename MF<R>::V cr[kCnTilesPerWave], ci[kCnTilesPerWave];
#pragma unroll
    for (int t = 0; t < kCnTilesPerWave; ++t) {
        cr[t] = typename MF<R>::V{0, 0, 0, 0};
        ci[t] = typename MF<R>::V{0, 0, 0, 0};
    }
    // A[0..Mp)[k0..k0+16) and B[0..Np)[k0..k0+16) of one chunk, kCnStage
    // elements per thread; rows past M / Nn and k past the range read as zero
    const int nst = (Mp + Np) * kCnChunk;
    double2 stage[kCnStage];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int j = 0; j < kCnStage; ++j) {
            const int e = threadIdx.x + j * kCnThreads;
            const int row = e / kCnChunk, kx = k0 + (e - row * kCnChunk);
            const bool isA = row < Mp;
            const int r = isA ? row : row - Mp;
            // unconditional global loads (an element outside the operands is
            // read from a zero in device memory): no branch around a load, and
            // no flat load, whose pending count would also hold up the LDS reads
            // of the products below
            const bool in = e < nst && kx < kend && (isA ? r < g.M : r < g.Nn);
            stage[j] = gload(!in ? &g_zero2 : isA ? A + (long long)r * g.lda + kx : B + (long long)r * g.ldb + kx);
        }
    };
    fetch(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += kCnChunk) {
#pragma unroll
        for (int j = 0; j < kCnStage; ++j) {
            const int e = threadIdx.x + j * kCnThreads;
            if (e < nst) {
                const int row = e / kCnChunk;
                const bool isA = row < Mp;
                const int r = isA ? row : row - Mp;
                LdsC<R>* dst = isA ? As : Bs;
                dst[r * LS + (e - row * kCnChunk)] = LdsC<R>{(R)stage[j].x, (R)stage[j].y};
            }
        }
        __syncthreads();
        if (k0 + kCnChunk < kend) fetch(k0 + kCnChunk);  // in flight during the products below
#pragma unroll
        for (int t = 0; t < kCnTilesPerWave; ++t) {
            const int tile = w + 8 * t;
            if (tile < ntiles) {
                const int m0 = (tile / g.nt) * 16, n0 = (tile % g.nt) * 16;
#pragma unroll
                for (int k4 = 0; k4 < kCnChunk; k4 += 4) {
                    const LdsC<R> a = As[(m0 + i) * LS + k4 + kk];
                    const LdsC<R> bv = Bs[(n0 + i) * LS + k4 + kk];
                    cr[t] = mfma(a.re, bv.re, cr[t]);
                    cr[t] = mfma(a.im, bv.im, cr[t]);
                    ci[t] = mfma(a.re, bv.im, ci[t]);
                    ci[t] = mfma(-a.im, bv.re, ci[t]);
                }
            }
        }
        __syncthreads();
    }
    double2* out = g.part + ((long long)b * g.ksplit + ks) * g.M * g.Nn;
#pragma unroll
    for (int t = 0; t < kCnTilesPerWave; ++t) {
        const int tile = w + 8 * t;
        if (tile < ntiles) {
            const int m0 = (tile / g.nt) * 16, n0 = (tile % g.nt) * 16;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + MF<R>::row(v, kk), n = n0 + i;
                if (m < g.M && n < g.Nn) out[(long long)m * g.Nn + n] = cmk((double)cr[t][v], (double)ci[t][v]);
            }
        }
    }
}

__global__ void k_reduce_parts(const double2* part, double2* out, int ksplit, long long mn, int nbatch) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= mn * nbatch) return;
    long long b = idx / mn, e = idx - b * mn;
    double2 s = cmk(0.0, 0.0);
    for (int k = 0; k < ksplit; ++k) s = cadd(s, part[(b * ksplit + k) * mn + e]);
    out[idx] = s;
}

struct GemmUpd {
    double2* Y_base;
    long long y_bstride;
    int ldy;
    const double2* C_base;        // per batch C_base + b*c_bstride, [Minner][Nout]
    long long c_bstride;
    int ldc;
    const double2* const* A_tab;  // per batch b % tmod
    int tmod;
    int lda;
    int Nout, K, Minner;
    double cs;
    double os_x, os_y;            // output sign of side 0 / side 1 batches
    int nk;
};

// One block per 16 rows k of A and batch; its waves take the 16-wide tiles of
// n, so that the A rows are fetched once (into one XCD's L2 and the CU's L1)
// for all of them.  U = 0: one step of 4 at a time (loads, then products);
// U > 0: the inner dimension goes in groups of U steps, two register groups
// in turn, the loads of the next group issued before the products of the
// current one and the outputs' current values read at the start, so that a
// wave does not wait a full memory latency per step (more registers, fewer
// waves per CU).  The products run in the same order in every variant, so the
// results are identical; the autotuner picks per shape.
template <class R, int U>
__global__ void __launch_bounds__(1024) k_gemm_update(GemmUpd g) {
    const int b = blockIdx.z;
    const int n0 = (threadIdx.x >> 6) * 16, k0 = blockIdx.y * 16;
    const int l = threadIdx.x & 63, i = l & 15, kk = l >> 4;
    const int bt = b % (2 * g.nk);  // side and k point (the output sign)
    const double2* A = g.A_tab[b % g.tmod];
    const double2* C = g.C_base + (long long)b * g.c_bstride;
    double2* Y = g.Y_base + (long long)b * g.y_bstride;
    typename MF<R>::V dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
    const bool ncol = (n0 + i) < g.Nout, kcol = (k0 + i) < g.K;
    const double os = bt < g.nk ? g.os_x : g.os_y;
    if constexpr (U == 0) {
        for (int m = 0; m < g.Minner; m += 4) {
            int mm = m + kk;
            double2 c = (mm < g.Minner && ncol) ? C[(long long)mm * g.ldc + n0 + i] : cmk(0.0, 0.0);
            double2 a = (mm < g.Minner && kcol) ? A[(long long)mm * g.lda + k0 + i] : cmk(0.0, 0.0);
            const R cx = (R)c.x, cy = (R)c.y, ax = (R)a.x, ay = (R)a.y;
            dr = mfma(cx, ax, dr);
            dr = mfma(-cy, ay, dr);
            di = mfma(cx, ay, di);
            di = mfma(cy, ax, di);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int n = n0 + MF<R>::row(v, kk), k = k0 + i;
            if (n < g.Nout && k < g.K) {
                double2* y = Y + (long long)n * g.ldy + k;
                double2 cur = *y;
                *y = cmk(os * (cur.x + g.cs * (double)dr[v]), os * (cur.y + g.cs * (double)di[v]));
            }
        }
    } else {
        // every load is issued unconditionally (an element outside the
        // operands is read from a zero in device memory), so that no branch
        // separates the loads from their uses and a group's products wait only
        // for that group's loads
        auto load = [&](int m, double2* c, double2* a) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int mm = m + 4 * u + kk;
                const double2* pc = (mm < g.Minner && ncol) ? C + (long long)mm * g.ldc + n0 + i : &g_zero2;
                const double2* pa = (mm < g.Minner && kcol) ? A + (long long)mm * g.lda + k0 + i : &g_zero2;
                c[u] = gload(pc);
                a[u] = gload(pa);
            }
        };
        auto products = [&](int m, const double2* c, const double2* a) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (m + 4 * u < g.Minner) {
                    const R cx = (R)c[u].x, cy = (R)c[u].y, ax = (R)a[u].x, ay = (R)a[u].y;
                    dr = mfma(cx, ax, dr);
                    dr = mfma(-cy, ay, dr);
                    di = mfma(cx, ay, di);
                    di = mfma(cy, ax, di);
                }
            }
        };
        DVec2 ycur[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int n = n0 + MF<R>::row(v, kk), k = k0 + i;
            const double2* py = (n < g.Nout && k < g.K) ? Y + (long long)n * g.ldy + k : &g_zero2;
            ycur[v] = *(const GlobalD2*)py;
        }
        // two register groups in turn (no copies, which would wait for the loads)
        double2 c0[U], a0[U], c1[U], a1[U];
        load(0, c0, a0);
        for (int m = 0; m < g.Minner; m += 8 * U) {
            load(m + 4 * U, c1, a1);  // in flight during the products below (past the end: zeros, unused)
            products(m, c0, a0);
            load(m + 8 * U, c0, a0);
            products(m + 4 * U, c1, a1);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            int n = n0 + MF<R>::row(v, kk), k = k0 + i;
            if (n < g.Nout && k < g.K)
                Y[(long long)n * g.ldy + k] =
                    cmk(os * (ycur[v].x + g.cs * (double)dr[v]), os * (ycur[v].y + g.cs * (double)di[v]));
        }
    }
}

// W[b][i][(n,s)] = sum_j sum_t D[i][j][s][t] Bm[b][j][(n,t)]
__global__ void k_dmat(const double2* Bm, const double2* D, double2* Wm, int nproj, int nb, int nbatch) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long per = (long long)nproj * 2 * nb;
    if (idx >= per * nbatch) return;
    long long b = idx / per;
    int r = (int)(idx - b * per);
    int i = r / (2 * nb), ns = r % (2 * nb);
    int n = ns >> 1, s = ns & 1;
    const double2* Bb = Bm + b * per;
    double2 acc = cmk(0.0, 0.0);
    for (int j = 0; j < nproj; ++j)
        for (int t = 0; t < 2; ++t)
            acc = cadd(acc, cmul(D[((i * nproj + j) * 2 + s) * 2 + t], Bb[(long long)j * 2 * nb + 2 * n + t]));
    Wm[idx] = acc;
}

// the LDS-staged kernel needs its tiles to fit the waves, and enough tiles to
// keep its 8 waves busy (single-tile products stay on k_gemm_cn)
bool cn_lds_fits(int M, int Nn) {
    const int mt = (M + 15) / 16, nt = (Nn + 15) / 16;
    return mt <= kMaxTiles1D && nt <= kMaxTiles1D && mt + nt <= kCnMaxTilesSum && mt * nt <= 8 * kCnTilesPerWave &&
           mt * nt >= 8;
}

// K range per block: about 4 blocks per CU over all batches, a multiple of the LDS chunk
// K chunk per block: about `target` blocks over the batches of one right-hand
// side (the autotuner times 1024, 512 and 2048)
int cn_lds_kchunk(int K, int nbatch, int target = 1024) {
    const int ks = std::max(1, target / std::max(1, nbatch));
    int kc = (K + ks - 1) / ks;
    kc = std::max(kCnChunk * 4, (kc + kCnChunk - 1) / kCnChunk * kCnChunk);
    return kc;
}

int choose_kchunk(int K, long long tiles_times_batch, long long target = 8192) {
    // enough waves to fill the chip, but chunks of at least 64
    int ks = (int)std::max<long long>(1, target / std::max<long long>(1, tiles_times_batch));
    int kc = (K + ks - 1) / ks;
    kc = std::max(64, (kc + 3) / 4 * 4);
    return kc;
}

// nbatch batches per right-hand side, nrhs right-hand sides (the K chunking
// depends on nbatch only, so each right-hand side is summed as when alone);
// batch b takes A_tab[b % amod]
void run_gemm_cn(const System& s, const double2* const* A_tab, int amod, int lda, const double2* B_base,
                 long long b_bstride, int ldb, int M, int Nn, int K, int nbatch, int nrhs, double2* out,
                 hipStream_t st, bool f32 = false) {
    GemmCN g;
    g.A_tab = A_tab;
    g.amod = amod;
    g.A_base = nullptr;
    g.a_bstride = 0;
    g.lda = lda;
    g.B_base = B_base;
    g.b_bstride = b_bstride;
    g.ldb = ldb;
    g.M = M;
    g.Nn = Nn;
    g.K = K;
    int mt = (M + 15) / 16;
    g.nt = (Nn + 15) / 16;
    g.part = s.ws.gpart;
    if (!cn_lds_fits(M, Nn) && K <= kSmallK) {
        dim3 grid(mt * g.nt, nrhs * nbatch);
        if (f32) {
            TM_LAUNCH(k_gemm_cn_small<float>, grid, dim3(64 * kSmallWaves), 0, st, g, out);
        } else {
            TM_LAUNCH(k_gemm_cn_small<double>, grid, dim3(64 * kSmallWaves), 0, st, g, out);
        }
        return;
    }
    // the K split the autotuner picked for this contraction (per right-hand side,
    // so that every right-hand side is summed as when alone); FP64 only.  The
    // key is the output shape and the batch count, not K: the q sets of a
    // system differ only in K, so all of them take the choice made at the
    // system's first apply, and a chain's arithmetic does not depend on which
    // q set happened to be applied first.
    constexpr int kTargets[3] = {1024, 512, 2048};
    const int tv = f32 ? 0 : tune_pick(kTuneGemm, tune_key(M, Nn, nbatch), 3);
    if (cn_lds_fits(M, Nn)) {
        g.kchunk = cn_lds_kchunk(K, nbatch, kTargets[tv]);
        g.ksplit = (K + g.kchunk - 1) / g.kchunk;
        TM_CHECK((size_t)nrhs * nbatch * g.ksplit * M * Nn <= s.ws.cap_gpart, TM_EINVAL,
                 "GEMM partial buffer too small");
        const size_t shm = (size_t)(mt + g.nt) * 16 * (kCnChunk + 1) * (f32 ? 8 : 16);
        dim3 grid(g.ksplit, nrhs * nbatch);
        const void* fn = f32 ? (const void*)k_gemm_cn_lds<float> : (const void*)k_gemm_cn_lds<double>;
        TM_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) == hipSuccess,
                 TM_EDEVICE, "cannot raise the LDS limit of k_gemm_cn_lds");
        if (f32) {
            TM_LAUNCH(k_gemm_cn_lds<float>, grid, dim3(kCnThreads), shm, st, g, mt);
        } else {
            TM_LAUNCH(k_gemm_cn_lds<double>, grid, dim3(kCnThreads), shm, st, g, mt);
        }
    } else {
        g.kchunk = choose_kchunk(K, (long long)mt * g.nt * nbatch, 8LL * kTargets[tv]);
        g.ksplit = (K + g.kchunk - 1) / g.kchunk;
        TM_CHECK((size_t)nrhs * nbatch * g.ksplit * M * Nn <= s.ws.cap_gpart, TM_EINVAL,
                 "GEMM partial buffer too small");
        dim3 grid(mt * g.nt, g.ksplit, nrhs * nbatch);
        if (f32) {
            TM_LAUNCH(k_gemm_cn<float>, grid, dim3(64), 0, st, g);
        } else {
            TM_LAUNCH(k_gemm_cn<double>, grid, dim3(64), 0, st, g);
        }
    }
    long long mn = (long long)M * Nn;
    TM_LAUNCH(k_reduce_parts, dim3((unsigned)((mn * nrhs * nbatch + 255) / 256)), dim3(256), 0, st, s.ws.gpart,
                       out, g.ksplit, mn, nrhs * nbatch);
}

void run_gemm_update(double2* Y, long long y_bstride, int ldy, const double2* C, long long c_bstride, int ldc,
                     const double2* const* A_tab, int tmod, int lda, int Nout, int K, int Minner, double cs,
                     double osx, double osy, int nk, int nrhs, hipStream_t st, bool f32 = false) {
    GemmUpd g;
    g.tmod = tmod;
    g.Y_base = Y;
    g.y_bstride = y_bstride;
    g.ldy = ldy;
    g.C_base = C;
    g.c_bstride = c_bstride;
    g.ldc = ldc;
    g.A_tab = A_tab;
    g.lda = lda;
    g.Nout = Nout;
    g.K = K;
    g.Minner = Minner;
    g.cs = cs;
    g.os_x = osx;
    g.os_y = osy;
    g.nk = nk;
    const int ntile = (Nout + 15) / 16;
    TM_CHECK(ntile <= 16, TM_EUNSUPPORTED, "more than 256 output columns per batch");
    dim3 grid(1, (K + 15) / 16, 2 * nk * nrhs);
    if (f32) {
        TM_LAUNCH((k_gemm_update<float, 0>), grid, dim3(64 * ntile), 0, st, g);
        return;
    }
    // the variant the autotuner picked for this shape (tuned with one
    // right-hand side; every variant gives the same result)
    switch (tune_pick(kTuneUpd, tune_key(Nout, Minner, 2 * nk), 3)) {
        case 0: TM_LAUNCH((k_gemm_update<double, 0>), grid, dim3(64 * ntile), 0, st, g); break;
        case 1: TM_LAUNCH((k_gemm_update<double, 2>), grid, dim3(64 * ntile), 0, st, g); break;
        default: TM_LAUNCH((k_gemm_update<double, 3>), grid, dim3(64 * ntile), 0, st, g); break;
    }
}

}  // namespace

// partial sums of the finest K split any variant uses
size_t gemm_partial_elems(int nbatch, int M, int Nn, int K) {
    int mt = (M + 15) / 16, nt = (Nn + 15) / 16;
    int kc = cn_lds_fits(M, Nn) ? cn_lds_kchunk(K, nbatch, 2048) : choose_kchunk(K, (long long)mt * nt * nbatch, 16384);
    int ks = (K + kc - 1) / kc;
    return (size_t)nbatch * ks * M * Nn;
}

// x and out hold nrhs BR vectors back to back
void launch_nonlocal(const System& s, const QSet& q, const double2* x, double2* out, hipStream_t st, bool f32,
                     int nrhs) {
    if (s.nproj == 0) return;
    const int nb = s.nbnd, P = q.npw_pad, nbatch = 2 * q.nk;
    const long long bstride = (long long)nb * 2 * P;
    double2* Bm = s.ws.gsmall;
    double2* Wm = s.ws.gsmall + (size_t)nrhs * nbatch * s.nproj * 2 * nb;
    run_gemm_cn(s, q.d_vkb, q.tmod, P, x, bstride, P, s.nproj, 2 * nb, P, nbatch, nrhs, Bm, st, f32);
    long long tot = (long long)nrhs * nbatch * s.nproj * 2 * nb;
    TM_LAUNCH(k_dmat, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Bm, s.dvan, Wm, s.nproj, nb,
                       nrhs * nbatch);
    run_gemm_update(out, bstride, P, Wm, (long long)s.nproj * 2 * nb, 2 * nb, q.d_vkb, q.tmod, P, 2 * nb, P,
                    s.nproj, 1.0, 1.0, 1.0, q.nk, nrhs, st, f32);
}

void launch_project_signed(const System& s, const QSet& q, double2* phi, double osx, double osy, hipStream_t st,
                           bool f32, int nrhs) {
    const int nb = s.nbnd, P = q.npw_pad, nbatch = 2 * q.nk;
    const long long bstride = (long long)nb * 2 * P;
    double2* S = s.ws.gsmall;
    run_gemm_cn(s, (const double2* const*)q.d_occ, q.tmod, 2 * P, phi, bstride, 2 * P, nb, nb, 2 * P, nbatch, nrhs,
                S, st, f32);
    run_gemm_update(phi, bstride, 2 * P, S, (long long)nb * nb, nb, (const double2* const*)q.d_occ, q.tmod, 2 * P,
                    nb, 2 * P, nb, -1.0, osx, osy, q.nk, nrhs, st, f32);
}

void launch_project(const System& s, const QSet& q, double2* out, hipStream_t st, bool f32, int nrhs) {
    launch_project_signed(s, q, out, 1.0, -1.0, st, f32, nrhs);
}

}  // namespace tml

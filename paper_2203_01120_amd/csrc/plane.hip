// Plane kernels with compile-time plane sizes (n1 x n2 <= 64 x 64).
//
// Same arithmetic as the generic k_density / k_apply_planes in apply.hip
// (see the comments there for the physics); the organisation differs:
//   * the four component planes of a band (x_up, x_dn, u_up, u_dn) sit in LDS
//     together, so every radix pass of the 2D FFT serves four planes per
//     barrier;
//   * plane sizes and radices are template constants (no integer division,
//     fully unrolled butterflies); rows are padded to n2+1 entries so that
//     row-wise accesses of neighbouring lanes fall in different LDS banks;
//   * the first (row) direction of the inverse transform and the last
//     direction of the forward transform run only over the rows that the
//     plane-wave sphere occupies; the column direction reads inactive rows as
//     zero instead of clearing them;
//   * the local fields of a block's points stay in registers across bands.
#include "fft_lds.h"
#include "plane.h"

namespace tml {

namespace {

struct CPlan {
    int nrad;
    int rad[8];
    int pre[8];  // product of the radices before stage s
};

constexpr CPlan cplan(int n) {
    CPlan p{};
    p.nrad = 0;
    int m = n, pre = 1;
    const int order[4] = {4, 5, 3, 2};
    for (int oi = 0; oi < 4; ++oi) {
        int r = order[oi];
        while (m % r == 0) {
            p.rad[p.nrad] = r;
            p.pre[p.nrad] = pre;
            pre *= r;
            ++p.nrad;
            m /= r;
        }
    }
    return p;
}

constexpr int cdiv(int a, int b) { return (a + b - 1) / b; }

// line addressing in the 4-plane LDS block
template <int N1, int N2>
struct Geom {
    static constexpr int N2P = N2 + 1;
    static constexpr int PS = N1 * N2P;
    static constexpr int NP = N1 * N2;
};

// rows of the planes: line l has base rowbase[l], elements contiguous
struct RowLines {
    const int* rowbase;
    static constexpr int ES = 1;
    __device__ int base(int l) const { return rowbase[l]; }
    __device__ bool valid(int, int) const { return true; }
};

// columns: line l = plane * N2 + i2, elements at stride N2P; inactive rows of
// the plane's sphere read as zero in the first stage
template <int N1, int N2>
struct ColLines {
    static constexpr int ES = Geom<N1, N2>::N2P;
    unsigned long long mx, mu;  // occupied rows of planes 0, 1 (x) and 2, 3 (u)
    __device__ int base(int l) const {
        int plane = l / N2;
        return plane * Geom<N1, N2>::PS + (l - plane * N2);
    }
    __device__ bool valid(int l, int row) const { return ((l < 2 * N2 ? mx : mu) >> row) & 1ULL; }
};

// One in-place mixed-radix stage over sub-transforms of length LB.
// DIF (decimation in frequency): DFT_R of x[j + t M] then twiddle W_LB^{r j}
// on output r; applied with LB = N, N/R0, ... it maps natural order to the
// mixed-radix digit-reversed order.  DIT (decimation in time): twiddle W_LB^{t j}
// on input t, then DFT_R; applied in the reverse stage order it maps
// digit-reversed input to natural order.  Every butterfly reads and writes the
// same R locations, so a thread may process any number of butterflies of a
// stage without an intermediate barrier.
template <int N, int R, int LB, int SIGN, bool DIF, bool MASKED, int NT, class Lines>
__device__ __forceinline__ void ipass(double2* pl, int nlines, const Lines& L, const double2* tw) {
    constexpr int M = LB / R;
    constexpr int BPL = N / R;
    constexpr int TWS = N / LB;
    constexpr int ES = Lines::ES;
    const int nb = nlines * BPL;
    for (int b = threadIdx.x; b < nb; b += NT) {
        const int line = b / BPL;
        const int r0 = b - line * BPL;
        const int blk = r0 / M;
        const int j = r0 - blk * M;
        const int e0 = blk * LB + j;
        const int base = L.base(line) + e0 * ES;
        double2 u[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            double2 x = cmk(0.0, 0.0);
            if (!MASKED || L.valid(line, e0 + t * M)) x = pl[base + t * M * ES];
            if (!DIF && t > 0 && j > 0) {
                double2 w = tw[t * j * TWS];
                if (SIGN > 0) w.y = -w.y;
                x = cmul(x, w);
            }
            u[t] = x;
        }
        dft_small<R>(u, SIGN);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double2 y = u[r];
            if (DIF && r > 0 && j > 0) {
                double2 w = tw[r * j * TWS];
                if (SIGN > 0) w.y = -w.y;
                y = cmul(y, w);
            }
            pl[base + r * M * ES] = y;
        }
    }
    __syncthreads();
}

// natural -> digit-reversed (inverse direction of the apply, SIGN = +1)
template <int N, int SIGN, int NT, bool MASKED, int STAGE = 0, int LB = N, class Lines>
__device__ __forceinline__ void fft_dif(double2* pl, int nlines, const Lines& L, const double2* tw) {
    constexpr CPlan cp = cplan(N);
    if constexpr (STAGE < cp.nrad) {
        constexpr int R = cp.rad[STAGE];
        ipass<N, R, LB, SIGN, true, MASKED && STAGE == 0, NT>(pl, nlines, L, tw);
        fft_dif<N, SIGN, NT, MASKED, STAGE + 1, LB / R>(pl, nlines, L, tw);
    }
}

// digit-reversed -> natural; stages in reverse order (LB = N / (R0 ... R_{s-1}))
template <int N, int SIGN, int NT, int STAGE, class Lines>
__device__ __forceinline__ void fft_dit(double2* pl, int nlines, const Lines& L, const double2* tw) {
    constexpr CPlan cp = cplan(N);
    if constexpr (STAGE >= 0) {
        constexpr int R = cp.rad[STAGE];
        constexpr int LB = N / cp.pre[STAGE];
        ipass<N, R, LB, SIGN, false, false, NT>(pl, nlines, L, tw);
        fft_dit<N, SIGN, NT, STAGE - 1>(pl, nlines, L, tw);
    }
}

template <int N, int SIGN, int NT, class Lines>
__device__ __forceinline__ void fft_dit_all(double2* pl, int nlines, const Lines& L, const double2* tw) {
    constexpr CPlan cp = cplan(N);
    fft_dit<N, SIGN, NT, cp.nrad - 1>(pl, nlines, L, tw);
}

template <int N1, int N2, int NT>
struct PlaneKernel {
    using G = Geom<N1, N2>;
    static constexpr int PTS = cdiv(G::NP, NT);

    // LDS carve-up: 4 planes, twiddles, row line table, digit-reversal tables
    struct Smem {
        double2* pl;
        double2* tw1;
        double2* tw2;
        int* rowbase;
        int* perm1;
        int* perm2;
    };
    __device__ static Smem carve(double2* lds) {
        Smem m;
        m.pl = lds;
        m.tw1 = lds + 4 * G::PS;
        m.tw2 = m.tw1 + N1;
        m.rowbase = reinterpret_cast<int*>(m.tw2 + N2);
        m.perm1 = m.rowbase + 4 * N1;
        m.perm2 = m.perm1 + N1;
        return m;
    }
    static constexpr size_t bytes() {
        return (size_t)4 * G::PS * sizeof(double2) + (N1 + N2) * sizeof(double2) + (4 * N1 + N1 + N2) * sizeof(int);
    }

    __device__ static void setup(const PlaneTabs& t, int b, const Smem& m, int& nrx, int& nru,
                                 unsigned long long& mx, unsigned long long& mu) {
        nrx = t.nrows_kq[b];
        nru = t.nrows_u[b];
        mx = t.rmask_kq[b];
        mu = t.rmask_u[b];
        const int* rx = t.rows_kq[b];
        const int* ru = t.rows_u[b];
        for (int i = threadIdx.x; i < N1; i += NT) {
            m.tw1[i] = t.tw1[i];
            m.perm1[i] = t.perm1[i];
        }
        for (int i = threadIdx.x; i < N2; i += NT) {
            m.tw2[i] = t.tw2[i];
            m.perm2[i] = t.perm2[i];
        }
        for (int i = threadIdx.x; i < 2 * nrx + 2 * nru; i += NT) {
            int plane, row;
            if (i < 2 * nrx) {
                plane = i / nrx;
                row = rx[i - plane * nrx];
            } else {
                int j = i - 2 * nrx;
                plane = 2 + j / nru;
                row = ru[j - (plane - 2) * nru];
            }
            m.rowbase[i] = plane * G::PS + row * G::N2P;
        }
        __syncthreads();
    }

    // x_up, x_dn, u_up, u_dn of band n at plane i3 -> real space in the 4 LDS
    // planes, stored at digit-reversed positions along both axes
    __device__ static void inverse4(const Smem& m, const PlaneArgs& a, int b, int n, int i3, int nrx, int nru,
                                    unsigned long long mx, unsigned long long mu) {
        double2* pl = m.pl;
        const int nrl = 2 * nrx + 2 * nru;
        for (int i = threadIdx.x; i < nrl * N2; i += NT) {  // clear the occupied rows
            int l = i / N2;
            pl[m.rowbase[l] + (i - l * N2)] = cmk(0.0, 0.0);
        }
        __syncthreads();
        const int ncx = a.ncol_kq[b], ncu = a.ncol_u[b];
        const int* cpx = a.colpos_kq[b];
        const int* cpu = a.colpos_u[b];
        const double2* cx = a.xcols + (((long long)b * a.nitems + 2 * n) * a.n3 + i3) * a.ncol_max;
        const long long xs = (long long)a.n3 * a.ncol_max;
        const double2* cu = a.ucols + (((long long)b * a.nitems + 2 * n) * a.n3 + i3) * a.ncol_u_max;
        const long long us = (long long)a.n3 * a.ncol_u_max;
        for (int i = threadIdx.x; i < 2 * ncx; i += NT) {
            int s = i >= ncx, c = i - s * ncx;
            int pos = cpx[c];
            int i1 = pos / N2, i2 = pos - i1 * N2;
            pl[s * G::PS + i1 * G::N2P + i2] = cx[s * xs + c];
        }
        for (int i = threadIdx.x; i < 2 * ncu; i += NT) {
            int s = i >= ncu, c = i - s * ncu;
            int pos = cpu[c];
            int i1 = pos / N2, i2 = pos - i1 * N2;
            pl[(2 + s) * G::PS + i1 * G::N2P + i2] = cu[s * us + c];
        }
        __syncthreads();
        RowLines rl{m.rowbase};
        fft_dif<N2, +1, NT, false>(pl, nrl, rl, m.tw2);
        ColLines<N1, N2> cl;
        cl.mx = mx;
        cl.mu = mu;
        fft_dif<N1, +1, NT, true>(pl, 4 * N2, cl, m.tw1);
    }
};

template <int N1, int N2, int NT>
__global__ void __launch_bounds__(NT) k_density_t(PlaneArgs a, PlaneTabs t) {
    using K = PlaneKernel<N1, N2, NT>;
    using G = typename K::G;
    constexpr int PTS = K::PTS;
    extern __shared__ double2 lds[];
    const typename K::Smem m = K::carve(lds);
    double2* pl = m.pl;
    const int i3 = blockIdx.x, chunk = blockIdx.y, b = blockIdx.z;
    int nrx, nru;
    unsigned long long mx, mu;
    K::setup(t, b, m, nrx, nru, mx, mu);
    const int n0 = chunk * a.bpc;
    const int n1e = min(a.nb, n0 + a.bpc);
    const bool yside = b >= a.nk;
    double2 acc[4][PTS];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int j = 0; j < PTS; ++j) acc[c][j] = cmk(0.0, 0.0);
    for (int n = n0; n < n1e; ++n) {
        K::inverse4(m, a, b, n, i3, nrx, nru, mx, mu);
#pragma unroll
        for (int j = 0; j < PTS; ++j) {
            const int pt = threadIdx.x + j * NT;
            if (pt < G::NP) {
                const int p1 = pt / N2, o = p1 * G::N2P + (pt - p1 * N2);
                double2 xu = pl[o], xd = pl[G::PS + o], uu = pl[2 * G::PS + o], ud = pl[3 * G::PS + o];
                if (yside) {  // u' = T U_-k: (a, b) -> (conj b, -conj a)
                    double2 t0 = uu;
                    uu = cconj(ud);
                    ud = cmk(-t0.x, t0.y);
                }
                double2 uu_xu = cmulc(uu, xu), ud_xd = cmulc(ud, xd);
                double2 uu_xd = cmulc(uu, xd), ud_xu = cmulc(ud, xu);
                acc[0][j] = cadd(acc[0][j], cadd(uu_xu, ud_xd));
                acc[1][j] = cadd(acc[1][j], cadd(uu_xd, ud_xu));
                acc[2][j] = cadd(acc[2][j], cmuli(csub(ud_xu, uu_xd)));
                acc[3][j] = cadd(acc[3][j], csub(uu_xu, ud_xd));
            }
        }
        __syncthreads();
    }
    const long long N = (long long)G::NP * a.n3;
    double2* out = a.rho_part + ((long long)b * a.nchunk + chunk) * 4 * N + (long long)i3 * G::NP;
#pragma unroll
    for (int j = 0; j < PTS; ++j) {
        const int pt = threadIdx.x + j * NT;
        if (pt < G::NP) {
            const int p1 = pt / N2, p2 = pt - p1 * N2;
            const int g = m.perm1[p1] * N2 + m.perm2[p2];
#pragma unroll
            for (int c = 0; c < 4; ++c) out[c * N + g] = acc[c][j];
        }
    }
}

template <int N1, int N2, int NT>
__global__ void __launch_bounds__(NT) k_apply_t(PlaneArgs a, PlaneTabs t) {
    using K = PlaneKernel<N1, N2, NT>;
    using G = typename K::G;
    constexpr int PTS = K::PTS;
    extern __shared__ double2 lds[];
    const typename K::Smem m = K::carve(lds);
    double2* pl = m.pl;
    const int i3 = blockIdx.x, chunk = blockIdx.y, b = blockIdx.z;
    int nrx, nru;
    unsigned long long mx, mu;
    K::setup(t, b, m, nrx, nru, mx, mu);
    const int n0 = chunk * a.bpc;
    const int n1e = min(a.nb, n0 + a.bpc);
    const double sg = b < a.nk ? 1.0 : -1.0;
    const bool yside = b >= a.nk;
    const long long N = (long long)G::NP * a.n3;
    const long long off = (long long)i3 * G::NP;
    // local fields of my points (at the digit-reversed positions the planes use):
    // V0 = v + sg B.sigma, V' = W0 + sg W.sigma
    double vv[PTS], bx[PTS], by[PTS], bz[PTS];
    double2 w0[PTS], wx[PTS], wy[PTS], wz[PTS];
#pragma unroll
    for (int j = 0; j < PTS; ++j) {
        const int pt = threadIdx.x + j * NT;
        if (pt < G::NP) {
            const int p1 = pt / N2, p2 = pt - p1 * N2;
            const long long g = off + m.perm1[p1] * N2 + m.perm2[p2];
            vv[j] = a.vrs[g];
            bx[j] = sg * a.vrs[N + g];
            by[j] = sg * a.vrs[2 * N + g];
            bz[j] = sg * a.vrs[3 * N + g];
            w0[j] = a.W[g];
            wx[j] = cscale(a.W[N + g], sg);
            wy[j] = cscale(a.W[2 * N + g], sg);
            wz[j] = cscale(a.W[3 * N + g], sg);
        } else {
            vv[j] = bx[j] = by[j] = bz[j] = 0.0;
            w0[j] = wx[j] = wy[j] = wz[j] = cmk(0.0, 0.0);
        }
    }
    const int ncx = a.ncol_kq[b];
    const int* cpx = a.colpos_kq[b];
    for (int n = n0; n < n1e; ++n) {
        K::inverse4(m, a, b, n, i3, nrx, nru, mx, mu);
#pragma unroll
        for (int j = 0; j < PTS; ++j) {
            const int pt = threadIdx.x + j * NT;
            if (pt < G::NP) {
                const int p1 = pt / N2, o = p1 * G::N2P + (pt - p1 * N2);
                double2 xu = pl[o], xd = pl[G::PS + o], uu = pl[2 * G::PS + o], ud = pl[3 * G::PS + o];
                if (yside) {
                    double2 t0 = uu;
                    uu = cconj(ud);
                    ud = cmk(-t0.x, t0.y);
                }
                double2 bm = cmk(bx[j], -by[j]), bp = cmk(bx[j], by[j]);
                double2 pu = cadd(cscale(xu, vv[j] + bz[j]), cmul(bm, xd));
                double2 pd = cadd(cscale(xd, vv[j] - bz[j]), cmul(bp, xu));
                double2 wm = csub(wx[j], cmuli(wy[j])), wp = cadd(wx[j], cmuli(wy[j]));
                pu = cadd(pu, cadd(cmul(cadd(w0[j], wz[j]), uu), cmul(wm, ud)));
                pd = cadd(pd, cadd(cmul(csub(w0[j], wz[j]), ud), cmul(wp, uu)));
                pl[o] = pu;
                pl[G::PS + o] = pd;
            }
        }
        __syncthreads();
        // forward, digit-reversed -> natural: columns of planes 0, 1, then the
        // occupied rows of the k+q sphere
        ColLines<N1, N2> cl;
        cl.mx = cl.mu = ~0ULL;
        fft_dit_all<N1, -1, NT>(pl, 2 * N2, cl, m.tw1);
        RowLines rl{m.rowbase};
        fft_dit_all<N2, -1, NT>(pl, 2 * nrx, rl, m.tw2);
        double2* co = a.xcols + (((long long)b * a.nitems + 2 * n) * a.n3 + i3) * a.ncol_max;
        const long long cs = (long long)a.n3 * a.ncol_max;
        for (int i = threadIdx.x; i < 2 * ncx; i += NT) {
            int s = i >= ncx, c = i - s * ncx;
            int pos = cpx[c];
            int i1 = pos / N2, i2 = pos - i1 * N2;
            co[s * cs + c] = pl[s * G::PS + i1 * G::N2P + i2];
        }
        __syncthreads();
    }
}

template <int N1, int N2, int NT>
void launch_t(bool density, const PlaneArgs& a, const PlaneTabs& t, dim3 grid, hipStream_t st) {
    size_t shm = PlaneKernel<N1, N2, NT>::bytes();
    if (density) {
        TM_CHECK(hipFuncSetAttribute((const void*)k_density_t<N1, N2, NT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) == hipSuccess,
                 TM_EDEVICE, "cannot raise the LDS limit of k_density_t");
        TM_LAUNCH((k_density_t<N1, N2, NT>), grid, dim3(NT), shm, st, a, t);
    } else {
        TM_CHECK(hipFuncSetAttribute((const void*)k_apply_t<N1, N2, NT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) == hipSuccess,
                 TM_EDEVICE, "cannot raise the LDS limit of k_apply_t");
        TM_LAUNCH((k_apply_t<N1, N2, NT>), grid, dim3(NT), shm, st, a, t);
    }
}

}  // namespace

// ---------------------------------------------------------------- z passes
// Sphere <-> column transforms along i3 with a compile-time length.  Lines of
// L = CT x IT (column, item) pairs sit in LDS with a padded stride; the
// in-place stages leave the inverse output digit-reversed, so the write-out
// puts LDS position p at grid index perm3[p], and the forward load does the
// converse before the DIT stages restore natural order.
namespace {

template <int LS>
struct ZLines {
    static constexpr int ES = 1;
    __device__ int base(int l) const { return l * LS; }
    __device__ bool valid(int, int) const { return true; }
};

template <int N3, int NT, int CT, int IT>
__global__ void __launch_bounds__(NT) k_zinv_t(ZPassArgs a) {
    constexpr int L = CT * IT;
    constexpr int LS = N3 + 1;
    extern __shared__ double2 lds[];
    double2* tw = lds + L * LS;
    int* perm = reinterpret_cast<int*>(tw + N3);
    const int b = blockIdx.z;
    const int ncol = a.ncol[b];
    const int col0 = blockIdx.x * CT;
    if (col0 >= ncol) return;
    const int item0 = blockIdx.y * IT;
    for (int i = threadIdx.x; i < N3; i += NT) {
        tw[i] = a.tw[i];
        perm[i] = a.perm[i];
    }
    for (int i = threadIdx.x; i < L * LS; i += NT) lds[i] = cmk(0.0, 0.0);
    __syncthreads();
    const int* cp = a.colptr[b];
    const int* eg = a.entg[b];
    const int* ei = a.enti3[b];
    const double2* coef = a.coef_table ? a.coef_table[b] : a.coef_base + (long long)b * a.coef_bstride;
    const long long istr = a.istride_tab ? a.istride_tab[b] : a.istride;
    constexpr int PER = NT / L > 0 ? NT / L : 1;
    for (int l = threadIdx.x / PER; l < L; l += NT / PER) {
        const int c = col0 + l % CT, item = item0 + l / CT;
        if (c < ncol && item < a.nitems) {
            const double2* src = coef + (long long)item * istr;
            for (int e = cp[c] + threadIdx.x % PER; e < cp[c + 1]; e += PER) lds[l * LS + ei[e]] = src[eg[e]];
        }
    }
    __syncthreads();
    fft_dif<N3, +1, NT, false>(lds, L, ZLines<LS>{}, tw);
    double2* out = a.cols + (long long)b * a.nitems * N3 * a.ncol_stride;
    for (int i = threadIdx.x; i < L * N3; i += NT) {
        const int cl = i % CT, rest = i / CT;
        const int p = rest % N3, il = rest / N3;
        const int c = col0 + cl, item = item0 + il;
        if (c < ncol && item < a.nitems)
            out[((long long)item * N3 + perm[p]) * a.ncol_stride + c] = lds[(il * CT + cl) * LS + p];
    }
}

template <int N3, int NT, int CT, int IT>
__global__ void __launch_bounds__(NT) k_zfwd_t(ZPassArgs a) {
    constexpr int L = CT * IT;
    constexpr int LS = N3 + 1;
    extern __shared__ double2 lds[];
    double2* tw = lds + L * LS;
    int* perm = reinterpret_cast<int*>(tw + N3);
    const int b = blockIdx.z;
    const int ncol = a.ncol[b];
    const int col0 = blockIdx.x * CT;
    const int item0 = blockIdx.y * IT;
    const long long bbase = (long long)b * a.nitems * a.npw_pad;
    if (blockIdx.x == 0) {  // the first column tile clears the padding of its items
        const int npw = a.npw[b], padn = a.npw_pad - npw;
        for (int i = threadIdx.x; i < IT * padn; i += NT) {
            const int item = item0 + i / padn;
            if (item < a.nitems) a.out[bbase + (long long)item * a.npw_pad + npw + i % padn] = cmk(0.0, 0.0);
        }
    }
    if (col0 >= ncol) return;
    for (int i = threadIdx.x; i < N3; i += NT) {
        tw[i] = a.tw[i];
        perm[i] = a.perm[i];
    }
    __syncthreads();
    const double2* cin = a.cols + (long long)b * a.nitems * N3 * a.ncol_stride;
    for (int i = threadIdx.x; i < L * N3; i += NT) {
        const int cl = i % CT, rest = i / CT;
        const int p = rest % N3, il = rest / N3;
        const int c = col0 + cl, item = item0 + il;
        double2 v = cmk(0.0, 0.0);
        if (c < ncol && item < a.nitems) v = cin[((long long)item * N3 + perm[p]) * a.ncol_stride + c];
        lds[(il * CT + cl) * LS + p] = v;
    }
    __syncthreads();
    fft_dit_all<N3, -1, NT>(lds, L, ZLines<LS>{}, tw);
    const int* cp = a.colptr[b];
    const int* eg = a.entg[b];
    const int* ei = a.enti3[b];
    const double* kin = a.kin[b];
    const double* eps = a.eps[b];
    constexpr int PER = NT / L > 0 ? NT / L : 1;
    for (int l = threadIdx.x / PER; l < L; l += NT / PER) {
        const int c = col0 + l % CT, item = item0 + l / CT;
        if (c < ncol && item < a.nitems) {
            const double e = eps[item >> 1];
            const long long off = bbase + (long long)item * a.npw_pad;
            for (int en = cp[c] + threadIdx.x % PER; en < cp[c + 1]; en += PER) {
                const int g = eg[en];
                const double2 f = cscale(lds[l * LS + ei[en]], a.inv_n);
                const double2 x = a.xin[off + g];
                const double s = kin[g] - e;
                a.out[off + g] = cmk(f.x + s * x.x, f.y + s * x.y);
            }
        }
    }
}

template <int N3, int NT, int CT, int IT>
void launch_z(bool inverse, const ZPassArgs& a, int ncolmax, int nbatch, hipStream_t st) {
    constexpr int L = CT * IT;
    const size_t shm = (size_t)L * (N3 + 1) * sizeof(double2) + N3 * sizeof(double2) + N3 * sizeof(int);
    dim3 grid((ncolmax + CT - 1) / CT, (a.nitems + IT - 1) / IT, nbatch);
    if (inverse) {
        TM_LAUNCH((k_zinv_t<N3, NT, CT, IT>), grid, dim3(NT), shm, st, a);
    } else {
        TM_LAUNCH((k_zfwd_t<N3, NT, CT, IT>), grid, dim3(NT), shm, st, a);
    }
}

}  // namespace

bool zpass_fixed_supported(int n3) {
    return n3 == 8 || n3 == 20 || n3 == 24 || n3 == 32 || n3 == 48 || n3 == 96 || n3 == 180;
}

void launch_zpass_fixed(bool inverse, const ZPassArgs& a, int ncolmax, int nbatch, int n3, hipStream_t st) {
    switch (n3) {
        case 8: launch_z<8, 256, 16, 4>(inverse, a, ncolmax, nbatch, st); break;
        case 20: launch_z<20, 256, 16, 4>(inverse, a, ncolmax, nbatch, st); break;
        case 24: launch_z<24, 256, 16, 4>(inverse, a, ncolmax, nbatch, st); break;
        case 32: launch_z<32, 256, 16, 2>(inverse, a, ncolmax, nbatch, st); break;
        case 48: launch_z<48, 256, 16, 2>(inverse, a, ncolmax, nbatch, st); break;
        case 96: launch_z<96, 256, 16, 1>(inverse, a, ncolmax, nbatch, st); break;
        case 180: launch_z<180, 256, 16, 1>(inverse, a, ncolmax, nbatch, st); break;
        default: throw Error{TM_EUNSUPPORTED, "no fixed-size z pass for this grid"};
    }
}

std::vector<int> digit_reversal(int n) {
    FFTPlan p;
    std::vector<int> perm(n, 0);
    if (!make_radices(n, p)) return perm;
    for (int pos = 0; pos < n; ++pos) {
        int rem = pos, place = n, weight = 1, k = 0;
        for (int s = 0; s < p.nrad; ++s) {
            place /= p.rad[s];
            int d = rem / place;
            rem -= d * place;
            k += d * weight;
            weight *= p.rad[s];
        }
        perm[pos] = k;
    }
    return perm;
}

bool plane_fixed_supported(int n1, int n2) {
    return (n1 == 8 && n2 == 8) || (n1 == 20 && n2 == 20) || (n1 == 24 && n2 == 24) || (n1 == 32 && n2 == 32) ||
           (n1 == 48 && n2 == 48);
}

void launch_plane_fixed(bool density, const PlaneArgs& a, const PlaneTabs& t, dim3 grid, int n1, int n2,
                        hipStream_t st) {
    if (n1 == 8 && n2 == 8) launch_t<8, 8, 64>(density, a, t, grid, st);
    else if (n1 == 20 && n2 == 20) launch_t<20, 20, 256>(density, a, t, grid, st);
    else if (n1 == 24 && n2 == 24) launch_t<24, 24, 256>(density, a, t, grid, st);
    else if (n1 == 32 && n2 == 32) launch_t<32, 32, 512>(density, a, t, grid, st);
    else if (n1 == 48 && n2 == 48) launch_t<48, 48, 1024>(density, a, t, grid, st);
    else throw Error{TM_EUNSUPPORTED, "no fixed-size plane kernel for this grid"};
}

}  // namespace tml

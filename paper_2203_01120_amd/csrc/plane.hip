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
#include <type_traits>

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
template <int N, int R, int LB, int SIGN, bool DIF, bool MASKED, int NT, class Lines, class T2>
__device__ __forceinline__ void ipass(T2* pl, int nlines, const Lines& L, const T2* tw) {
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
        T2 u[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
            T2 x = Cx<T2>::mk(0, 0);
            if (!MASKED || L.valid(line, e0 + t * M)) x = pl[base + t * M * ES];
            if (!DIF && t > 0 && j > 0) {
                T2 w = tw[t * j * TWS];
                if (SIGN > 0) w.y = -w.y;
                x = cmul(x, w);
            }
            u[t] = x;
        }
        dft_small<R>(u, SIGN);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            T2 y = u[r];
            if (DIF && r > 0 && j > 0) {
                T2 w = tw[r * j * TWS];
                if (SIGN > 0) w.y = -w.y;
                y = cmul(y, w);
            }
            pl[base + r * M * ES] = y;
        }
    }
    __syncthreads();
}

// natural -> digit-reversed (inverse direction of the apply, SIGN = +1)
template <int N, int SIGN, int NT, bool MASKED, int STAGE = 0, int LB = N, class Lines, class T2>
__device__ __forceinline__ void fft_dif(T2* pl, int nlines, const Lines& L, const T2* tw) {
    constexpr CPlan cp = cplan(N);
    if constexpr (STAGE < cp.nrad) {
        constexpr int R = cp.rad[STAGE];
        ipass<N, R, LB, SIGN, true, MASKED && STAGE == 0, NT>(pl, nlines, L, tw);
        fft_dif<N, SIGN, NT, MASKED, STAGE + 1, LB / R>(pl, nlines, L, tw);
    }
}

// digit-reversed -> natural; stages in reverse order (LB = N / (R0 ... R_{s-1}))
template <int N, int SIGN, int NT, int STAGE, class Lines, class T2>
__device__ __forceinline__ void fft_dit(T2* pl, int nlines, const Lines& L, const T2* tw) {
    constexpr CPlan cp = cplan(N);
    if constexpr (STAGE >= 0) {
        constexpr int R = cp.rad[STAGE];
        constexpr int LB = N / cp.pre[STAGE];
        ipass<N, R, LB, SIGN, false, false, NT>(pl, nlines, L, tw);
        fft_dit<N, SIGN, NT, STAGE - 1>(pl, nlines, L, tw);
    }
}

template <int N, int SIGN, int NT, class Lines, class T2>
__device__ __forceinline__ void fft_dit_all(T2* pl, int nlines, const Lines& L, const T2* tw) {
    constexpr CPlan cp = cplan(N);
    fft_dit<N, SIGN, NT, cp.nrad - 1>(pl, nlines, L, tw);
}

// Which planes a block-synchronous kernel keeps in LDS.
//   kXU: x_up, x_dn, u_up, u_dn; the ground-state band is transformed in the
//        kernel from its z-transformed columns (column path);
//   kU:  u_up, u_dn; builds the resident real-space copy.
enum PlaneSet { kXU = 0, kU = 2 };

template <int N1, int N2, int NT, int SET>
struct PlaneKernel {
    using G = Geom<N1, N2>;
    static constexpr int NPL = SET == kXU ? 4 : 2;
    static constexpr int PTS = cdiv(G::NP, NT);

    // LDS carve-up: planes, twiddles, row line table, digit-reversal tables
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
        m.tw1 = lds + NPL * G::PS;
        m.tw2 = m.tw1 + N1;
        m.rowbase = reinterpret_cast<int*>(m.tw2 + N2);
        m.perm1 = m.rowbase + NPL * N1;
        m.perm2 = m.perm1 + N1;
        return m;
    }
    static constexpr size_t bytes() {
        return (size_t)NPL * G::PS * sizeof(double2) + (N1 + N2) * sizeof(double2) +
               (NPL * N1 + N1 + N2) * sizeof(int);
    }

    // occupied rows of the block's planes
    struct Rows {
        int nrl;                  // row lines in the row table
        int nrx;                  // occupied rows of the k+q sphere
        unsigned long long m01;   // row mask of planes 0, 1
        unsigned long long m23;   // row mask of planes 2, 3
    };

    __device__ static Rows setup(const PlaneTabs& t, int b, const Smem& m) {
        Rows R;
        const int nrx = t.nrows_kq[b], nru = t.nrows_u[b];
        const int* rx = t.rows_kq[b];
        const int* ru = t.rows_u[b];
        R.nrx = nrx;
        if (SET == kU) {
            R.m01 = R.m23 = t.rmask_u[b];
            R.nrl = 2 * nru;
        } else {
            R.m01 = t.rmask_kq[b];
            R.m23 = t.rmask_u[b];
            R.nrl = 2 * nrx + 2 * nru;
        }
        for (int i = threadIdx.x; i < N1; i += NT) {
            m.tw1[i] = t.tw1[i];
            m.perm1[i] = t.perm1[i];
        }
        for (int i = threadIdx.x; i < N2; i += NT) {
            m.tw2[i] = t.tw2[i];
            m.perm2[i] = t.perm2[i];
        }
        const int nr0 = SET == kU ? nru : nrx;
        const int* r0 = SET == kU ? ru : rx;
        for (int i = threadIdx.x; i < R.nrl; i += NT) {
            int plane, row;
            if (i < 2 * nr0) {
                plane = i / nr0;
                row = r0[i - plane * nr0];
            } else {
                const int j = i - 2 * nr0;
                plane = 2 + j / nru;
                row = ru[j - (plane - 2) * nru];
            }
            m.rowbase[i] = plane * G::PS + row * G::N2P;
        }
        __syncthreads();
        return R;
    }

    // scatter the z-transformed columns of item pair (2n, 2n+1) of one sphere
    // into planes p0, p0+1
    __device__ static void scatter(double2* pl, int p0, const double2* cols, long long cstride, int ncol,
                                   const int* colpos) {
        for (int i = threadIdx.x; i < 2 * ncol; i += NT) {
            const int s = i >= ncol, c = i - s * ncol;
            const int pos = colpos[c];
            const int i1 = pos / N2, i2 = pos - i1 * N2;
            pl[(p0 + s) * G::PS + i1 * G::N2P + i2] = cols[s * cstride + c];
        }
    }

    // band n at plane i3 -> real space in the LDS planes, stored at
    // digit-reversed positions along both axes
    __device__ static void inverse(const Smem& m, const PlaneArgs& a, int b, int bt, int tb, int n, int i3,
                                   const Rows& R) {
        double2* pl = m.pl;
        for (int i = threadIdx.x; i < R.nrl * N2; i += NT) {  // clear the occupied rows
            const int l = i / N2;
            pl[m.rowbase[l] + (i - l * N2)] = cmk(0.0, 0.0);
        }
        __syncthreads();
        if (SET == kXU) {
            const double2* cx = a.xcols + (((long long)b * a.nitems + 2 * n) * a.n3 + i3) * a.ncol_max;
            scatter(pl, 0, cx, (long long)a.n3 * a.ncol_max, a.ncol_kq[tb], a.colpos_kq[tb]);
        }
        const double2* cu = a.ucols + (((long long)bt * a.nitems + 2 * n) * a.n3 + i3) * a.ncol_u_max;
        scatter(pl, SET == kXU ? 2 : 0, cu, (long long)a.n3 * a.ncol_u_max, a.ncol_u[bt], a.colpos_u[bt]);
        __syncthreads();
        RowLines rl{m.rowbase};
        fft_dif<N2, +1, NT, false>(pl, R.nrl, rl, m.tw2);
        ColLines<N1, N2> cl;
        cl.mx = R.m01;
        cl.mu = R.m23;
        fft_dif<N1, +1, NT, true>(pl, NPL * N2, cl, m.tw1);
    }
};

// time reversal of the spinor (u_up, u_dn) -> (conj u_dn, -conj u_up)
__device__ __forceinline__ void time_reverse(double2& uu, double2& ud) {
    const double2 t0 = uu;
    uu = cconj(ud);
    ud = cmk(-t0.x, t0.y);
}

// Column path, block-synchronous: every radix stage of a plane transform is
// one workgroup-wide pass over all lines of the four planes.
template <int N1, int N2, int NT>
__global__ void __launch_bounds__(NT) k_density_t(PlaneArgs a, PlaneTabs t) {
    using K = PlaneKernel<N1, N2, NT, kXU>;
    using G = typename K::G;
    constexpr int PTS = K::PTS;
    extern __shared__ double2 lds[];
    const typename K::Smem m = K::carve(lds);
    double2* pl = m.pl;
    // bt: side and k point (and the row of the q set's ground-state columns); tb: sphere tables
    const int i3 = blockIdx.x, chunk = blockIdx.y, b = blockIdx.z, bt = b % a.nb2, tb = b % a.tmod;
    const typename K::Rows R = K::setup(t, tb, m);
    const int n0 = chunk * a.bpc;
    const int n1e = min(a.nb, n0 + a.bpc);
    const bool yside = bt >= a.nk;
    double2 acc[4][PTS];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int j = 0; j < PTS; ++j) acc[c][j] = cmk(0.0, 0.0);
    for (int n = n0; n < n1e; ++n) {
        K::inverse(m, a, b, bt, tb, n, i3, R);
#pragma unroll
        for (int j = 0; j < PTS; ++j) {
            const int pt = threadIdx.x + j * NT;
            if (pt < G::NP) {
                const int p1 = pt / N2, o = p1 * G::N2P + (pt - p1 * N2);
                double2 xu = pl[o], xd = pl[G::PS + o], uu = pl[2 * G::PS + o], ud = pl[3 * G::PS + o];
                if (yside) time_reverse(uu, ud);  // u' = T U_-k
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
    using K = PlaneKernel<N1, N2, NT, kXU>;
    using G = typename K::G;
    constexpr int PTS = K::PTS;
    extern __shared__ double2 lds[];
    const typename K::Smem m = K::carve(lds);
    double2* pl = m.pl;
    // bt: side and k point (and the row of the q set's ground-state columns); tb: sphere tables
    const int i3 = blockIdx.x, chunk = blockIdx.y, b = blockIdx.z, bt = b % a.nb2, tb = b % a.tmod;
    const typename K::Rows R = K::setup(t, tb, m);
    const int n0 = chunk * a.bpc;
    const int n1e = min(a.nb, n0 + a.bpc);
    const double sg = bt < a.nk ? 1.0 : -1.0;
    const bool yside = bt >= a.nk;
    const double2* Wr = a.W + (long long)(b / a.nb2) * a.wstride;
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
            w0[j] = Wr[g];
            wx[j] = cscale(Wr[N + g], sg);
            wy[j] = cscale(Wr[2 * N + g], sg);
            wz[j] = cscale(Wr[3 * N + g], sg);
        } else {
            vv[j] = bx[j] = by[j] = bz[j] = 0.0;
            w0[j] = wx[j] = wy[j] = wz[j] = cmk(0.0, 0.0);
        }
    }
    const int ncx = a.ncol_kq[tb];
    const int* cpx = a.colpos_kq[tb];
    for (int n = n0; n < n1e; ++n) {
        K::inverse(m, a, b, bt, tb, n, i3, R);
#pragma unroll
        for (int j = 0; j < PTS; ++j) {
            const int pt = threadIdx.x + j * NT;
            if (pt < G::NP) {
                const int p1 = pt / N2, o = p1 * G::N2P + (pt - p1 * N2);
                double2 xu = pl[o], xd = pl[G::PS + o], uu = pl[2 * G::PS + o], ud = pl[3 * G::PS + o];
                if (yside) time_reverse(uu, ud);
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
        // occupied rows of the k+q sphere (the first 2 nrx row lines)
        ColLines<N1, N2> cl;
        cl.mx = cl.mu = ~0ULL;
        fft_dit_all<N1, -1, NT>(pl, 2 * N2, cl, m.tw1);
        RowLines rl{m.rowbase};
        fft_dit_all<N2, -1, NT>(pl, 2 * R.nrx, rl, m.tw2);
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

// Point order of a plane in the resident ground state, the per-apply field
// table and the wave kernels' point-wise phases: column-major over the LDS
// positions (p1, p2 digit-reversed), and within a column the row p1 = R blk + t
// (R the last radix of n1's plan) at r = t (n1 / R) + blk.  The last column
// stage works on butterflies of R consecutive rows, one per lane, so the lanes
// of a column read consecutive points of this order.
template <int N1>
__device__ __forceinline__ int wrow(int r) {
    constexpr CPlan cp = cplan(N1);
    constexpr int R = cp.rad[cp.nrad - 1], BPC = N1 / R;
    const int t = r / BPC, blk = r - t * BPC;
    return blk * R + t;
}

// Resident real-space ground state: [slot][band][i3][spin][plane point], the
// points in the order above, time reversal applied on the y side.

template <int N1, int N2, int NT>
__global__ void __launch_bounds__(NT) k_ureal_t(PlaneArgs a, PlaneTabs t) {
    using K = PlaneKernel<N1, N2, NT, kU>;
    using G = typename K::G;
    extern __shared__ double2 lds[];
    const typename K::Smem m = K::carve(lds);
    double2* pl = m.pl;
    const int i3 = blockIdx.x, chunk = blockIdx.y, b = blockIdx.z;
    const typename K::Rows R = K::setup(t, b, m);
    const int n0 = chunk * a.bpc;
    const int n1e = min(a.nb, n0 + a.bpc);
    const bool yside = b >= a.nk;
    for (int n = n0; n < n1e; ++n) {
        K::inverse(m, a, b, b, b, n, i3, R);
        double2* out = a.ureal + (((long long)a.uslot[b] * a.nb + n) * a.n3 + i3) * 2 * G::NP;
        for (int idx = threadIdx.x; idx < G::NP; idx += NT) {
            const int p2 = idx / N1, p1 = wrow<N1>(idx - p2 * N1);
            const int o = p1 * G::N2P + p2;
            double2 uu = pl[o], ud = pl[G::PS + o];
            if (yside) time_reverse(uu, ud);
            out[idx] = uu;
            out[G::NP + idx] = ud;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- wave-local kernels
// Resident ground state.  Each wave owns whole lines: in the row phase a
// subset of the occupied rows, in the column phase the columns
// p2 in [w CPW, (w+1) CPW) of both x planes.  The radix stages of a line then
// need no workgroup barrier: LDS instructions of one wave complete in issue
// order, and a wave-scope fence keeps the compiler from reordering them.  The
// point-wise products run inside the column phase on the wave's own columns,
// and two LDS buffers alternate between bands, so a band costs one workgroup
// barrier in the density and two in the apply.

// the double- or single-precision member of a pair of buffers
template <class T2, class D, class F>
__host__ __device__ inline auto pick(D d, F f) {
    if constexpr (std::is_same<T2, double2>::value) return d;
    else return f;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// lane slots per line of a stage with bpl butterflies per line
constexpr int wslots(int bpl) { return (bpl > 8 && bpl < 16) ? 16 : bpl; }

// true when every stage's slots per line divide the wave: a lane then sits at
// the same butterfly position of its line in every iteration, line and band
constexpr bool lane_fixed(int n) {
    const CPlan p = cplan(n);
    for (int s = 0; s < p.nrad; ++s)
        if (64 % wslots(n / p.rad[s]) != 0) return false;
    return true;
}

// Twiddles of a wave's stages.  With lane_fixed(N) a lane's twiddles are the
// same for the whole kernel: they are read from the table once, into
// registers, and the radix stages issue no global loads (whose in-order
// completion counter would also make them wait for the band's ground-state
// and column loads).  Otherwise they come from the table through the vector L1.
template <int N, class T2>
struct WTw {
    static constexpr CPlan cp = cplan(N);
    static constexpr bool kReg = lane_fixed(N);
    const T2* __restrict__ tab;
    T2 w[cp.nrad][4];

    template <int S = 0>
    __device__ __forceinline__ void init(int lane) {
        if constexpr (kReg && S < cp.nrad) {
            constexpr int R = cp.rad[S];
            constexpr int LB = N / cp.pre[S];
            constexpr int M = LB / R;
            constexpr int BPL = N / R;
            constexpr int TWS = N / LB;
            if constexpr (M > 1) {
                const int r0 = lane % wslots(BPL);
                const int j = r0 < BPL ? r0 % M : 0;
#pragma unroll
                for (int t = 1; t < R; ++t) w[S][t - 1] = tab[t * j * TWS];
            }
            init<S + 1>(lane);
        }
    }
    // twiddle t of butterfly j at stage S (LB = N / pre[S])
    template <int S, int LB>
    __device__ __forceinline__ T2 get(int t, int j) const {
        if constexpr (kReg) return w[S][t - 1];
        else return tab[t * j * (N / LB)];
    }
};

// one in-place stage (see ipass) over the nl lines of one wave.
//  * A line's butterflies sit on consecutive lanes; a line of 12 butterflies
//    takes a whole 16-lane group, so the 16 lanes that LDS serves together
//    address distinct banks (row pitch n2+1 puts element e of column c at bank
//    group (e + c) mod 16; offsets within a line are distinct mod 16 for every
//    stage of 48 = 4 x 4 x 3).
//  * Twiddles come from the table in device memory (vector L1), not from LDS.
//  * The lane's butterflies go in groups of BT whose loads are all issued
//    before their stores (BT trades registers for memory-level parallelism).
template <int N, int S, int R, int LB, int SIGN, bool DIF, bool MASKED, int MAXL, int BT, class WL, class T2>
__device__ __forceinline__ void wpass(T2* pl, const WL& L, int nl, const WTw<N, T2>& tw, int lane) {
    constexpr int M = LB / R;
    constexpr int BPL = N / R;
    constexpr int SPL = wslots(BPL);  // lane slots per line
    constexpr int ES = WL::ES;
    constexpr int IT = cdiv(MAXL * SPL, 64);
    constexpr int B = BT < IT ? BT : IT;
    const int ns = nl * SPL;
#pragma unroll
    for (int g0 = 0; g0 < IT; g0 += B) {
        T2 u[B][R];
        int base[B], jv[B];
#pragma unroll
        for (int it = 0; it < B; ++it) {
            const int sl = lane + (g0 + it) * 64;
            const int li = sl / SPL;
            const int r0 = sl - li * SPL;
            base[it] = -1;
            jv[it] = 0;
            if (g0 + it < IT && sl < ns && r0 < BPL) {
                const int blk = r0 / M;
                const int j = r0 - blk * M;
                const int e0 = blk * LB + j;
                const int bs = L.base(li, g0 + it) + e0 * ES;
                base[it] = bs;
                jv[it] = j;
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    T2 x = Cx<T2>::mk(0, 0);
                    if (!MASKED || L.valid(e0 + t * M)) x = pl[bs + t * M * ES];
                    if (!DIF && t > 0 && j > 0) {
                        T2 w = tw.template get<S, LB>(t, j);
                        if (SIGN > 0) w.y = -w.y;
                        x = cmul(x, w);
                    }
                    u[it][t] = x;
                }
            }
        }
#pragma unroll
        for (int it = 0; it < B; ++it) {
            if (base[it] >= 0) {
                dft_small<R>(u[it], SIGN);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    T2 y = u[it][r];
                    if (DIF && r > 0 && jv[it] > 0) {
                        T2 w = tw.template get<S, LB>(r, jv[it]);
                        if (SIGN > 0) w.y = -w.y;
                        y = cmul(y, w);
                    }
                    pl[base[it] + r * M * ES] = y;
                }
            }
        }
    }
    wave_sync();
}

// stages 0 .. NST - 1 of the plan
template <int N, int SIGN, bool MASKED, int MAXL, int BT, int NST = cplan(N).nrad, int STAGE = 0, int LB = N, class WL,
          class T2>
__device__ __forceinline__ void wfft_dif(T2* pl, const WL& L, int nl, const WTw<N, T2>& tw, int lane) {
    constexpr CPlan cp = cplan(N);
    if constexpr (STAGE < NST) {
        constexpr int R = cp.rad[STAGE];
        wpass<N, STAGE, R, LB, SIGN, true, MASKED && STAGE == 0, MAXL, BT>(pl, L, nl, tw, lane);
        wfft_dif<N, SIGN, MASKED, MAXL, BT, NST, STAGE + 1, LB / R>(pl, L, nl, tw, lane);
    }
}

// stages STAGE, STAGE - 1, ..., STOP of the plan
template <int N, int SIGN, int MAXL, int BT, int STAGE, int STOP = 0, class WL, class T2>
__device__ __forceinline__ void wfft_dit(T2* pl, const WL& L, int nl, const WTw<N, T2>& tw, int lane) {
    constexpr CPlan cp = cplan(N);
    if constexpr (STAGE >= STOP) {
        constexpr int R = cp.rad[STAGE];
        constexpr int LB = N / cp.pre[STAGE];
        wpass<N, STAGE, R, LB, SIGN, false, false, MAXL, BT>(pl, L, nl, tw, lane);
        wfft_dit<N, SIGN, MAXL, BT, STAGE - 1, STOP>(pl, L, nl, tw, lane);
    }
}

// true when every stage of a length-n transform gives a line the same lane
// slots, a divisor of 64: a lane then works on the same lines in every stage
constexpr bool rows_fixed(int n) {
    const CPlan p = cplan(n);
    const int s0 = wslots(n / p.rad[0]);
    if (64 % s0 != 0) return false;
    for (int s = 1; s < p.nrad; ++s)
        if (wslots(n / p.rad[s]) != s0) return false;
    return true;
}

// row lines w, w + NW, ... of the block's row table (nl of them).  With
// rows_fixed(N) the bases of the lane's lines are read from the table once,
// into registers (the table does not change within a block), so that a
// stage's loads do not wait on a dependent table read.
template <int NW, int N, int MAXL, bool CACHE>
struct WRows {
    static constexpr int ES = 1;
    static constexpr bool kFix = CACHE && rows_fixed(N);
    static constexpr int SPL = wslots(N / cplan(N).rad[0]);
    static constexpr int IT = kFix ? cdiv(MAXL * SPL, 64) : 1;
    const int* rowbase;
    int w, boff;
    int lb[IT];
    __device__ WRows(const int* rb, int w_, int nl, int lane) : rowbase(rb), w(w_), boff(0) {
        if constexpr (kFix) {
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int li = (lane + 64 * it) / SPL;
                lb[it] = li < nl ? rb[w + li * NW] : 0;
            }
        }
    }
    // line li, met in the lane's iteration it of a stage
    __device__ int base(int li, int it) const {
        if constexpr (kFix) return boff + lb[it];
        else return boff + rowbase[w + li * NW];
    }
    __device__ bool valid(int) const { return true; }
};

// columns c0 .. c0 + CPW - 1 of x planes 0 and 1; rows outside `mask` are
// read as zero by a masked first stage
// (ILV: line li is spin plane li % 2 of column c0 + li / 2, so that the two
// 16-lane groups of each half-wave hold one column of both spin planes)
template <int N1, int N2, int CPW, bool ILV = false>
struct WCols {
    static constexpr int ES = Geom<N1, N2>::N2P;
    int c0, boff;
    unsigned long long mask;
    __device__ int base(int li, int) const {
        if constexpr (ILV) return boff + (li & 1) * Geom<N1, N2>::PS + c0 + (li >> 1);
        const int s = li / CPW;
        return boff + s * Geom<N1, N2>::PS + c0 + (li - s * CPW);
    }
    __device__ bool valid(int row) const { return (mask >> row) & 1ULL; }
};

// The last column stage of the inverse transform (radix R, butterflies of R
// consecutive rows, no twiddles) and the first of the forward one, fused with
// the point-wise work in registers: slot sl of a wave's CPW n1 / R butterflies
// holds rows R blk .. R blk + R - 1 of column cc in both spin planes.
template <int N1, int N2, int CPW>
struct WTail {
    static constexpr CPlan cp = cplan(N1);
    static constexpr int R = cp.rad[cp.nrad - 1];
    static constexpr int BPC = N1 / R;        // butterflies per column
    static constexpr int SLOTS = CPW * BPC;
    static constexpr int IT = cdiv(SLOTS, 64);
    static_assert(cp.nrad >= 2, "the first column stage reads the row mask");
    int lo[IT];   // LDS offset (plane 0) of the slot's first row
    int lq[IT];   // wave point of the slot's first row; row t at lq + t BPC
    __device__ void init(int w, int lane) {
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            const int sl = min(lane + 64 * i, SLOTS - 1);
            const int cc = sl / BPC, blk = sl - cc * BPC;
            lo[i] = blk * R * Geom<N1, N2>::N2P + w * CPW + cc;
            lq[i] = cc * N1 + blk;
        }
    }
    __device__ static bool live(int lane, int i) { return lane + 64 * i < SLOTS; }
};

template <int N1, int N2, int BT_, int CPW_, class T2, int NBUF_, int FCH_ = 64, bool FUSE_ = false>
struct WaveKernel {
    using G = Geom<N1, N2>;
    // FP64 48 x 48: the lines a wave works on together come in spin pairs (a
    // row or a column of both planes in the two 16-lane groups of each
    // half-wave).  The four lines of a 16-byte LDS access then take no extra
    // cycles; adjacent columns or rows of one plane in those groups take 4
    // extra cycles per access (measured with a probe).
    static constexpr bool ILV = sizeof(T2) == 16 && N2 == 48;
    using Cols = WCols<N1, N2, CPW_, ILV>;
    // FUSE: the row fill is fused with the first inverse row stage, and the last
    // forward row stage with the output (a row's values skip one LDS round trip
    // at each end)
    static constexpr bool FUSE = FUSE_;
    static constexpr int NBUF = NBUF_;              // LDS buffers alternating between bands (1 or 2)
    static constexpr int CPW = CPW_;                // columns per wave
    static constexpr int NW = N2 / CPW;             // waves
    static constexpr int NT = 64 * NW;
    static constexpr int WPTS = CPW * N1;           // points of a wave (per plane)
    static constexpr int MAXR = cdiv(2 * N1, NW);   // row lines of a wave, at most
    static_assert(!ILV || 2 * cdiv(N1, NW) <= MAXR, "row pairs of a wave");
    static constexpr int BUF = 2 * G::PS;           // one buffer: planes x_up, x_dn
    static constexpr int BT = BT_;                  // butterflies per load group
    static_assert(N2 % CPW == 0 && NW <= 16, "plane shape");

    struct Smem {
        T2* pl;            // NBUF buffers
        int* rowbase;      // [2 N1] plane * PS + row * N2P of the occupied rows of planes 0, 1
        int* rowinfo;      // [2 N1] plane * N1 + row
        int* perm1;
        int* perm2;
        short* colidx;     // [N1 N2] column of the k+q sphere at natural plane position, or -1
    };
    __device__ static Smem carve(void* lds) {
        Smem m;
        m.pl = static_cast<T2*>(lds);
        m.rowbase = reinterpret_cast<int*>(m.pl + NBUF * BUF);
        m.rowinfo = m.rowbase + 2 * N1;
        m.perm1 = m.rowinfo + 2 * N1;
        m.perm2 = m.perm1 + N1;
        m.colidx = reinterpret_cast<short*>(m.perm2 + N2);
        return m;
    }
    static constexpr size_t bytes() {
        return (size_t)NBUF * BUF * sizeof(T2) + (4 * N1 + N1 + N2) * sizeof(int) +
               (size_t)N1 * N2 * sizeof(short);
    }

    __device__ static int setup(const PlaneTabs& t, int b, const Smem& m) {
        const int nrx = t.nrows_kq[b];
        const int* rx = t.rows_kq[b];
        const short* ci = t.colidx_kq[b];
        for (int i = threadIdx.x; i < N1; i += NT) m.perm1[i] = t.perm1[i];
        for (int i = threadIdx.x; i < N2; i += NT) m.perm2[i] = t.perm2[i];
        if constexpr (ILV) {
            // line l = w + k NW of wave w is spin k % 2 of row pair w + (k / 2) NW
            for (int l = threadIdx.x; l < 2 * N1; l += NT) {
                const int w = l % NW, k = l / NW;
                const int pr = w + (k >> 1) * NW, s = k & 1;
                if (pr < nrx) {
                    const int row = rx[pr];
                    m.rowbase[l] = s * G::PS + row * G::N2P;
                    m.rowinfo[l] = s * N1 + row;
                }
            }
        } else {
            for (int i = threadIdx.x; i < 2 * nrx; i += NT) {
                const int s = i >= nrx;
                const int row = rx[i - s * nrx];
                m.rowbase[i] = s * G::PS + row * G::N2P;
                m.rowinfo[i] = s * N1 + row;
            }
        }
        for (int i = threadIdx.x; i < N1 * N2; i += NT) m.colidx[i] = ci[i];
        __syncthreads();
        return nrx;
    }

    // row lines of wave w among nrl
    __device__ static int wave_rows(int nrl, int w) { return w < nrl ? (nrl - 1 - w) / NW + 1 : 0; }
    // row lines of wave w for nrx occupied rows of each of the two planes
    __device__ static int wave_lines(int nrx, int w) {
        if constexpr (ILV) return 2 * wave_rows(nrx, w);
        return wave_rows(2 * nrx, w);
    }

    static constexpr int FIT = cdiv(MAXR * N2, 64);  // row elements per lane, at most
    static constexpr int FCH = FCH_ < FIT ? FCH_ : FIT;  // of them in flight together
    using Rows = WRows<NW, N2, MAXR, true>;             // line bases in registers (when lane-fixed)

    // row element k = lane + 64 it of the wave: LDS offset within a buffer, and
    // sphere column (spin plane s, column c; c < 0 outside the sphere)
    __device__ static bool row_elem(const Smem& m, int nlw, int w, int lane, int it, int& dst, int& s, int& c) {
        const int k = lane + 64 * it;
        if (k >= nlw * N2) return false;
        const int li = k / N2, p2 = k - li * N2;
        const int l = w + li * NW;
        const int info = m.rowinfo[l];
        s = info / N1;
        const int row = info - s * N1;
        c = m.colidx[row * N2 + p2];
        dst = m.rowbase[l] + p2;
        return true;
    }

    // fill the wave's occupied rows of buffer boff from the z-transformed
    // columns of item pair (2n, 2n+1), then the inverse transforms along i2.
    // FCH > 1: the table reads and column loads of FCH elements are issued
    // before their LDS stores, so that a lane's elements do not wait on each
    // other (more registers); FCH = 1: one element at a time.
    // The row fill fused with the first (DIF) stage of the inverse row
    // transform: the lane of butterfly j of row line li loads that row's
    // elements j + t M (t < R) straight from the z-transformed columns (zero
    // outside the sphere), all of its butterflies' loads in flight together,
    // transforms and twiddles them exactly as the stage does in LDS, and stores
    // the R results; then the remaining stages.
    __device__ static void rows_inverse_fused(const Smem& m, const T2* cx, long long cs, int nlw, int w, int boff,
                                              int lane, const WTw<N2, T2>& gtw2, Rows rl) {
        constexpr CPlan cp = cplan(N2);
        constexpr int R = cp.rad[0];
        constexpr int M = N2 / R;                  // butterflies per line; stage 0 has LB = N2
        constexpr int SPL = wslots(M);
        constexpr int IT = cdiv(MAXR * SPL, 64);
        const int ns = nlw * SPL;
        T2 u[IT][R];
        int base[IT], jv[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int sl = lane + it * 64;
            const int li = sl / SPL, j = sl - li * SPL;
            base[it] = -1;
            jv[it] = j;
            if (sl < ns && j < M) {
                const int l = w + li * NW;
                const int info = m.rowinfo[l];
                const int s = info / N1, row = info - s * N1;
                const short* ci = m.colidx + row * N2;
                base[it] = boff + m.rowbase[l] + j;
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    const int c = ci[j + t * M];
                    u[it][t] = c >= 0 ? cx[s * cs + c] : Cx<T2>::mk(0, 0);
                }
            }
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            if (base[it] >= 0) {
                dft_small<R>(u[it], +1);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    T2 y = u[it][r];
                    if (r > 0 && jv[it] > 0) {
                        T2 wv = gtw2.template get<0, N2>(r, jv[it]);
                        wv.y = -wv.y;
                        y = cmul(y, wv);
                    }
                    m.pl[base[it] + r * M] = y;
                }
            }
        }
        wave_sync();
        rl.boff = boff;
        wfft_dif<N2, +1, false, MAXR, BT, cp.nrad, 1, N2 / R>(m.pl, rl, nlw, gtw2, lane);
    }

    // The fused row fill split in two, for a band's row elements loaded ahead
    // (during the previous band's forward row stage): fill_load issues the
    // loads of the lane's butterflies into registers, fill_finish transforms
    // and stores them into buffer boff exactly as rows_inverse_fused does, then
    // runs the remaining stages.
    struct Fill {
        static constexpr CPlan cp = cplan(N2);
        static constexpr int R = cp.rad[0];
        static constexpr int M = N2 / R;
        static constexpr int SPL = wslots(M);
        static constexpr int IT = cdiv(MAXR * SPL, 64);
        T2 u[IT][R];
        int base[IT], jv[IT];
    };
    __device__ static void fill_load(const Smem& m, const T2* cx, long long cs, int nlw, int w, int lane, Fill& f) {
        constexpr int R = Fill::R, M = Fill::M, SPL = Fill::SPL;
        const int ns = nlw * SPL;
#pragma unroll
        for (int it = 0; it < Fill::IT; ++it) {
            const int sl = lane + it * 64;
            const int li = sl / SPL, j = sl - li * SPL;
            f.base[it] = -1;
            f.jv[it] = j;
            if (sl < ns && j < M) {
                const int l = w + li * NW;
                const int info = m.rowinfo[l];
                const int s = info / N1, row = info - s * N1;
                const short* ci = m.colidx + row * N2;
                f.base[it] = m.rowbase[l] + j;
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    const int c = ci[j + t * M];
                    f.u[it][t] = c >= 0 ? cx[s * cs + c] : Cx<T2>::mk(0, 0);
                }
            }
        }
    }
    __device__ static void fill_finish(const Smem& m, int nlw, int boff, int lane, const WTw<N2, T2>& gtw2, Rows rl,
                                       Fill& f) {
        constexpr int R = Fill::R, M = Fill::M;
#pragma unroll
        for (int it = 0; it < Fill::IT; ++it) {
            if (f.base[it] >= 0) {
                dft_small<R>(f.u[it], +1);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    T2 y = f.u[it][r];
                    if (r > 0 && f.jv[it] > 0) {
                        T2 wv = gtw2.template get<0, N2>(r, f.jv[it]);
                        wv.y = -wv.y;
                        y = cmul(y, wv);
                    }
                    m.pl[boff + f.base[it] + r * M] = y;
                }
            }
        }
        wave_sync();
        rl.boff = boff;
        wfft_dif<N2, +1, false, MAXR, BT, Fill::cp.nrad, 1, N2 / R>(m.pl, rl, nlw, gtw2, lane);
    }

    // The forward row transform of the wave's rows of buffer boff with its last
    // (DIT) stage fused with the output: the lane of butterfly j reads its R
    // inputs from LDS, twiddles and transforms them exactly as the stage does
    // in LDS, and stores the results that lie on the sphere to co.
    __device__ static void rows_forward_out(const Smem& m, T2* co, long long cs, int nlw, int w, int boff, int lane,
                                            const WTw<N2, T2>& gtw2, Rows rl) {
        constexpr CPlan cp = cplan(N2);
        rl.boff = boff;
        wfft_dit<N2, -1, MAXR, BT, cp.nrad - 1, 1>(m.pl, rl, nlw, gtw2, lane);
        constexpr int R = cp.rad[0];
        constexpr int M = N2 / R;
        constexpr int SPL = wslots(M);
        constexpr int IT = cdiv(MAXR * SPL, 64);
        const int ns = nlw * SPL;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int sl = lane + it * 64;
            const int li = sl / SPL, j = sl - li * SPL;
            if (sl < ns && j < M) {
                const int l = w + li * NW;
                const int info = m.rowinfo[l];
                const int s = info / N1, row = info - s * N1;
                const short* ci = m.colidx + row * N2;
                const T2* px = m.pl + boff + m.rowbase[l] + j;
                T2 u[R];
#pragma unroll
                for (int t = 0; t < R; ++t) {
                    T2 x = px[t * M];
                    if (t > 0 && j > 0) x = cmul(x, gtw2.template get<0, N2>(t, j));
                    u[t] = x;
                }
                dft_small<R>(u, -1);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int c = ci[j + r * M];
                    if (c >= 0) co[s * cs + c] = u[r];
                }
            }
        }
    }

    __device__ static void rows_inverse(const Smem& m, const T2* cx, long long cs, int nlw, int w, int boff,
                                        int lane, const WTw<N2, T2>& gtw2, Rows rl) {
        if constexpr (FUSE) {
            rows_inverse_fused(m, cx, cs, nlw, w, boff, lane, gtw2, rl);
            return;
        }
        if constexpr (FCH == 1) {
            for (int k = lane; k < nlw * N2; k += 64) {
                const int li = k / N2, p2 = k - li * N2;
                const int l = w + li * NW;
                const int info = m.rowinfo[l];
                const int s = info / N1, row = info - s * N1;
                const int c = m.colidx[row * N2 + p2];
                m.pl[boff + m.rowbase[l] + p2] = c >= 0 ? cx[s * cs + c] : Cx<T2>::mk(0, 0);
            }
        } else {
#pragma unroll
            for (int i0 = 0; i0 < FIT; i0 += FCH) {
                T2 v[FCH];
                int dst[FCH];
#pragma unroll
                for (int i = 0; i < FCH; ++i) {
                    int s, c;
                    v[i] = Cx<T2>::mk(0, 0);
                    dst[i] = -1;
                    if (i0 + i < FIT && row_elem(m, nlw, w, lane, i0 + i, dst[i], s, c) && c >= 0)
                        v[i] = cx[s * cs + c];
                }
#pragma unroll
                for (int i = 0; i < FCH; ++i)
                    if (dst[i] >= 0) m.pl[boff + dst[i]] = v[i];
            }
        }
        wave_sync();
        rl.boff = boff;
        wfft_dif<N2, +1, false, MAXR, BT>(m.pl, rl, nlw, gtw2, lane);
    }

    // the sphere columns of the wave's rows of buffer boff, to co
    __device__ static void rows_out(const Smem& m, T2* co, long long cs, int nlw, int w, int boff, int lane) {
        for (int k = lane; k < nlw * N2; k += 64) {
            const int li = k / N2, p2 = k - li * N2;
            const int l = w + li * NW;
            const int info = m.rowinfo[l];
            const int s = info / N1, row = info - s * N1;
            const int c = m.colidx[row * N2 + p2];
            if (c >= 0) co[s * cs + c] = m.pl[boff + m.rowbase[l] + p2];
        }
    }
};

// MINW: waves per SIMD the register allocation must leave room for; FCH: row
// elements per lane whose loads are in flight together; EARLY: the band's
// ground-state loads are issued before its row phase instead of after it
// (longer in flight, more registers held through the row stages)
template <int N1, int N2, int BT, int CPW, class T2, int NBUF, int MINW, int FCH, bool FUSE = false,
          bool EARLY = false>
__global__ void __launch_bounds__(64 * (N2 / CPW), MINW) k_density_w(PlaneArgs a, PlaneTabs t) {
    using K = WaveKernel<N1, N2, BT, CPW, T2, NBUF, FCH, FUSE>;
    using G = typename K::G;
    using TL = WTail<N1, N2, CPW>;
    constexpr int R = TL::R, IT = TL::IT;
    extern __shared__ double2 lds[];
    const typename K::Smem m = K::carve(lds);
    const T2* xcols = pick<T2>(a.xcols, a.xcols32);
    // bt: side and k point of the batch; tb: its row in the sphere and slot tables
    const int b = blockIdx.x, i3 = blockIdx.z, bt = b % a.nb2, tb = b % a.tmod;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    WTw<N1, T2> tw1{pick<T2>(t.tw1, t.tw1f)};
    // equal lengths share one table, so the two register sets are one
    WTw<N2, T2> tw2{N1 == N2 ? pick<T2>(t.tw1, t.tw1f) : pick<T2>(t.tw2, t.tw2f)};
    tw1.init(lane);
    tw2.init(lane);
    const int nrx = K::setup(t, tb, m);
    const unsigned long long mask = t.rmask_kq[tb];
    const int nlw = K::wave_lines(nrx, w);
    const long long cs = (long long)a.n3 * a.ncol_max;
    // the side's resident slot, read once (the loop's stores could alias it)
    const double2* ub = a.ureal + (long long)a.uslot[tb] * a.nb * a.n3 * 2 * G::NP + w * K::WPTS;
    TL tl;
    tl.init(w, lane);
    const typename K::Rows rl(m.rowbase, w, nlw, lane);
    const long long N = (long long)G::NP * a.n3;
    // the block's chunks of bands, each summed into its own partial density
    // exactly as when it has a block of its own
    const int ch0 = blockIdx.y * a.cpb, ch1 = min(a.nchunk, ch0 + a.cpb);
    for (int chunk = ch0; chunk < ch1; ++chunk) {
        const int n0 = chunk * a.bpc;
        const int n1e = min(a.nb, n0 + a.bpc);
        T2 acc[4][IT][R];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < IT; ++i)
#pragma unroll
                for (int r = 0; r < R; ++r) acc[c][i][r] = Cx<T2>::mk(0, 0);
        for (int n = n0; n < n1e; ++n) {
            const int boff = NBUF == 2 ? (n & 1) * K::BUF : 0;
            const T2* cx = xcols + (((long long)b * a.nitems + 2 * n) * a.n3 + i3) * a.ncol_max;
            const double2* ur = ub + ((long long)n * a.n3 + i3) * 2 * G::NP;
            // the band's ground state, in flight during the column stages (and
            // with EARLY the row stages)
            T2 uu[IT][R], ud[IT][R];
            auto load_u = [&] {
#pragma unroll
                for (int i = 0; i < IT; ++i)
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        uu[i][r] = Cx<T2>::from(ur[tl.lq[i] + r * TL::BPC]);
                        ud[i][r] = Cx<T2>::from(ur[G::NP + tl.lq[i] + r * TL::BPC]);
                    }
            };
            if constexpr (EARLY) load_u();
            K::rows_inverse(m, cx, cs, nlw, w, boff, lane, tw2, rl);
            __syncthreads();
            if constexpr (!EARLY) load_u();
            typename K::Cols cl{w * CPW, boff, mask};
            wfft_dif<N1, +1, true, 2 * CPW, K::BT, TL::cp.nrad - 1>(m.pl, cl, 2 * CPW, tw1, lane);
            // last inverse stage in registers, then the four density components
#pragma unroll
            for (int i = 0; i < IT; ++i) {
                if (TL::live(lane, i)) {
                    const T2* px = m.pl + boff + tl.lo[i];
                    T2 xu[R], xd[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        xu[r] = px[r * G::N2P];
                        xd[r] = px[G::PS + r * G::N2P];
                    }
                    dft_small<R>(xu, +1);
                    dft_small<R>(xd, +1);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const T2 uu_xu = cmulc(uu[i][r], xu[r]), ud_xd = cmulc(ud[i][r], xd[r]);
                        const T2 uu_xd = cmulc(uu[i][r], xd[r]), ud_xu = cmulc(ud[i][r], xu[r]);
                        acc[0][i][r] = cadd(acc[0][i][r], cadd(uu_xu, ud_xd));
                        acc[1][i][r] = cadd(acc[1][i][r], cadd(uu_xd, ud_xu));
                        acc[2][i][r] = cadd(acc[2][i][r], cmuli(csub(ud_xu, uu_xd)));
                        acc[3][i][r] = cadd(acc[3][i][r], csub(uu_xu, ud_xd));
                    }
                }
            }
            // one buffer: the next band's rows may not overwrite columns still being read
            if (NBUF == 1) __syncthreads();
        }
        T2* out = pick<T2>(a.rho_part, a.rho_part32) + ((long long)b * a.nchunk + chunk) * 4 * N +
                  (long long)i3 * G::NP;
#pragma unroll
        for (int i = 0; i < IT; ++i) {
            if (TL::live(lane, i)) {
                const int sl = lane + 64 * i;
                const int cc = sl / TL::BPC, blk = sl - cc * TL::BPC;
                const int g2 = m.perm2[w * CPW + cc];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int g = m.perm1[blk * R + r] * N2 + g2;
#pragma unroll
                    for (int c = 0; c < 4; ++c) out[c * N + g] = acc[c][i][r];
                }
            }
        }
    }
}

// Local fields, six complex values per point:
//   (v + Bz, v - Bz), (Bx, By), W0 + Wz, W0 - Wz, Wx - i Wy, Wx + i Wy
// (x side; the y side flips the sign of B and of the vector part of W), laid
// out per plane i3 and LDS column p2 as [t][value][blk] for the row
// p1 = R blk + t, so that the lanes holding the butterflies blk of the last
// column stage read 16-lane runs, and a lane's 6 R values sit at small
// constant offsets from one address.
// (right-hand side blockIdx.z: its W and its table, wstride / fstride apart)
template <int N1, int N2, class T2>
__global__ void k_fields_w(const double* __restrict__ vrs, const double2* __restrict__ W, const int* perm1,
                           const int* perm2, T2* __restrict__ F, int n3, long long wstride, long long fstride) {
    constexpr int NP = N1 * N2;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int i3 = blockIdx.y;
    if (idx >= NP) return;
    W += blockIdx.z * wstride;
    F += blockIdx.z * fstride;
    using TL = WTail<N1, N2, 1>;
    const int p2 = idx / N1, r = idx - p2 * N1;
    const int tt = r / TL::BPC, blk = r - tt * TL::BPC;
    const int p1 = blk * TL::R + tt;
    const long long N = (long long)NP * n3;
    const long long g = (long long)i3 * NP + perm1[p1] * N2 + perm2[p2];
    const double v = vrs[g], bx = vrs[N + g], by = vrs[2 * N + g], bz = vrs[3 * N + g];
    const double2 w0 = W[g], wx = W[N + g], wy = W[2 * N + g], wz = W[3 * N + g];
    constexpr int B = TL::BPC;
    T2* f = F + ((long long)i3 * N2 + p2) * 6 * N1 + tt * 6 * B + blk;
    f[0] = Cx<T2>::from(cmk(v + bz, v - bz));
    f[B] = Cx<T2>::from(cmk(bx, by));
    f[2 * B] = Cx<T2>::from(cadd(w0, wz));
    f[3 * B] = Cx<T2>::from(csub(w0, wz));
    f[4 * B] = Cx<T2>::from(csub(wx, cmuli(wy)));
    f[5 * B] = Cx<T2>::from(cadd(wx, cmuli(wy)));
}

// grid: (batch b, chunk, plane i3), so that the blocks in flight share a few
// planes and their field tables stay in L2
// AHEAD (with FUSE): 1, the next band's row elements are loaded during this
// band's forward row stage, so that its row fill does not wait for them (nor,
// the memory counter being in order, for this band's output stores); 2, the
// next band's ground state too, right after this band's products.
template <int N1, int N2, int BT, int CPW, class T2, int NBUF, int MINW, int FCH, bool FUSE = false,
          int AHEAD = 0>
__global__ void __launch_bounds__(64 * (N2 / CPW), MINW) k_apply_w(PlaneArgs a, PlaneTabs t) {
    using K = WaveKernel<N1, N2, BT, CPW, T2, NBUF, FCH, FUSE>;
    using G = typename K::G;
    using TL = WTail<N1, N2, CPW>;
    constexpr int PPL = cdiv(K::WPTS, 64);
    constexpr int B = TL::BPC;
    extern __shared__ double2 lds[];
    const typename K::Smem m = K::carve(lds);
    T2* xcols = pick<T2>(a.xcols, a.xcols32);
    // bt: side and k point of the batch; tb: its row in the sphere and slot tables
    const int b = blockIdx.x, i3 = blockIdx.z, bt = b % a.nb2, tb = b % a.tmod;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    WTw<N1, T2> tw1{pick<T2>(t.tw1, t.tw1f)};
    // equal lengths share one table, so the two register sets are one
    WTw<N2, T2> tw2{N1 == N2 ? pick<T2>(t.tw1, t.tw1f) : pick<T2>(t.tw2, t.tw2f)};
    tw1.init(lane);
    tw2.init(lane);
    const int nrx = K::setup(t, tb, m);
    const unsigned long long mask = t.rmask_kq[tb];
    const int nlw = K::wave_lines(nrx, w);
    // the bands of the block's chunks (the apply of a band does not depend on its chunk)
    const int n0 = blockIdx.y * a.cpb * a.bpc;
    const int n1e = min(a.nb, n0 + a.cpb * a.bpc);
    const long long cs = (long long)a.n3 * a.ncol_max;
    // the side's resident slot, read once (the loop's stores could alias it)
    const double2* ub = a.ureal + (long long)a.uslot[tb] * a.nb * a.n3 * 2 * G::NP + w * K::WPTS;
    const bool yside = bt >= a.nk;
    // the lane's points q = lane + 64 j of the wave (column cc, row position
    // r = t B + blk in the point order): LDS offset, and field table offset
    int o[PPL], fo[PPL];
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
        const int q = min(lane + 64 * j, K::WPTS - 1);
        const int cc = q / N1, r = q - cc * N1;
        const int tt = r / B, blk = r - tt * B;
        o[j] = (blk * TL::R + tt) * G::N2P + w * CPW + cc;
        fo[j] = cc * 6 * N1 + tt * 6 * B + blk;
    }
    const T2* fw = pick<T2>(a.fields, a.fields32) + (long long)(b / a.nb2) * a.fstride +
                   ((long long)i3 * N2 + w * CPW) * 6 * N1;
    const typename K::Rows rl(m.rowbase, w, nlw, lane);
    static_assert(!AHEAD || FUSE, "row elements loaded ahead need the fused row fill");
    typename K::Fill fill;
    // AHEAD 2: the next band's ground state at the lane's points, loaded ahead
    T2 nu[PPL], nd[PPL];
    auto load_next_u = [&](int n) {
        const double2* ur = ub + ((long long)n * a.n3 + i3) * 2 * G::NP;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            const int q = min(lane + 64 * j, K::WPTS - 1);
            nu[j] = Cx<T2>::from(ur[q]);
            nd[j] = Cx<T2>::from(ur[G::NP + q]);
        }
    };
    if constexpr (AHEAD > 0)
        if (n0 < n1e)
            K::fill_load(m, xcols + (((long long)b * a.nitems + 2 * n0) * a.n3 + i3) * a.ncol_max, cs, nlw, w, lane,
                         fill);
    if constexpr (AHEAD > 1)
        if (n0 < n1e) load_next_u(n0);
    for (int n = n0; n < n1e; ++n) {
        const int boff = NBUF == 2 ? (n & 1) * K::BUF : 0;
        const T2* cx = xcols + (((long long)b * a.nitems + 2 * n) * a.n3 + i3) * a.ncol_max;
        const double2* ur = ub + ((long long)n * a.n3 + i3) * 2 * G::NP;
        T2 uu[PPL], ud[PPL];
        if constexpr (AHEAD > 1) {
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                uu[j] = nu[j];
                ud[j] = nd[j];
            }
        } else {
#pragma unroll
            for (int j = 0; j < PPL; ++j) {
                const int q = lane + 64 * j;
                if (q < K::WPTS) {
                    uu[j] = Cx<T2>::from(ur[q]);
                    ud[j] = Cx<T2>::from(ur[G::NP + q]);
                }
            }
        }
        if constexpr (AHEAD > 0)
            K::fill_finish(m, nlw, boff, lane, tw2, rl, fill);
        else
            K::rows_inverse(m, cx, cs, nlw, w, boff, lane, tw2, rl);
        __syncthreads();
        // columns: inverse along i1, point-wise products, forward along i1
        typename K::Cols cl{w * CPW, boff, mask};
        wfft_dif<N1, +1, true, 2 * CPW, K::BT>(m.pl, cl, 2 * CPW, tw1, lane);
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
            const int q = lane + 64 * j;
            if (q < K::WPTS) {
                const T2* f = fw + fo[j];
                T2 f0 = f[0], f1 = f[B], f2 = f[2 * B], f3 = f[3 * B], f4 = f[4 * B], f5 = f[5 * B];
                if (yside) {  // B -> -B, W -> (W0, -W)
                    f0 = Cx<T2>::mk(f0.y, f0.x);
                    f1 = Cx<T2>::mk(-f1.x, -f1.y);
                    const T2 t2 = f2;
                    f2 = f3;
                    f3 = t2;
                    f4 = Cx<T2>::mk(-f4.x, -f4.y);
                    f5 = Cx<T2>::mk(-f5.x, -f5.y);
                }
                T2* px = m.pl + boff + o[j];
                const T2 xu = px[0], xd = px[G::PS];
                const T2 bm = Cx<T2>::mk(f1.x, -f1.y), bp = f1;
                T2 pu = cadd(cscale(xu, f0.x), cmul(bm, xd));
                T2 pd = cadd(cscale(xd, f0.y), cmul(bp, xu));
                pu = cadd(pu, cadd(cmul(f2, uu[j]), cmul(f4, ud[j])));
                pd = cadd(pd, cadd(cmul(f3, ud[j]), cmul(f5, uu[j])));
                px[0] = pu;
                px[G::PS] = pd;
            }
        }
        if constexpr (AHEAD > 1)
            if (n + 1 < n1e) load_next_u(n + 1);
        wave_sync();
        constexpr CPlan c1 = cplan(N1);
        wfft_dit<N1, -1, 2 * CPW, K::BT, c1.nrad - 1>(m.pl, cl, 2 * CPW, tw1, lane);
        __syncthreads();
        // rows: forward along i2 on the occupied rows of the k+q sphere, then
        // the output columns
        T2* co = xcols + (((long long)b * a.nitems + 2 * n) * a.n3 + i3) * a.ncol_max;
        if constexpr (AHEAD > 0)
            if (n + 1 < n1e) K::fill_load(m, co + 2 * a.n3 * a.ncol_max, cs, nlw, w, lane, fill);
        if constexpr (K::FUSE) {
            K::rows_forward_out(m, co, cs, nlw, w, boff, lane, tw2, rl);
        } else {
            constexpr CPlan c2 = cplan(N2);
            typename K::Rows rlb = rl;
            rlb.boff = boff;
            wfft_dit<N2, -1, K::MAXR, K::BT, c2.nrad - 1>(m.pl, rlb, nlw, tw2, lane);
            K::rows_out(m, co, cs, nlw, w, boff, lane);
        }
        // no barrier here: with two buffers the next band works in the other
        // one; with one, each wave rewrites only the rows it has just finished
    }
}

enum PlaneOp { kOpDensity = 0, kOpApply = 1, kOpUreal = 2 };

template <class F>
void launch_with_lds(F kernel, const char* name, size_t shm, dim3 grid, int nt, hipStream_t st, PlaneArgs a,
                     PlaneTabs t) {
    TM_CHECK(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) ==
                 hipSuccess,
             TM_EDEVICE, std::string("cannot raise the LDS limit of ") + name);
    ProfScope ps(name, st);
    void* args[] = {&a, &t};
    TM_CHECK(hipLaunchKernel((const void*)kernel, grid, dim3(nt), args, shm, st) == hipSuccess, TM_EDEVICE,
             std::string("launch of ") + name + " failed");
    check_launch(name);
}

// Variants of the FP64 wave plane kernels that the autotuner times, variant 0
// being the hand-picked default: BT butterflies per load group, CPW columns
// per wave, FCH row elements in flight per lane, fused first / last row
// stages, loads issued ahead (the density: a band's ground state before its
// row phase; the apply: the next band's row elements during this band's
// forward row stage; all with two LDS buffers and no occupancy floor).  They
// split the work differently and do the same arithmetic per point in the same
// order, so their results are identical.
template <int N1, int N2>
struct WaveVariants {  // 8x8, 24x24, 32x32
    static constexpr int n = 3;
    static constexpr int bt[n] = {2, 1, 2}, cpw[n] = {4, 4, 4}, fch[n] = {1, 1, 1};
    static constexpr bool fuse[n] = {false, false, true};
    static constexpr int ahead[n] = {0, 0, 0};
};
template <>
struct WaveVariants<48, 48> {
    static constexpr int n = 9;
    static constexpr int bt[n] = {2, 1, 4, 2, 2, 1, 1, 2, 1}, cpw[n] = {4, 4, 4, 4, 4, 4, 4, 4, 4},
                         fch[n] = {1, 1, 1, 4, 1, 1, 1, 1, 1}, ahead[n] = {0, 0, 0, 0, 0, 0, 1, 1, 2};
    static constexpr bool fuse[n] = {false, false, false, false, true, true, true, true, true};
};
template <>
struct WaveVariants<20, 20> {
    static constexpr int n = 5;
    static constexpr int bt[n] = {2, 2, 1, 2, 2}, cpw[n] = {5, 4, 5, 10, 5}, fch[n] = {1, 1, 1, 1, 1};
    static constexpr bool fuse[n] = {false, false, false, false, true};
    static constexpr int ahead[n] = {0, 0, 0, 0, 0};
};

template <int N1, int N2, int V>
void launch_wave_one(bool density, const PlaneArgs& a, const PlaneTabs& t, dim3 wgrid, hipStream_t st) {
    using VV = WaveVariants<N1, N2>;
    constexpr int BT = VV::bt[V], CPW = VV::cpw[V], FCH = VV::fch[V];
    constexpr bool FU = VV::fuse[V];
    constexpr int AH = VV::ahead[V];
    using K = WaveKernel<N1, N2, BT, CPW, double2, 2, FCH, FU>;
    if (density)
        launch_with_lds(k_density_w<N1, N2, BT, CPW, double2, 2, 1, FCH, FU, (AH > 0)>, "k_density_w", K::bytes(),
                        wgrid, K::NT, st, a, t);
    else
        launch_with_lds(k_apply_w<N1, N2, BT, CPW, double2, 2, 1, FCH, FU, AH>, "k_apply_w", K::bytes(), wgrid,
                        K::NT, st, a, t);
}

// launches variant v (0 .. V) of the FP64 density or apply
template <int N1, int N2, int V>
void launch_wave_v(bool density, int v, const PlaneArgs& a, const PlaneTabs& t, dim3 wgrid, hipStream_t st, int) {
    if constexpr (V >= 0) {
        if (v == V) return launch_wave_one<N1, N2, V>(density, a, t, wgrid, st);
        launch_wave_v<N1, N2, V - 1>(density, v, a, t, wgrid, st, 0);
    }
}

// NT: threads of the block-synchronous kernels (column path, builder)
template <int N1, int N2, int NT>
void launch_t(int op, const PlaneArgs& a, const PlaneTabs& t, dim3 grid, hipStream_t st, bool fp32) {
    // FP64: the variants of WaveVariants, picked per shape by the autotuner
    // (defaults: 4 columns per wave, 12 waves for 48 x 48 -- 3 columns and 16
    // waves measured slower: idle lanes in the column stages and register
    // spills at 128 VGPRs; one buffer with 6 or 8 columns, or 6 waves per SIMD,
    // spill in FP64; 20 x 20 planes: 5 columns per wave).  Single precision
    // (fixed): the apply at 48 x 48 runs 6 columns per wave and 4 waves per
    // SIMD (2 blocks per CU in 2 x 81 KB of LDS, no spills): 7 % faster; the
    // density's row fill keeps all of a lane's loads in flight together
    // (FCH = 64, 10 % faster at 48 x 48); the 6-column apply would spill with it.
    constexpr int CPW32 = N2 == 20 ? 5 : 4, CPWA32 = N2 == 48 ? 6 : N2 == 20 ? 5 : 4;
    constexpr int BTD = 2, BTA = N2 == 48 ? 1 : 2;  // 48: two butterflies per load group spill at 128 registers
    constexpr int NBUF32 = 2, MINW32 = 1, MINWA32 = N2 == 48 ? 4 : 1;
    constexpr int FCHD32 = 64, FCHA32 = 1;
    if (op == kOpUreal) {
        launch_with_lds(k_ureal_t<N1, N2, NT>, "k_ureal_t", PlaneKernel<N1, N2, NT, kU>::bytes(), grid, NT, st, a, t);
    } else if (a.ureal) {
        TM_CHECK(t.colidx_kq != nullptr, TM_EINVAL, "missing column index tables");
        // several chunks of bands per block once the grid has blocks to spare
        // (their set-up -- tables, twiddle registers -- is then shared), as
        // long as about 2048 blocks remain; the results do not change
        PlaneArgs aw = a;
        const long long blocks = (long long)grid.x * grid.y * grid.z;
        aw.cpb = (int)std::max<long long>(1, std::min<long long>(a.nchunk, blocks / 2048));
        const dim3 wgrid(grid.z, (a.nchunk + aw.cpb - 1) / aw.cpb, grid.x);  // (b, chunk group, i3)
        const int nrhs = (int)grid.z / a.nb2;
        if (fp32) {
            using WD = WaveKernel<N1, N2, BTD, CPW32, float2, NBUF32>;
            using WA = WaveKernel<N1, N2, BTA, CPWA32, float2, NBUF32>;
            if (op == kOpDensity) {
                launch_with_lds(k_density_w<N1, N2, BTD, CPW32, float2, NBUF32, MINW32, FCHD32>, "k_density_w32",
                                WD::bytes(), wgrid, WD::NT, st, aw, t);
            } else {
                TM_LAUNCH((k_fields_w<N1, N2, float2>), dim3((N1 * N2 + 255) / 256, a.n3, nrhs), dim3(256), 0, st,
                          a.vrs, a.W, t.perm1, t.perm2, a.fields32, a.n3, a.wstride, a.fstride);
                launch_with_lds(k_apply_w<N1, N2, BTA, CPWA32, float2, NBUF32, MINWA32, FCHA32>, "k_apply_w32",
                                WA::bytes(), wgrid, WA::NT, st, aw, t);
            }
            return;
        }
        // FP64: the variant the autotuner picked for this shape (plane, planes,
        // bands and sides, and the size class of the right-hand side count)
        const long long key = tune_key(N1 * 1000 + N2, a.n3, a.nb, a.nb2 * 64 + rhs_class(nrhs));
        if (op == kOpDensity) {
            constexpr int NV = WaveVariants<N1, N2>::n;
            launch_wave_v<N1, N2, NV - 1>(true, tune_pick(kTuneDensity, key, NV), aw, t, wgrid, st, nrhs);
        } else {
            TM_CHECK(a.fields != nullptr, TM_EINVAL, "missing field table");
            TM_LAUNCH((k_fields_w<N1, N2, double2>), dim3((N1 * N2 + 255) / 256, a.n3, nrhs), dim3(256), 0, st,
                      a.vrs, a.W, t.perm1, t.perm2, a.fields, a.n3, a.wstride, a.fstride);
            constexpr int NV = WaveVariants<N1, N2>::n;
            launch_wave_v<N1, N2, NV - 1>(false, tune_pick(kTuneApply, key, NV), aw, t, wgrid, st, nrhs);
        }
    } else {
        TM_CHECK(!fp32, TM_EUNSUPPORTED, "single-precision plane kernels need the resident ground state");
        if (op == kOpDensity)
            launch_with_lds(k_density_t<N1, N2, NT>, "k_density_t", PlaneKernel<N1, N2, NT, kXU>::bytes(), grid, NT,
                            st, a, t);
        else
            launch_with_lds(k_apply_t<N1, N2, NT>, "k_apply_t", PlaneKernel<N1, N2, NT, kXU>::bytes(), grid, NT, st,
                            a, t);
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

template <int N3, int NT, int CT, int IT, class T2>
__global__ void __launch_bounds__(NT) k_zinv_t(ZPassArgs a) {
    constexpr int L = CT * IT;
    constexpr int LS = N3 + 1;
    extern __shared__ double2 lds_raw[];
    T2* lds = reinterpret_cast<T2*>(lds_raw);
    T2* tw = lds + L * LS;
    const T2* gtw = pick<T2>(a.tw, a.tw32);
    int* perm = reinterpret_cast<int*>(tw + N3);
    const int b = blockIdx.z, bt = b % a.nb2;
    const int ncol = a.ncol[bt];
    const int col0 = blockIdx.x * CT;
    if (col0 >= ncol) return;
    const int item0 = blockIdx.y * IT;
    for (int i = threadIdx.x; i < N3; i += NT) {
        tw[i] = gtw[i];
        perm[i] = a.perm[i];
    }
    for (int i = threadIdx.x; i < L * LS; i += NT) lds[i] = Cx<T2>::mk(0, 0);
    __syncthreads();
    const int* cp = a.colptr[bt];
    const int* eg = a.entg[bt];
    const int* ei = a.enti3[bt];
    const double2* coef = a.coef_table ? a.coef_table[bt] : a.coef_base + (long long)b * a.coef_bstride;
    const long long istr = a.istride_tab ? a.istride_tab[bt] : a.istride;
    constexpr int PER = NT / L > 0 ? NT / L : 1;
    for (int l = threadIdx.x / PER; l < L; l += NT / PER) {
        const int c = col0 + l % CT, item = item0 + l / CT;
        if (c < ncol && item < a.nitems) {
            const double2* src = coef + (long long)item * istr;
            for (int e = cp[c] + threadIdx.x % PER; e < cp[c + 1]; e += PER)
                lds[l * LS + ei[e]] = Cx<T2>::from(src[eg[e]]);
        }
    }
    __syncthreads();
    fft_dif<N3, +1, NT, false>(lds, L, ZLines<LS>{}, tw);
    T2* out = pick<T2>(a.cols, a.cols32) + (long long)b * a.nitems * N3 * a.ncol_stride;
    for (int i = threadIdx.x; i < L * N3; i += NT) {
        const int cl = i % CT, rest = i / CT;
        const int p = rest % N3, il = rest / N3;
        const int c = col0 + cl, item = item0 + il;
        if (c < ncol && item < a.nitems)
            out[((long long)item * N3 + perm[p]) * a.ncol_stride + c] = lds[(il * CT + cl) * LS + p];
    }
}

template <int N3, int NT, int CT, int IT, class T2>
__global__ void __launch_bounds__(NT) k_zfwd_t(ZPassArgs a) {
    constexpr int L = CT * IT;
    constexpr int LS = N3 + 1;
    extern __shared__ double2 lds_raw[];
    T2* lds = reinterpret_cast<T2*>(lds_raw);
    T2* tw = lds + L * LS;
    const T2* gtw = pick<T2>(a.tw, a.tw32);
    int* perm = reinterpret_cast<int*>(tw + N3);
    const int b = blockIdx.z, bt = b % a.nb2;
    const int ncol = a.ncol[bt];
    const int col0 = blockIdx.x * CT;
    const int item0 = blockIdx.y * IT;
    const long long bbase = (long long)b * a.nitems * a.npw_pad;
    if (blockIdx.x == 0) {  // the first column tile clears the padding of its items
        const int npw = a.npw[bt], padn = a.npw_pad - npw;
        for (int i = threadIdx.x; i < IT * padn; i += NT) {
            const int item = item0 + i / padn;
            if (item < a.nitems) a.out[bbase + (long long)item * a.npw_pad + npw + i % padn] = cmk(0.0, 0.0);
        }
    }
    if (col0 >= ncol) return;
    for (int i = threadIdx.x; i < N3; i += NT) {
        tw[i] = gtw[i];
        perm[i] = a.perm[i];
    }
    __syncthreads();
    const T2* cin = pick<T2>(a.cols, a.cols32) + (long long)b * a.nitems * N3 * a.ncol_stride;
    for (int i = threadIdx.x; i < L * N3; i += NT) {
        const int cl = i % CT, rest = i / CT;
        const int p = rest % N3, il = rest / N3;
        const int c = col0 + cl, item = item0 + il;
        T2 v = Cx<T2>::mk(0, 0);
        if (c < ncol && item < a.nitems) v = cin[((long long)item * N3 + perm[p]) * a.ncol_stride + c];
        lds[(il * CT + cl) * LS + p] = v;
    }
    __syncthreads();
    fft_dit_all<N3, -1, NT>(lds, L, ZLines<LS>{}, tw);
    const int* cp = a.colptr[bt];
    const int* eg = a.entg[bt];
    const int* ei = a.enti3[bt];
    const double* kin = a.kin[bt];
    const double* eps = a.eps[bt];
    constexpr int PER = NT / L > 0 ? NT / L : 1;
    for (int l = threadIdx.x / PER; l < L; l += NT / PER) {
        const int c = col0 + l % CT, item = item0 + l / CT;
        if (c < ncol && item < a.nitems) {
            const double e = eps[item >> 1];
            const long long off = bbase + (long long)item * a.npw_pad;
            for (int en = cp[c] + threadIdx.x % PER; en < cp[c + 1]; en += PER) {
                const int g = eg[en];
                const double2 f = cscale(Cx<double2>::from(lds[l * LS + ei[en]]), a.inv_n);
                const double2 x = a.xin[off + g];
                const double s = kin[g] - e;
                a.out[off + g] = cmk(f.x + s * x.x, f.y + s * x.y);
            }
        }
    }
}

// A pointer read from a pointer table, as a global-memory pointer: the
// compiler cannot tell the address space of such a pointer once the kernel
// has stored to global memory, and would issue flat loads through it, whose
// pending count also holds up LDS operations.
template <class T>
__device__ __forceinline__ const T __attribute__((address_space(1)))* gptr(const T* p) {
    return (const T __attribute__((address_space(1)))*)p;
}

// digit-reversed position -> natural index of the in-place transforms of
// length N (the radix plan's digits reversed; the same map as the host table)
template <int N>
__device__ __forceinline__ int dperm(int pos) {
    constexpr CPlan cp = cplan(N);
    int rem = pos, k = 0, weight = 1, place = N;
#pragma unroll
    for (int s = 0; s < cp.nrad; ++s) {
        place /= cp.rad[s];
        const int d = rem / place;
        rem -= d * place;
        k += d * weight;
        weight *= cp.rad[s];
    }
    return k;
}

// The z passes with every global load of a tile issued up front.  A thread
// owns a fixed share of one line's sphere entries (at most EPT of them, the
// loop fully unrolled), so the table reads, the coefficient gathers and (in
// the forward pass) the vector and kinetic-energy reads of all of them are
// in flight together instead of one dependent chain per entry; the digit
// reversal of a line position is computed, not read.  Same per-line
// arithmetic as k_zinv_t / k_zfwd_t, so the results are identical.
template <int N3, int NT, int CT, int IT, class T2>
__global__ void __launch_bounds__(NT) k_zinv_p(ZPassArgs a) {
    constexpr int L = CT * IT;
    constexpr int LS = N3 + 1;
    static_assert(NT % L == 0, "a line's entries take NT / L threads");
    constexpr int PER = NT / L;
    constexpr int EPT = cdiv(N3, PER);  // a column holds at most N3 entries
    extern __shared__ double2 lds_raw[];
    T2* lds = reinterpret_cast<T2*>(lds_raw);
    T2* tw = lds + L * LS;
    const T2* gtw = pick<T2>(a.tw, a.tw32);
    const int b = blockIdx.z, bt = b % a.nb2;
    const int ncol = a.ncol[bt];
    const int col0 = blockIdx.x * CT;
    if (col0 >= ncol) return;
    const int item0 = blockIdx.y * IT;
    const int l = threadIdx.x / PER, sub = threadIdx.x - l * PER;
    const int c = col0 + l % CT, item = item0 + l / CT;
    const bool live = c < ncol && item < a.nitems;
    int e0 = 0, e1 = 0;
    if (live) {
        const int* cp = a.colptr[bt];
        e0 = cp[c];
        e1 = cp[c + 1];
    }
    const int* eg = a.entg[bt];
    const int* ei = a.enti3[bt];
    int g[EPT], z[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int en = e0 + sub + k * PER;
        g[k] = -1;
        if (en < e1) {
            g[k] = eg[en];
            z[k] = ei[en];
        }
    }
    const double2* coef = a.coef_table ? a.coef_table[bt] : a.coef_base + (long long)b * a.coef_bstride;
    const long long istr = a.istride_tab ? a.istride_tab[bt] : a.istride;
    const double2* src = coef + (long long)item * istr;
    double2 v[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k)
        if (g[k] >= 0) v[k] = src[g[k]];
    // while the gathers are in flight: twiddles and the zero lines
    for (int i = threadIdx.x; i < N3; i += NT) tw[i] = gtw[i];
    for (int i = threadIdx.x; i < L * LS; i += NT) lds[i] = Cx<T2>::mk(0, 0);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < EPT; ++k)
        if (g[k] >= 0) lds[l * LS + z[k]] = Cx<T2>::from(v[k]);
    __syncthreads();
    fft_dif<N3, +1, NT, false>(lds, L, ZLines<LS>{}, tw);
    T2* out = pick<T2>(a.cols, a.cols32) + (long long)b * a.nitems * N3 * a.ncol_stride;
    for (int i = threadIdx.x; i < L * N3; i += NT) {
        const int cl = i % CT, rest = i / CT;
        const int p = rest % N3, il = rest / N3;
        const int cc = col0 + cl, it = item0 + il;
        if (cc < ncol && it < a.nitems)
            out[((long long)it * N3 + dperm<N3>(p)) * a.ncol_stride + cc] = lds[(il * CT + cl) * LS + p];
    }
}

template <int N3, int NT, int CT, int IT, class T2>
__global__ void __launch_bounds__(NT) k_zfwd_p(ZPassArgs a) {
    constexpr int L = CT * IT;
    constexpr int LS = N3 + 1;
    static_assert(NT % L == 0, "a line's entries take NT / L threads");
    constexpr int PER = NT / L;
    constexpr int EPT = cdiv(N3, PER);
    constexpr int VPT = cdiv(L * N3, NT);  // line values per thread
    extern __shared__ double2 lds_raw[];
    T2* lds = reinterpret_cast<T2*>(lds_raw);
    T2* tw = lds + L * LS;
    const T2* gtw = pick<T2>(a.tw, a.tw32);
    const int b = blockIdx.z, bt = b % a.nb2;
    const int ncol = a.ncol[bt];
    const int col0 = blockIdx.x * CT;
    const int item0 = blockIdx.y * IT;
    const long long bbase = (long long)b * a.nitems * a.npw_pad;
    if (blockIdx.x == 0) {  // the first column tile clears the padding of its items
        const int npw = a.npw[bt], padn = a.npw_pad - npw;
        for (int i = threadIdx.x; i < IT * padn; i += NT) {
            const int item = item0 + i / padn;
            if (item < a.nitems) a.out[bbase + (long long)item * a.npw_pad + npw + i % padn] = cmk(0.0, 0.0);
        }
    }
    if (col0 >= ncol) return;
    // the tile's column values (a line position's natural index computed in registers)
    const T2* cin = pick<T2>(a.cols, a.cols32) + (long long)b * a.nitems * N3 * a.ncol_stride;
    T2 v[VPT];
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
        const int i = threadIdx.x + j * NT;
        v[j] = Cx<T2>::mk(0, 0);
        if (i < L * N3) {
            const int cl = i % CT, rest = i / CT;
            const int p = rest % N3, il = rest / N3;
            const int cc = col0 + cl, it = item0 + il;
            if (cc < ncol && it < a.nitems) v[j] = cin[((long long)it * N3 + dperm<N3>(p)) * a.ncol_stride + cc];
        }
    }
    // the thread's sphere entries: table rows, then the input vector and the kinetic energies
    const int l = threadIdx.x / PER, sub = threadIdx.x - l * PER;
    const int c = col0 + l % CT, item = item0 + l / CT;
    const bool live = c < ncol && item < a.nitems;
    int e0 = 0, e1 = 0;
    double e = 0.0;
    if (live) {
        const auto cp = gptr(a.colptr[bt]);
        e0 = cp[c];
        e1 = cp[c + 1];
        e = gptr(a.eps[bt])[item >> 1];
    }
    const auto eg = gptr(a.entg[bt]);
    const auto ei = gptr(a.enti3[bt]);
    int g[EPT], z[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int en = e0 + sub + k * PER;
        g[k] = -1;
        if (en < e1) {
            g[k] = eg[en];
            z[k] = ei[en];
        }
    }
    const auto kin = gptr(a.kin[bt]);
    const long long off = bbase + (long long)item * a.npw_pad;
    double2 x[EPT];
    double kv[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k)
        if (g[k] >= 0) {
            x[k] = a.xin[off + g[k]];
            kv[k] = kin[g[k]];
        }
    for (int i = threadIdx.x; i < N3; i += NT) tw[i] = gtw[i];
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
        const int i = threadIdx.x + j * NT;
        if (i < L * N3) {
            const int cl = i % CT, rest = i / CT;
            const int p = rest % N3, il = rest / N3;
            lds[(il * CT + cl) * LS + p] = v[j];
        }
    }
    __syncthreads();
    fft_dit_all<N3, -1, NT>(lds, L, ZLines<LS>{}, tw);
#pragma unroll
    for (int k = 0; k < EPT; ++k)
        if (g[k] >= 0) {
            const double2 f = cscale(Cx<double2>::from(lds[l * LS + z[k]]), a.inv_n);
            const double s = kv[k] - e;
            a.out[off + g[k]] = cmk(f.x + s * x[k].x, f.y + s * x[k].y);
        }
}

template <int N3, int NT, int CT, int IT, bool PF = false>
void launch_z(bool inverse, const ZPassArgs& a, int ncolmax, int nbatch, hipStream_t st, bool fp32) {
    constexpr int L = CT * IT;
    const size_t esz = fp32 ? sizeof(float2) : sizeof(double2);
    const size_t shm = (size_t)L * (N3 + 1) * esz + N3 * esz + N3 * sizeof(int);
    dim3 grid((ncolmax + CT - 1) / CT, (a.nitems + IT - 1) / IT, nbatch);
    auto lds = [&](const void* fn) {  // above 64 KB the limit must be raised first
        if (shm > 65536)
            TM_CHECK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) == hipSuccess,
                     TM_EDEVICE, "cannot raise the LDS limit of a z pass");
    };
    if (fp32) {
        TM_CHECK(a.cols32 != nullptr && a.tw32 != nullptr, TM_EINVAL, "missing single-precision buffers");
        if (inverse) {
            lds((const void*)k_zinv_t<N3, NT, CT, IT, float2>);
            TM_LAUNCH((k_zinv_t<N3, NT, CT, IT, float2>), grid, dim3(NT), shm, st, a);
        } else {
            lds((const void*)k_zfwd_t<N3, NT, CT, IT, float2>);
            TM_LAUNCH((k_zfwd_t<N3, NT, CT, IT, float2>), grid, dim3(NT), shm, st, a);
        }
    } else if constexpr (PF) {
        if (inverse) {
            lds((const void*)k_zinv_p<N3, NT, CT, IT, double2>);
            TM_LAUNCH((k_zinv_p<N3, NT, CT, IT, double2>), grid, dim3(NT), shm, st, a);
        } else {
            lds((const void*)k_zfwd_p<N3, NT, CT, IT, double2>);
            TM_LAUNCH((k_zfwd_p<N3, NT, CT, IT, double2>), grid, dim3(NT), shm, st, a);
        }
    } else if (inverse) {
        lds((const void*)k_zinv_t<N3, NT, CT, IT, double2>);
        TM_LAUNCH((k_zinv_t<N3, NT, CT, IT, double2>), grid, dim3(NT), shm, st, a);
    } else {
        lds((const void*)k_zfwd_t<N3, NT, CT, IT, double2>);
        TM_LAUNCH((k_zfwd_t<N3, NT, CT, IT, double2>), grid, dim3(NT), shm, st, a);
    }
}

}  // namespace

bool zpass_fixed_supported(int n3) {
    return n3 == 8 || n3 == 20 || n3 == 24 || n3 == 32 || n3 == 48 || n3 == 96 || n3 == 180;
}

// Launch shapes of the fixed-length z passes (threads NT, columns CT and items
// IT per block; P: the prefetching kernels) that the autotuner times.
// Variant 0 is the default, taken untuned and in single precision: a
// prefetching shape that measured well in both directions for 20, 24, 32, 96
// and 180.  Every line is transformed alike, so the results are identical.
// Longer lines: more waves per CU pay (the passes wait on memory, one block
// per tile of lines), and so does prefetching: on the 48 x 48 x 180 slab
// 3.5 ms inverse (P 512 / 16 / 1) and 3.7 ms forward (P 256 / 8 / 1) against
// 4.6 and 5.9 ms for 256 / 16 / 1.  (128 / 16 / 1, 512 / 32 / 1 and 128 / 8 /
// 1 never won at 180.)
namespace {
template <int N3, int NT, int CT, int IT, bool PF = false>
struct ZV {};
template <int N3, class... V>
struct ZVariants {
    static constexpr int n = sizeof...(V);
};

template <int N3, int NT, int CT, int IT, bool PF, class... Rest>
void launch_z_v(int v, bool inverse, const ZPassArgs& a, int ncolmax, int nbatch, hipStream_t st, bool fp32,
                ZV<N3, NT, CT, IT, PF>, Rest... rest) {
    if (v == 0) return launch_z<N3, NT, CT, IT, PF>(inverse, a, ncolmax, nbatch, st, fp32);
    if constexpr (sizeof...(Rest) > 0) launch_z_v(v - 1, inverse, a, ncolmax, nbatch, st, fp32, rest...);
}

template <class... V>
void launch_z_tuned(bool inverse, const ZPassArgs& a, int ncolmax, int nbatch, int n3, hipStream_t st, bool fp32,
                    V... vs) {
    constexpr int n = sizeof...(V);
    // single precision keeps the default; FP64 takes the tuned variant of this shape
    const int v = fp32 ? 0 : tune_pick(inverse ? kTuneZInv : kTuneZFwd, tune_key(n3, ncolmax, nbatch, a.nitems), n);
    launch_z_v(v, inverse, a, ncolmax, nbatch, st, fp32, vs...);
}
}  // namespace

void launch_zpass_fixed(bool inverse, const ZPassArgs& a, int ncolmax, int nbatch, int n3, hipStream_t st,
                        bool fp32) {
    switch (n3) {
        case 8: launch_z_tuned(inverse, a, ncolmax, nbatch, n3, st, fp32, ZV<8, 256, 16, 4>{}, ZV<8, 128, 16, 2>{}); break;
        case 20:
            launch_z_tuned(inverse, a, ncolmax, nbatch, n3, st, fp32, ZV<20, 128, 16, 1, true>{}, ZV<20, 128, 16, 1>{},
                           ZV<20, 256, 16, 4>{}, ZV<20, 64, 16, 1>{}, ZV<20, 256, 16, 4, true>{});
            break;
        case 24:
            launch_z_tuned(inverse, a, ncolmax, nbatch, n3, st, fp32, ZV<24, 256, 16, 1, true>{}, ZV<24, 256, 16, 4>{},
                           ZV<24, 128, 16, 2>{}, ZV<24, 256, 16, 4, true>{});
            break;
        case 32:
            launch_z_tuned(inverse, a, ncolmax, nbatch, n3, st, fp32, ZV<32, 256, 16, 1, true>{}, ZV<32, 256, 16, 2>{},
                           ZV<32, 128, 16, 1>{}, ZV<32, 256, 16, 2, true>{});
            break;
        case 48: launch_z_tuned(inverse, a, ncolmax, nbatch, n3, st, fp32, ZV<48, 256, 16, 2>{}, ZV<48, 128, 16, 1>{}); break;
        case 96:
            launch_z_tuned(inverse, a, ncolmax, nbatch, n3, st, fp32, ZV<96, 256, 8, 1, true>{}, ZV<96, 256, 16, 1>{},
                           ZV<96, 128, 16, 1>{}, ZV<96, 512, 32, 1>{}, ZV<96, 256, 8, 1>{}, ZV<96, 512, 16, 1>{},
                           ZV<96, 512, 8, 1>{}, ZV<96, 512, 8, 1, true>{}, ZV<96, 512, 16, 1, true>{});
            break;
        case 180:
            launch_z_tuned(inverse, a, ncolmax, nbatch, n3, st, fp32, ZV<180, 256, 8, 1, true>{},
                           ZV<180, 256, 16, 1>{}, ZV<180, 256, 8, 1>{}, ZV<180, 512, 16, 1>{}, ZV<180, 512, 8, 1>{},
                           ZV<180, 512, 8, 1, true>{}, ZV<180, 512, 16, 1, true>{});
            break;
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

static void launch_plane_op(int op, const PlaneArgs& a, const PlaneTabs& t, dim3 grid, int n1, int n2,
                            hipStream_t st, bool fp32) {
    if (n1 == 8 && n2 == 8) launch_t<8, 8, 64>(op, a, t, grid, st, fp32);
    else if (n1 == 20 && n2 == 20) launch_t<20, 20, 256>(op, a, t, grid, st, fp32);
    else if (n1 == 24 && n2 == 24) launch_t<24, 24, 256>(op, a, t, grid, st, fp32);
    else if (n1 == 32 && n2 == 32) launch_t<32, 32, 512>(op, a, t, grid, st, fp32);
    else if (n1 == 48 && n2 == 48) launch_t<48, 48, 1024>(op, a, t, grid, st, fp32);
    else throw Error{TM_EUNSUPPORTED, "no fixed-size plane kernel for this grid"};
}

void launch_plane_fixed(bool density, const PlaneArgs& a, const PlaneTabs& t, dim3 grid, int n1, int n2,
                        hipStream_t st, bool fp32) {
    launch_plane_op(density ? kOpDensity : kOpApply, a, t, grid, n1, n2, st, fp32);
}

void launch_ureal_fixed(const PlaneArgs& a, const PlaneTabs& t, dim3 grid, int n1, int n2, hipStream_t st) {
    TM_CHECK(a.ureal != nullptr && a.uslot != nullptr, TM_EINVAL, "no resident ground-state buffer");
    launch_plane_op(kOpUreal, a, t, grid, n1, n2, st, false);
}

}  // namespace tml

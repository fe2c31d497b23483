// Sphere <-> column transforms (the z direction of the 3D FFTs) and the
// full-grid 3D FFT used by the response Hartree potential.
//
// A spinor component on its plane-wave sphere is first scattered into the
// (m1, m2) columns it occupies and transformed along i3 here; the plane
// kernels in apply.hip finish the transform in the (i1, i2) planes.  Column
// buffers are laid out [batch][item][i3][column] so a plane kernel reads all
// columns of one plane contiguously.
#include "fft_lds.h"
#include "plane.h"

namespace tml {

namespace {

constexpr int kZThreads = 256;

struct ZArgs {
    // per batch b (side*nk + ik, plus 2nk per further right-hand side):
    // coefficients of item 0 at coef_table[b % nb2] when the table is given,
    // else at coef_base + b * coef_bstride; sphere tables are per b % nb2
    // (nb2: the table period, 2 nk or 2 nk times the right-hand sides when
    // each has its own q set)
    int nb2;
    const double2* const* coef_table;
    const double2* coef_base;
    long long coef_bstride;
    long long coef_item_stride;   // complex elements between items
    const int* coef_item_stride_tab;  // per-batch item stride (overrides when non-null)
    const int* const* colptr;
    const int* const* entg;
    const int* const* enti3;
    const int* ncol;
    double2* cols;                // [b][item][n3][ncol_stride]
    int ncol_stride;
    int nitems;
    int lines_per_block;          // CT * IT
    int ct;                       // columns per block
};

__global__ void __launch_bounds__(kZThreads) k_zpass_inv(ZArgs a, FFTPlan pl) {
    extern __shared__ double2 lds[];
    const int n3 = pl.n;
    const int b = blockIdx.z, bt = b % a.nb2;
    const int ncol = a.ncol[bt];
    const int col0 = blockIdx.x * a.ct;
    if (col0 >= ncol) return;
    const int it = a.lines_per_block / a.ct;
    const int item0 = blockIdx.y * it;
    const int L = a.lines_per_block;
    for (int i = threadIdx.x; i < L * n3; i += blockDim.x) lds[i] = cmk(0.0, 0.0);
    __syncthreads();
    const int* cp = a.colptr[bt];
    const int* eg = a.entg[bt];
    const int* ei = a.enti3[bt];
    const double2* coef = a.coef_table ? a.coef_table[bt] : a.coef_base + (long long)b * a.coef_bstride;
    // scatter: each (line, entry) pair by one thread
    const int per = (blockDim.x + L - 1) / L;
    for (int l = threadIdx.x / per; l < L; l += blockDim.x / per) {
        int c = col0 + (l % a.ct);
        int item = item0 + l / a.ct;
        if (c < ncol && item < a.nitems) {
            const long long istr = a.coef_item_stride_tab ? a.coef_item_stride_tab[bt] : a.coef_item_stride;
            const double2* src = coef + (long long)item * istr;
            for (int e = cp[c] + (threadIdx.x % per); e < cp[c + 1]; e += per)
                lds[l * n3 + ei[e]] = src[eg[e]];
        }
    }
    __syncthreads();
    lds_fft(lds, L, n3, 1, pl, +1);
    double2* out = a.cols + (long long)b * a.nitems * n3 * a.ncol_stride;
    for (int i = threadIdx.x; i < L * n3; i += blockDim.x) {
        int cl = i % a.ct;
        int rest = i / a.ct;
        int i3 = rest % n3;
        int il = rest / n3;
        int c = col0 + cl;
        int item = item0 + il;
        if (c < ncol && item < a.nitems)
            out[((long long)item * n3 + i3) * a.ncol_stride + c] = lds[(il * a.ct + cl) * n3 + i3];
    }
}

struct ZFwdArgs {
    int nb2;                      // sphere tables are per b % nb2 (see ZArgs)
    const double2* cols;          // [b][item][n3][ncol_stride]
    int ncol_stride;
    const int* const* colptr;
    const int* const* entg;
    const int* const* enti3;
    const int* ncol;
    const int* npw;
    const double* const* kin;     // [b] -> [npw_pad]
    const double* const* eps;     // [b] -> [nb]
    const double2* xin;           // BR input vector
    double2* out;                 // BR output vector
    int npw_pad;
    int nitems;                   // nb * 2
    int lines_per_block;
    int ct;
    double inv_n;
};

__global__ void __launch_bounds__(kZThreads) k_zpass_fwd(ZFwdArgs a, FFTPlan pl) {
    extern __shared__ double2 lds[];
    const int n3 = pl.n;
    const int b = blockIdx.z, bt = b % a.nb2;
    const int ncol = a.ncol[bt];
    const int col0 = blockIdx.x * a.ct;
    const int it = a.lines_per_block / a.ct;
    const int item0 = blockIdx.y * it;
    const int L = a.lines_per_block;
    const long long bbase = (long long)b * a.nitems * a.npw_pad;
    // the first column tile also clears the padding of its items
    if (blockIdx.x == 0) {
        int npw = a.npw[bt];
        int padn = a.npw_pad - npw;
        for (int i = threadIdx.x; i < it * padn; i += blockDim.x) {
            int item = item0 + i / padn;
            if (item < a.nitems) a.out[bbase + (long long)item * a.npw_pad + npw + i % padn] = cmk(0.0, 0.0);
        }
    }
    if (col0 >= ncol) return;
    const double2* cin = a.cols + (long long)b * a.nitems * n3 * a.ncol_stride;
    for (int i = threadIdx.x; i < L * n3; i += blockDim.x) {
        int cl = i % a.ct;
        int rest = i / a.ct;
        int i3 = rest % n3;
        int il = rest / n3;
        int c = col0 + cl;
        int item = item0 + il;
        double2 v = cmk(0.0, 0.0);
        if (c < ncol && item < a.nitems) v = cin[((long long)item * n3 + i3) * a.ncol_stride + c];
        lds[(il * a.ct + cl) * n3 + i3] = v;
    }
    __syncthreads();
    lds_fft(lds, L, n3, 1, pl, -1);
    const int* cp = a.colptr[bt];
    const int* eg = a.entg[bt];
    const int* ei = a.enti3[bt];
    const double* kin = a.kin[bt];
    const double* eps = a.eps[bt];
    const int per = (blockDim.x + L - 1) / L;
    for (int l = threadIdx.x / per; l < L; l += blockDim.x / per) {
        int c = col0 + (l % a.ct);
        int item = item0 + l / a.ct;
        if (c < ncol && item < a.nitems) {
            double e = eps[item >> 1];
            long long off = bbase + (long long)item * a.npw_pad;
            for (int en = cp[c] + (threadIdx.x % per); en < cp[c + 1]; en += per) {
                int g = eg[en];
                double2 f = cscale(lds[l * n3 + ei[en]], a.inv_n);
                double2 x = a.xin[off + g];
                double s = kin[g] - e;
                a.out[off + g] = cmk(f.x + s * x.x, f.y + s * x.y);
            }
        }
    }
}

// Batched strided line FFT over a full grid: line l starts at
// (l / inner) * outer_stride + (l % inner) * inner_stride, element t at + t*estride.
__global__ void __launch_bounds__(kZThreads) k_fft_lines(double2* data, int nlines, int inner, long long outer_stride,
                                                         long long inner_stride, long long estride, int lpb,
                                                         FFTPlan pl, int sign) {
    extern __shared__ double2 lds[];
    const int n = pl.n;
    const int l0 = blockIdx.x * lpb;
    // element-major loads: consecutive threads take consecutive lines
    for (int i = threadIdx.x; i < lpb * n; i += blockDim.x) {
        int ll = i % lpb, t = i / lpb;
        int l = l0 + ll;
        if (l < nlines) {
            long long base = (long long)(l / inner) * outer_stride + (long long)(l % inner) * inner_stride;
            lds[ll * n + t] = data[base + t * estride];
        }
    }
    __syncthreads();
    lds_fft(lds, lpb, n, 1, pl, sign);
    for (int i = threadIdx.x; i < lpb * n; i += blockDim.x) {
        int ll = i % lpb, t = i / lpb;
        int l = l0 + ll;
        if (l < nlines) {
            long long base = (long long)(l / inner) * outer_stride + (long long)(l % inner) * inner_stride;
            data[base + t * estride] = lds[ll * n + t];
        }
    }
}

int lines_for(int n, int cap_lines, int threads) {
    // lines per block such that every radix pass fits kMaxBfly butterflies per thread
    int L = cap_lines;
    while (L > 1 && (long long)L * n / 2 > (long long)kMaxBfly * threads) L /= 2;
    return L;
}

}  // namespace

void launch_zpass_inv(const System& s, const QSet& q, bool ucols, const double2* coef, long long coef_bstride,
                      int nitems, int item_stride, double2* cols, hipStream_t st, bool fp32, int nrhs) {
    const int nb2 = 2 * q.nk;
    TM_CHECK(nrhs == 1 || !ucols, TM_EINVAL, "ground-state columns have one right-hand side");
    ZArgs a;
    a.nb2 = q.tmod;  // the table period
    a.nitems = nitems;
    a.coef_item_stride = item_stride;
    if (ucols) {
        a.coef_table = q.d_ucoef;
        a.coef_item_stride_tab = q.d_npw_u;
        a.coef_base = nullptr;
        a.coef_bstride = 0;
        a.colptr = q.d_colptr_u;
        a.entg = q.d_entg_u;
        a.enti3 = q.d_enti3_u;
        a.ncol = q.d_ncol_u;
        a.ncol_stride = q.ncol_u_max;
    } else {
        a.coef_table = nullptr;
        a.coef_item_stride_tab = nullptr;
        a.coef_base = coef;
        a.coef_bstride = coef_bstride;
        a.colptr = q.d_colptr_kq;
        a.entg = q.d_entg_kq;
        a.enti3 = q.d_enti3_kq;
        a.ncol = q.d_ncol_kq;
        a.ncol_stride = q.ncol_max;
    }
    a.cols = cols;
    const int n3 = s.n3;
    int ncolmax = ucols ? q.ncol_u_max : q.ncol_max;
    if (zpass_fixed_supported(n3)) {
        ZPassArgs z{};
        z.nb2 = q.tmod;
        z.coef_table = a.coef_table;
        z.coef_base = a.coef_base;
        z.coef_bstride = a.coef_bstride;
        z.istride = a.coef_item_stride;
        z.istride_tab = a.coef_item_stride_tab;
        z.colptr = a.colptr;
        z.entg = a.entg;
        z.enti3 = a.enti3;
        z.ncol = a.ncol;
        z.cols = cols;
        z.ncol_stride = a.ncol_stride;
        z.nitems = nitems;
        z.tw = s.plan[2].tw;
        z.tw32 = s.twf[2];
        z.cols32 = reinterpret_cast<float2*>(cols);
        z.perm = s.perm[2];
        launch_zpass_fixed(true, z, ncolmax, nb2 * nrhs, n3, st, fp32);
        return;
    }
    TM_CHECK(!fp32, TM_EUNSUPPORTED, "single-precision z passes need a fixed-size grid length");
    int L = lines_for(n3, 64, kZThreads);
    a.ct = L >= 16 ? 16 : L;
    a.lines_per_block = L;
    int it = L / a.ct;
    dim3 grid((ncolmax + a.ct - 1) / a.ct, (nitems + it - 1) / it, nb2 * nrhs);
    size_t shm = (size_t)L * n3 * sizeof(double2);
    TM_LAUNCH(k_zpass_inv, grid, dim3(kZThreads), shm, st, a, s.plan[2]);
}

void launch_zpass_fwd(const System& s, const QSet& q, const double2* cols, const double2* xin, double2* out,
                      hipStream_t st, bool fp32, int nrhs) {
    ZFwdArgs a;
    a.nb2 = q.tmod;  // the table period
    a.cols = cols;
    a.ncol_stride = q.ncol_max;
    a.colptr = q.d_colptr_kq;
    a.entg = q.d_entg_kq;
    a.enti3 = q.d_enti3_kq;
    a.ncol = q.d_ncol_kq;
    a.npw = q.d_npw_kq;
    a.kin = q.d_kin;
    a.eps = q.d_eps;
    a.xin = xin;
    a.out = out;
    a.npw_pad = q.npw_pad;
    a.nitems = 2 * s.nbnd;
    const int n3 = s.n3;
    if (zpass_fixed_supported(n3)) {
        ZPassArgs z{};
        z.nb2 = q.tmod;
        z.colptr = a.colptr;
        z.entg = a.entg;
        z.enti3 = a.enti3;
        z.ncol = a.ncol;
        z.cols = const_cast<double2*>(cols);
        z.ncol_stride = q.ncol_max;
        z.nitems = a.nitems;
        z.tw = s.plan[2].tw;
        z.perm = s.perm[2];
        z.npw = a.npw;
        z.kin = a.kin;
        z.eps = a.eps;
        z.xin = xin;
        z.out = out;
        z.npw_pad = q.npw_pad;
        z.inv_n = 1.0 / (double)s.N;
        z.tw32 = s.twf[2];
        z.cols32 = reinterpret_cast<float2*>(const_cast<double2*>(cols));
        launch_zpass_fixed(false, z, q.ncol_max, 2 * q.nk * nrhs, n3, st, fp32);
        return;
    }
    TM_CHECK(!fp32, TM_EUNSUPPORTED, "single-precision z passes need a fixed-size grid length");
    int L = lines_for(n3, 64, kZThreads);
    a.ct = L >= 16 ? 16 : L;
    a.lines_per_block = L;
    a.inv_n = 1.0 / (double)s.N;
    int it = L / a.ct;
    dim3 grid((q.ncol_max + a.ct - 1) / a.ct, (a.nitems + it - 1) / it, 2 * q.nk * nrhs);
    size_t shm = (size_t)L * n3 * sizeof(double2);
    TM_LAUNCH(k_zpass_fwd, grid, dim3(kZThreads), shm, st, a, s.plan[2]);
}

// data: plane-major [i3][i1][i2]
// nrhs grids of N points back to back: the lines of every grid in one launch per axis
void launch_fft3d_full(const System& s, double2* data, int sign, hipStream_t st, int nrhs) {
    const int n1 = s.n1, n2 = s.n2, n3 = s.n3;
    const long long NP = (long long)n1 * n2;
    struct Pass {
        int n, axis;
    } passes[3] = {{n2, 1}, {n1, 0}, {n3, 2}};
    for (auto& p : passes) {
        int L = lines_for(p.n, 64, kZThreads);
        int nlines, inner;
        long long outer_stride, inner_stride, estride;
        const FFTPlan* pl;
        // (the grid index counts as an outer index: planes follow planes)
        if (p.axis == 1) {  // along i2: lines (grid, i3, i1)
            nlines = nrhs * n3 * n1; inner = n1; outer_stride = NP; inner_stride = n2; estride = 1; pl = &s.plan[1];
        } else if (p.axis == 0) {  // along i1: lines (grid, i3, i2)
            nlines = nrhs * n3 * n2; inner = n2; outer_stride = NP; inner_stride = 1; estride = n2; pl = &s.plan[0];
        } else {  // along i3: lines (grid, p) over the plane points
            nlines = nrhs * (int)NP; inner = (int)NP; outer_stride = NP * n3; inner_stride = 1; estride = NP;
            pl = &s.plan[2];
        }
        dim3 grid((nlines + L - 1) / L);
        size_t shm = (size_t)L * p.n * sizeof(double2);
        TM_LAUNCH(k_fft_lines, grid, dim3(kZThreads), shm, st, data, nlines, inner, outer_stride,
                           inner_stride, estride, L, *pl, sign);
    }
}

}  // namespace tml

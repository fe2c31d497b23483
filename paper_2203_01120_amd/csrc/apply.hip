// Plane kernels of the Liouvillian and the response potential.
//
// Phase A (k_density): for one (i1, i2) plane at fixed i3, one batch
// (side, k) and a chunk of bands, finish the inverse FFT of the response
// spinor x_n and of the ground-state spinor u_n (u'_n = T U_{n,-k} on the Y
// side), and accumulate the four response densities of
// Eqs. charge_dens_resp_q / spin_dens_resp_q,
//     rho'_a += u^dag S_a x,   S = (sigma_0, sigma_x, sigma_y, sigma_z),
// in registers; one partial per block, summed deterministically afterwards
// with the side signs s_a = (+, -, -, -) on the Y side and the 1/(Omega Nk)
// weight.
//
// Phase B: response Hartree potential 4 pi rho'_0(G) / |G+q|^2 (Eq. v_H_q) by
// a full-grid FFT, plus the local ALSDA kernel (Eqs. v_XC_q, b_XC_q):
//     W_a = delta_a0 v'_H + sum_b f_ab rho'_b,   V' = W_0 sigma_0 + W . sigma.
//
// Phase C (k_apply_planes): per band, rebuild x_n and u_n on the plane, form
//     phi = V0 x + V' u,   V0 = v_eff sigma_0 + sg B . sigma,  V' = W_0 + sg W . sigma
// (sg = -1 on the Y side: H+ and V'+ flip the magnetic parts, Sec. 2.2), and
// transform phi forward back to the columns of the k+q sphere.
#include "fft_lds.h"
#include "plane.h"

namespace tml {

namespace {

constexpr int kPts = 4;  // grid points per thread in the plane kernels

// scatter one column set into the zeroed plane and inverse-transform it
__device__ inline void plane_inverse(double2* plane, const double2* cols, const int* colpos, int ncol,
                                     const PlaneArgs& a, const FFTPlan& p1, const FFTPlan& p2) {
    for (int i = threadIdx.x; i < a.NP; i += blockDim.x) plane[i] = cmk(0.0, 0.0);
    __syncthreads();
    for (int c = threadIdx.x; c < ncol; c += blockDim.x) plane[colpos[c]] = cols[c];
    __syncthreads();
    lds_fft(plane, a.n1, a.n2, 1, p2, +1);  // along i2 for every i1
    lds_fft(plane, a.n2, 1, a.n2, p1, +1);  // along i1 for every i2
}

// b: batch (columns of x); bt = b % nb2: side and k point (u columns and
// tables of the q set); tb = b % tmod: the k+q sphere tables
__device__ inline void load_components(double2 (&val)[4][kPts], double2* plane, int b, int bt, int tb, int n,
                                       int i3, const PlaneArgs& a, const FFTPlan& p1, const FFTPlan& p2) {
    const int* cpos_x = a.colpos_kq[tb];
    const int ncx = a.ncol_kq[tb];
    const int* cpos_u = a.colpos_u[bt];
    const int ncu = a.ncol_u[bt];
#pragma unroll
    for (int comp = 0; comp < 4; ++comp) {
        const double2* cols;
        if (comp < 2)
            cols = a.xcols + (((long long)b * a.nitems + 2 * n + comp) * a.n3 + i3) * a.ncol_max;
        else
            cols = a.ucols + (((long long)bt * a.nitems + 2 * n + comp - 2) * a.n3 + i3) * a.ncol_u_max;
        plane_inverse(plane, cols, comp < 2 ? cpos_x : cpos_u, comp < 2 ? ncx : ncu, a, p1, p2);
#pragma unroll
        for (int j = 0; j < kPts; ++j) {
            int pt = threadIdx.x + j * blockDim.x;
            val[comp][j] = pt < a.NP ? plane[pt] : cmk(0.0, 0.0);
        }
        __syncthreads();
    }
    if (bt >= a.nk) {  // Y side: u' = T U_{-k} = i sigma_y K U: (a, b) -> (conj b, -conj a)
#pragma unroll
        for (int j = 0; j < kPts; ++j) {
            double2 up = val[2][j], dn = val[3][j];
            val[2][j] = cconj(dn);
            val[3][j] = cmk(-up.x, up.y);
        }
    }
}

__global__ void k_density(PlaneArgs a, FFTPlan p1, FFTPlan p2) {
    extern __shared__ double2 plane[];
    const int i3 = blockIdx.x, chunk = blockIdx.y, b = blockIdx.z, bt = b % a.nb2, tb = b % a.tmod;
    const int n0 = chunk * a.bpc;
    const int n1e = min(a.nb, n0 + a.bpc);
    double2 acc[4][kPts];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int j = 0; j < kPts; ++j) acc[c][j] = cmk(0.0, 0.0);
    for (int n = n0; n < n1e; ++n) {
        double2 val[4][kPts];
        load_components(val, plane, b, bt, tb, n, i3, a, p1, p2);
#pragma unroll
        for (int j = 0; j < kPts; ++j) {
            double2 xu = val[0][j], xd = val[1][j], uu = val[2][j], ud = val[3][j];
            double2 uu_xu = cmulc(uu, xu), ud_xd = cmulc(ud, xd);
            double2 uu_xd = cmulc(uu, xd), ud_xu = cmulc(ud, xu);
            acc[0][j] = cadd(acc[0][j], cadd(uu_xu, ud_xd));
            acc[1][j] = cadd(acc[1][j], cadd(uu_xd, ud_xu));
            // u^dag sigma_y x = -i uu* xd + i ud* xu = i (ud* xu - uu* xd)
            acc[2][j] = cadd(acc[2][j], cmuli(csub(ud_xu, uu_xd)));
            acc[3][j] = cadd(acc[3][j], csub(uu_xu, ud_xd));
        }
    }
    const long long N = (long long)a.NP * a.n3;
    double2* out = a.rho_part + ((long long)b * a.nchunk + chunk) * 4 * N + (long long)i3 * a.NP;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int j = 0; j < kPts; ++j) {
            int pt = threadIdx.x + j * blockDim.x;
            if (pt < a.NP) out[c * N + pt] = acc[c][j];
        }
}

// right-hand side blockIdx.y: its 2 nk batches of partials -> its rho [4][N]
template <class T2>
__global__ void k_density_reduce(const T2* part, double2* rho, long long N, int nk, int nchunk, double scale) {
    long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 4 * N) return;
    part += (long long)blockIdx.y * 2 * nk * nchunk * 4 * N;
    rho += (long long)blockIdx.y * 4 * N;
    int comp = (int)(idx / N);
    long long p = idx - comp * N;
    double2 sx = cmk(0.0, 0.0), sy = cmk(0.0, 0.0);
    for (int b = 0; b < 2 * nk; ++b)
        for (int c = 0; c < nchunk; ++c) {
            double2 v = Cx<double2>::from(part[(((long long)b * nchunk + c) * 4 + comp) * N + p]);
            if (b < nk) sx = cadd(sx, v); else sy = cadd(sy, v);
        }
    double sgn = comp == 0 ? 1.0 : -1.0;
    rho[idx] = cscale(cmk(sx.x + sgn * sy.x, sx.y + sgn * sy.y), scale);
}

// Right-hand side blockIdx.y: its rho (4 N), its scratch grid (N) and its W (4 N).
// the charge component of rho into the scratch grid
__global__ void k_copy_scale(const double2* rho, double2* dst, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    rho += blockIdx.y * 4 * n;
    dst += blockIdx.y * n;
    if (i < n) dst[i] = rho[i];
}

// right-hand side blockIdx.y times its multiplier hqt[blockIdx.y % hmod]
__global__ void k_mul_real(double2* data, const double* const* hqt, int hmod, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    data += blockIdx.y * n;
    const double* h = hqt[blockIdx.y % hmod];
    if (i < n) data[i] = cscale(data[i], h[i]);
}

// W_a = delta_a0 vH + sum_b f_ab rho_b with f stored as (00,01,02,03,11,12,13,22,23,33)
__global__ void k_assemble_W(const double2* rho, const double2* vH, const double* fxc, double2* W, long long N) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    rho += blockIdx.y * 4 * N;
    vH += blockIdx.y * N;
    W += blockIdx.y * 4 * N;
    if (i >= N) return;
    double f[10];
#pragma unroll
    for (int t = 0; t < 10; ++t) f[t] = fxc[t * N + i];
    double2 r0 = rho[i], r1 = rho[N + i], r2 = rho[2 * N + i], r3 = rho[3 * N + i];
    auto comb = [&](double a0, double a1, double a2, double a3) {
        return cmk(a0 * r0.x + a1 * r1.x + a2 * r2.x + a3 * r3.x, a0 * r0.y + a1 * r1.y + a2 * r2.y + a3 * r3.y);
    };
    W[i] = cadd(vH[i], comb(f[0], f[1], f[2], f[3]));
    W[N + i] = comb(f[1], f[4], f[5], f[6]);
    W[2 * N + i] = comb(f[2], f[5], f[7], f[8]);
    W[3 * N + i] = comb(f[3], f[6], f[8], f[9]);
}

__global__ void k_apply_planes(PlaneArgs a, FFTPlan p1, FFTPlan p2) {
    extern __shared__ double2 plane[];
    const int i3 = blockIdx.x, chunk = blockIdx.y, b = blockIdx.z, bt = b % a.nb2, tb = b % a.tmod;
    const int n0 = chunk * a.bpc;
    const int n1e = min(a.nb, n0 + a.bpc);
    const double sg = bt < a.nk ? 1.0 : -1.0;
    const long long N = (long long)a.NP * a.n3;
    const long long off = (long long)i3 * a.NP;
    const double2* Wr = a.W + (long long)(b / a.nb2) * a.wstride;
    // local fields of my points
    double v[kPts], Bx[kPts], By[kPts], Bz[kPts];
    double2 W0[kPts], Wx[kPts], Wy[kPts], Wz[kPts];
#pragma unroll
    for (int j = 0; j < kPts; ++j) {
        int pt = threadIdx.x + j * blockDim.x;
        if (pt < a.NP) {
            long long g = off + pt;
            v[j] = a.vrs[g];
            Bx[j] = sg * a.vrs[N + g];
            By[j] = sg * a.vrs[2 * N + g];
            Bz[j] = sg * a.vrs[3 * N + g];
            W0[j] = Wr[g];
            Wx[j] = cscale(Wr[N + g], sg);
            Wy[j] = cscale(Wr[2 * N + g], sg);
            Wz[j] = cscale(Wr[3 * N + g], sg);
        } else {
            v[j] = Bx[j] = By[j] = Bz[j] = 0.0;
            W0[j] = Wx[j] = Wy[j] = Wz[j] = cmk(0.0, 0.0);
        }
    }
    const int* cpos = a.colpos_kq[bt];
    const int ncx = a.ncol_kq[bt];
    for (int n = n0; n < n1e; ++n) {
        double2 val[4][kPts];
        load_components(val, plane, b, bt, tb, n, i3, a, p1, p2);
        double2 phi[2][kPts];
#pragma unroll
        for (int j = 0; j < kPts; ++j) {
            double2 xu = val[0][j], xd = val[1][j], uu = val[2][j], ud = val[3][j];
            // V0 x: v x + (Bz xu + (Bx - i By) xd,  (Bx + i By) xu - Bz xd)
            double2 bm = cmk(Bx[j], -By[j]), bp = cmk(Bx[j], By[j]);
            double2 pu = cadd(cscale(xu, v[j] + Bz[j]), cmul(bm, xd));
            double2 pd = cadd(cscale(xd, v[j] - Bz[j]), cmul(bp, xu));
            // V' u with complex W: W0 u + (Wz uu + (Wx - i Wy) ud, (Wx + i Wy) uu - Wz ud)
            double2 wm = csub(Wx[j], cmuli(Wy[j])), wp = cadd(Wx[j], cmuli(Wy[j]));
            pu = cadd(pu, cadd(cmul(cadd(W0[j], Wz[j]), uu), cmul(wm, ud)));
            pd = cadd(pd, cadd(cmul(csub(W0[j], Wz[j]), ud), cmul(wp, uu)));
            phi[0][j] = pu;
            phi[1][j] = pd;
        }
#pragma unroll
        for (int spin = 0; spin < 2; ++spin) {
#pragma unroll
            for (int j = 0; j < kPts; ++j) {
                int pt = threadIdx.x + j * blockDim.x;
                if (pt < a.NP) plane[pt] = phi[spin][j];
            }
            __syncthreads();
            lds_fft(plane, a.n2, 1, a.n2, p1, -1);  // along i1 for every i2
            lds_fft(plane, a.n1, a.n2, 1, p2, -1);  // along i2 for every i1
            double2* cols = a.xcols + (((long long)b * a.nitems + 2 * n + spin) * a.n3 + i3) * a.ncol_max;
            for (int c = threadIdx.x; c < ncx; c += blockDim.x) cols[c] = plane[cpos[c]];
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- setup kernels

// ALSDA Slater-exchange kernel from the ground-state density (Eqs. v_XC_q, b_XC_q):
//   e(n, s) with n_up/dn = (n +- s)/2, v_s = -(6/pi)^{1/3} n_s^{1/3}, g_s = dv_s/dn_s,
//   f_nn = f_ss = (g_up + g_dn)/4, f_ns = (g_up - g_dn)/4, transverse (v_up - v_dn)/(2s).
__global__ void k_fxc(const double* rho, double* fxc, long long N) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double NMIN = 1e-10, SREL = 1e-10, NSIG_MIN = 1e-12;
    const double cx = cbrt(6.0 / M_PI);
    double n = rho[i], mx = rho[N + i], my = rho[2 * N + i], mz = rho[3 * N + i];
    double f[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (n >= NMIN) {
        double s = sqrt(mx * mx + my * my + mz * mz);
        double nu = fmax(0.5 * (n + s), 0.0), nd = fmax(0.5 * (n - s), 0.0);
        double vu = -cx * cbrt(nu), vd = -cx * cbrt(nd);
        double gu = -(cx / 3.0) * pow(fmax(nu, NSIG_MIN), -2.0 / 3.0);
        double gd = -(cx / 3.0) * pow(fmax(nd, NSIG_MIN), -2.0 / 3.0);
        double enn = 0.25 * (gu + gd), ess = 0.25 * (gu + gd), ens = 0.25 * (gu - gd);
        double h[3] = {0, 0, 0};
        double ts;
        if (s >= SREL * n) {
            h[0] = mx / s; h[1] = my / s; h[2] = mz / s;
            ts = 0.5 * (vu - vd) / s;
        } else {
            ts = ess;
            ens = 0.0;
        }
        f[0] = enn;
        f[1] = ens * h[0]; f[2] = ens * h[1]; f[3] = ens * h[2];
        int t = 4;
        for (int p = 0; p < 3; ++p)
            for (int q = p; q < 3; ++q) f[t++] = ess * h[p] * h[q] + ts * ((p == q ? 1.0 : 0.0) - h[p] * h[q]);
    }
    for (int t = 0; t < 10; ++t) fxc[t * N + i] = f[t];
}

// 4 pi / |G+q|^2 / N on the plane-major grid; 0 on Nyquist planes and at G+q = 0
__global__ void k_coulomb(double* h, int n1, int n2, int n3, double3 b1, double3 b2, double3 b3, double3 q,
                          double invN) {
    long long N = (long long)n1 * n2 * n3;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int i3 = (int)(i / ((long long)n1 * n2));
    int rem = (int)(i - (long long)i3 * n1 * n2);
    int i1 = rem / n2, i2 = rem % n2;
    auto canon = [](int ii, int n) { return ii < (n + 1) / 2 ? ii : ii - n; };
    bool nyq = ((n1 % 2 == 0) && i1 == n1 / 2) || ((n2 % 2 == 0) && i2 == n2 / 2) || ((n3 % 2 == 0) && i3 == n3 / 2);
    int m1 = canon(i1, n1), m2 = canon(i2, n2), m3 = canon(i3, n3);
    double gx = m1 * b1.x + m2 * b2.x + m3 * b3.x + q.x;
    double gy = m1 * b1.y + m2 * b2.y + m3 * b3.y + q.y;
    double gz = m1 * b1.z + m2 * b2.z + m3 * b3.z + q.z;
    double k2 = gx * gx + gy * gy + gz * gz;
    h[i] = (!nyq && k2 > 1e-12) ? 4.0 * M_PI / k2 * invN : 0.0;
}

// |p + G|^2 / 2 for the sphere of a point (Miller indices of the point itself)
__global__ void k_kin(double* kin, const int* mill, int npw, int npw_pad, double3 p, double3 b1, double3 b2,
                      double3 b3) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npw_pad) return;
    if (g >= npw) {
        kin[g] = 0.0;
        return;
    }
    int m1 = mill[3 * g], m2 = mill[3 * g + 1], m3 = mill[3 * g + 2];
    double x = p.x + m1 * b1.x + m2 * b2.x + m3 * b3.x;
    double y = p.y + m1 * b1.y + m2 * b2.y + m3 * b3.y;
    double z = p.z + m1 * b1.z + m2 * b2.z + m3 * b3.z;
    kin[g] = 0.5 * (x * x + y * y + z * z);
}

PlaneArgs plane_args(const System& s, const QSet& q) {
    PlaneArgs a;
    a.n1 = s.n1; a.n2 = s.n2; a.n3 = s.n3; a.NP = s.n1 * s.n2;
    a.nk = q.nk; a.nb = s.nbnd; a.nitems = 2 * s.nbnd;
    a.nb2 = 2 * q.nk;
    a.tmod = q.tmod;
    a.wstride = 4 * s.N;
    a.fstride = 6 * s.N;
    a.nchunk = s.ws.nchunk;
    a.bpc = (s.nbnd + a.nchunk - 1) / a.nchunk;
    a.cpb = 1;
    a.xcols = s.ws.xcols;
    a.ncol_max = q.ncol_max;
    a.ucols = q.ucols;
    a.ncol_u_max = q.ncol_u_max;
    a.colpos_kq = q.d_colpos_kq;
    a.ncol_kq = q.d_ncol_kq;
    a.colpos_u = q.d_colpos_u;
    a.ncol_u = q.d_ncol_u;
    a.rho_part = s.ws.rho_part;
    a.vrs = s.vrs;
    a.W = s.ws.W;
    a.ureal = s.ureal_mode == 1 ? s.ureal : nullptr;
    a.uslot = q.d_uslot;
    a.fields = s.ws.fields;
    a.xcols32 = reinterpret_cast<float2*>(s.ws.xcols);
    a.rho_part32 = reinterpret_cast<float2*>(s.ws.rho_part);
    a.fields32 = reinterpret_cast<float2*>(s.ws.fields);
    return a;
}

int plane_threads(const System& s) {
    int NP = s.n1 * s.n2;
    int t = ((NP + kPts - 1) / kPts + 63) / 64 * 64;
    return t < 64 ? 64 : t;
}

}  // namespace

int plane_threads_for(int n1, int n2) {
    int NP = n1 * n2;
    int t = ((NP + kPts - 1) / kPts + 63) / 64 * 64;
    return t < 64 ? 64 : t;
}

static PlaneTabs plane_tabs(const System& s, const QSet& q) {
    PlaneTabs t;
    t.nrows_kq = q.d_nrows_kq;
    t.nrows_u = q.d_nrows_u;
    t.rmask_kq = q.d_rmask_kq;
    t.rmask_u = q.d_rmask_u;
    t.rows_kq = q.d_rows_kq;
    t.rows_u = q.d_rows_u;
    t.tw1 = s.plan[0].tw;
    t.tw2 = s.plan[1].tw;
    t.perm1 = s.perm[0];
    t.perm2 = s.perm[1];
    t.colidx_kq = q.d_colidx_kq;
    t.tw1f = s.twf[0];
    t.tw2f = s.twf[1];
    return t;
}

void launch_density(const System& s, const QSet& q, hipStream_t st, bool fp32, int nrhs) {
    PlaneArgs a = plane_args(s, q);
    dim3 grid(s.n3, a.nchunk, 2 * q.nk * nrhs);
    if (plane_fixed_supported(s.n1, s.n2)) {
        launch_plane_fixed(true, a, plane_tabs(s, q), grid, s.n1, s.n2, st, fp32);
    } else {
        TM_CHECK(!fp32, TM_EUNSUPPORTED, "single-precision plane kernels need a fixed-size plane");
        int th = plane_threads(s);
        size_t shm = (size_t)a.NP * sizeof(double2);
        TM_LAUNCH(k_density, grid, dim3(th), shm, st, a, s.plan[0], s.plan[1]);
    }
    long long n4 = 4 * s.N;
    const double scale = 1.0 / (s.omega * q.nk);
    const dim3 rgrid((unsigned)((n4 + 255) / 256), nrhs);
    if (fp32) {
        TM_LAUNCH(k_density_reduce<float2>, rgrid, dim3(256), 0, st, a.rho_part32, s.ws.rho, s.N, q.nk, a.nchunk,
                  scale);
    } else {
        TM_LAUNCH(k_density_reduce<double2>, rgrid, dim3(256), 0, st, s.ws.rho_part, s.ws.rho, s.N, q.nk, a.nchunk,
                  scale);
    }
}

// A grid of at most kPotLdsMax points: the response potential of right-hand
// side blockIdx.y in one launch.  Block 0 holds the grid in LDS and takes the
// same steps as the multi-kernel path below, in the same order: the charge
// component to G space along i2, i1, i3, times the Coulomb multiplier
// (Eq. v_H_q, normalisation included), back to real space, then
// W_0 = v'_H + sum_b f_0b rho'_b.  Blocks 1 .. kPotParts form the other three
// components W_a = sum_b f_ab rho'_b (Eqs. v_XC_q, b_XC_q), which do not wait
// for v'_H, over a share of the points each.
constexpr long long kPotLdsMax = 8192;  // 128 KB of LDS (and the twiddle tables)
constexpr int kPotThreads = 512;
constexpr int kPotParts = 8;

// Transform of length N with the radices of the plan (4s, then 5s, 3s, 2s),
// with N and the radices known at compile time: P = product of the earlier radices
constexpr int next_radix(int m) { return m % 4 == 0 ? 4 : m % 5 == 0 ? 5 : m % 3 == 0 ? 3 : 2; }

// NL lines, NT threads: a thread takes at most ceil(NL N / R / NT) butterflies
template <int N, int NL, int NT, int P = 1, class LN>
__device__ __forceinline__ void ct_fft(double2* lds, const LN& ln, int estride, const double2* tw, int sign) {
    if constexpr (P < N) {
        constexpr int R = next_radix(N / P);
        constexpr int BF = (NL * (N / R) + NT - 1) / NT;
        fft_pass<R, BF>(lds, NL, ln, estride, N, P, tw, sign);
        ct_fft<N, NL, NT, P * R>(lds, ln, estride, tw, sign);
    }
}

// Length-20 transform of whole lines in registers, one thread per line
// (n = 5 n1 + n2, k = k1 + 4 k2: four-point transforms over n1, the twiddles
// w20^(n2 k1), five-point transforms over n2), so an axis costs one LDS round
// trip instead of two radix passes; natural order in and out.  tw: the table
// exp(-2 pi i j / 20).  Ends with a barrier.
template <int NL, class LN>
__device__ __forceinline__ void line_dft20(double2* lds, const LN& ln, int estride, const double2* tw, int sign) {
    for (int l = threadIdx.x; l < NL; l += blockDim.x) {
        double2* base = lds + ln.base(l);
        double2 z[5][4];
#pragma unroll
        for (int n2 = 0; n2 < 5; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) z[n2][n1] = base[(5 * n1 + n2) * estride];
            dft_small<4>(z[n2], sign);
#pragma unroll
            for (int k1 = 1; k1 < 4; ++k1)
                if (n2 > 0) z[n2][k1] = cmul(z[n2][k1], twiddle(tw, n2 * k1, sign));
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            double2 v[5];
#pragma unroll
            for (int n2 = 0; n2 < 5; ++n2) v[n2] = z[n2][k1];
            dft_small<5>(v, sign);
#pragma unroll
            for (int k2 = 0; k2 < 5; ++k2) base[(k1 + 4 * k2) * estride] = v[k2];
        }
    }
    __syncthreads();
}

// 3D transform of the grid [i3][i1][i2] in LDS along i2, i1, i3; tw: the three
// twiddle tables (lengths n1, n2, n3) one after the other.  N1 > 0: the sizes
// are compile-time constants (the index arithmetic folds); else the plans'.
template <int N1, int N2, int N3, int NT>
__device__ void grid_fft(double2* g, int n1, int n2, int n3, const FFTPlan& p1, const FFTPlan& p2,
                         const FFTPlan& p3, const double2* tw, int sign) {
    if constexpr (N1 == 20 && N2 == 20 && N3 == 20) {
        constexpr int NP = N1 * N2;
        line_dft20<N3 * N1>(g, StrideLines{N2}, 1, tw + N1, sign);
        line_dft20<N3 * N2>(g, GridLines{N2, NP, 1}, N2, tw, sign);
        line_dft20<NP>(g, StrideLines{1}, NP, tw + N1 + N2, sign);
    } else if constexpr (N1 > 0) {
        constexpr int NP = N1 * N2;
        ct_fft<N2, N3 * N1, NT>(g, StrideLines{N2}, 1, tw + N1, sign);        // along i2: lines (i3, i1)
        ct_fft<N1, N3 * N2, NT>(g, GridLines{N2, NP, 1}, N2, tw, sign);       // along i1: lines (i3, i2)
        ct_fft<N3, NP, NT>(g, StrideLines{1}, NP, tw + N1 + N2, sign);        // along i3: over the plane
    } else {
        const int NP = n1 * n2;
        lds_fft_lines(g, n3 * n1, StrideLines{n2}, 1, p2, tw + n1, sign);
        lds_fft_lines(g, n3 * n2, GridLines{n2, NP, 1}, n2, p1, tw, sign);
        lds_fft_lines(g, NP, StrideLines{1}, NP, p3, tw + n1 + n2, sign);
    }
}

// threads of k_potential_lds: 512 for 20^3 (a line of 20 a thread, 400 lines
// an axis), 1024 for other compile-time sizes (few butterflies a thread),
// kPotThreads for the generic kernel (kMaxBfly a thread)
template <int N1>
constexpr int pot_threads() { return N1 == 20 ? 512 : N1 > 0 ? 1024 : kPotThreads; }

template <int N1, int N2, int N3>
__global__ void __launch_bounds__(pot_threads<N1>()) k_potential_lds(const double2* rho, const double* const* hqt,
                                                                     int hmod, const double* fxc, double2* W, int n1,
                                                                     int n2, int n3, FFTPlan p1, FFTPlan p2,
                                                                     FFTPlan p3) {
    constexpr int NT = pot_threads<N1>();
    extern __shared__ double2 g[];
    if constexpr (N1 > 0) {
        n1 = N1;
        n2 = N2;
        n3 = N3;
    }
    const int N = n1 * n2 * n3;
    rho += (size_t)blockIdx.y * 4 * N;
    W += (size_t)blockIdx.y * 4 * N;
    const double* hq = hqt[blockIdx.y % hmod];  // the right-hand side's q set's Coulomb multiplier
    if (blockIdx.x > 0) {
        const int per = (N + kPotParts - 1) / kPotParts;
        const int i0 = (blockIdx.x - 1) * per, i1 = min(N, i0 + per);
        for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
            double f[9];
#pragma unroll
            for (int t = 0; t < 9; ++t) f[t] = fxc[(size_t)(t + 1) * N + i];
            const double2 r0 = rho[i], r1 = rho[N + i], r2 = rho[2 * N + i], r3 = rho[3 * N + i];
            auto comb = [&](double a0, double a1, double a2, double a3) {
                return cmk(a0 * r0.x + a1 * r1.x + a2 * r2.x + a3 * r3.x,
                           a0 * r0.y + a1 * r1.y + a2 * r2.y + a3 * r3.y);
            };
            W[N + i] = comb(f[0], f[3], f[4], f[5]);
            W[2 * N + i] = comb(f[1], f[4], f[6], f[7]);
            W[3 * N + i] = comb(f[2], f[5], f[7], f[8]);
        }
        return;
    }
    // the twiddle tables next to the grid, so that the passes read them from LDS
    double2* tw = g + N;
    for (int i = threadIdx.x; i < n1 + n2 + n3; i += blockDim.x)
        tw[i] = i < n1 ? p1.tw[i] : i < n1 + n2 ? p2.tw[i - n1] : p3.tw[i - n1 - n2];
    // element-wise loops in groups of U points a thread, loads first, so that a
    // thread's global loads are in flight together
    constexpr int U = NT >= 1024 ? 2 : 4;
    const int step = U * blockDim.x;
    for (int i0 = threadIdx.x; i0 < N; i0 += step) {
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            v[u] = i < N ? rho[i] : cmk(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            if (i < N) g[i] = v[u];
        }
    }
    __syncthreads();
    grid_fft<N1, N2, N3, NT>(g, n1, n2, n3, p1, p2, p3, tw, -1);
    for (int i0 = threadIdx.x; i0 < N; i0 += step) {
        double h[U];
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            h[u] = i < N ? hq[i] : 0.0;
            v[u] = i < N ? g[i] : cmk(0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            if (i < N) g[i] = cscale(v[u], h[u]);
        }
    }
    __syncthreads();
    grid_fft<N1, N2, N3, NT>(g, n1, n2, n3, p1, p2, p3, tw, +1);
    for (int i0 = threadIdx.x; i0 < N; i0 += step) {
        double2 r[U][4];
        double f[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = min(i0 + u * (int)blockDim.x, N - 1);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                r[u][c] = rho[(size_t)c * N + i];
                f[u][c] = fxc[(size_t)c * N + i];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * (int)blockDim.x;
            if (i < N) {
                W[i] = cadd(g[i], cmk(f[u][0] * r[u][0].x + f[u][1] * r[u][1].x + f[u][2] * r[u][2].x +
                                          f[u][3] * r[u][3].x,
                                      f[u][0] * r[u][0].y + f[u][1] * r[u][1].y + f[u][2] * r[u][2].y +
                                          f[u][3] * r[u][3].y));
            }
        }
    }
}

// smallest radix of a plan
static int min_radix(const FFTPlan& p) {
    int m = p.n;
    for (int r = 0; r < p.nrad; ++r) m = std::min(m, p.rad[r]);
    return m;
}

void launch_potential(const System& s, const QSet& q, hipStream_t st, int nrhs) {
    long long N = s.N;
    // every radix pass of the in-LDS transform within kMaxBfly butterflies a thread
    const int rmin = std::min(min_radix(s.plan[0]), std::min(min_radix(s.plan[1]), min_radix(s.plan[2])));
    if (N <= kPotLdsMax && N / rmin <= (long long)kMaxBfly * kPotThreads) {
        const size_t shm = (size_t)(N + s.n1 + s.n2 + s.n3) * sizeof(double2);
        const bool c20 = s.n1 == 20 && s.n2 == 20 && s.n3 == 20, c8 = s.n1 == 8 && s.n2 == 8 && s.n3 == 8;
        auto kern = c20 ? k_potential_lds<20, 20, 20> : c8 ? k_potential_lds<8, 8, 8> : k_potential_lds<0, 0, 0>;
        const int nt = c20 ? pot_threads<20>() : c8 ? pot_threads<8>() : pot_threads<0>();
        TM_CHECK(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm) ==
                     hipSuccess,
                 TM_EDEVICE, "cannot raise the LDS limit of k_potential_lds");
        ProfScope ps("k_potential_lds", st);
        hipLaunchKernelGGL(kern, dim3(1 + kPotParts, nrhs), dim3(nt), shm, st, s.ws.rho,
                           (const double* const*)q.d_hqt, q.hmod, s.fxc, s.ws.W, s.n1, s.n2, s.n3, s.plan[0],
                           s.plan[1], s.plan[2]);
        check_launch("k_potential_lds");
        return;
    }
    // every right-hand side in each launch
    const dim3 grid((unsigned)((N + 255) / 256), nrhs);
    TM_LAUNCH(k_copy_scale, grid, dim3(256), 0, st, s.ws.rho, s.ws.work, N);
    launch_fft3d_full(s, s.ws.work, -1, st, nrhs);
    TM_LAUNCH(k_mul_real, grid, dim3(256), 0, st, s.ws.work, (const double* const*)q.d_hqt, q.hmod, N);
    launch_fft3d_full(s, s.ws.work, +1, st, nrhs);
    TM_LAUNCH(k_assemble_W, grid, dim3(256), 0, st, s.ws.rho, s.ws.work, s.fxc, s.ws.W, N);
}

void launch_apply_planes(const System& s, const QSet& q, hipStream_t st, bool fp32, int nrhs) {
    PlaneArgs a = plane_args(s, q);
    dim3 grid(s.n3, a.nchunk, 2 * q.nk * nrhs);
    if (plane_fixed_supported(s.n1, s.n2)) {
        launch_plane_fixed(false, a, plane_tabs(s, q), grid, s.n1, s.n2, st, fp32);
        return;
    }
    TM_CHECK(!fp32, TM_EUNSUPPORTED, "single-precision plane kernels need a fixed-size plane");
    int th = plane_threads(s);
    size_t shm = (size_t)a.NP * sizeof(double2);
    TM_LAUNCH(k_apply_planes, grid, dim3(th), shm, st, a, s.plan[0], s.plan[1]);
}

void launch_ureal(const System& s, const QSet& q, hipStream_t st) {
    PlaneArgs a = plane_args(s, q);
    a.ureal = s.ureal;
    dim3 grid(s.n3, a.nchunk, 2 * q.nk);
    launch_ureal_fixed(a, plane_tabs(s, q), grid, s.n1, s.n2, st);
}

void launch_fxc_setup(System& s, const double* rho_plane, hipStream_t st) {
    TM_LAUNCH(k_fxc, dim3((unsigned)((s.N + 255) / 256)), dim3(256), 0, st, rho_plane, s.fxc, s.N);
}

void launch_coulomb_setup(const System& s, QSet& q, hipStream_t st) {
    const double* B = s.recip;
    TM_LAUNCH(k_coulomb, dim3((unsigned)((s.N + 255) / 256)), dim3(256), 0, st, q.hq, s.n1, s.n2, s.n3,
                       make_double3(B[0], B[1], B[2]), make_double3(B[3], B[4], B[5]),
                       make_double3(B[6], B[7], B[8]), make_double3(q.xq[0], q.xq[1], q.xq[2]),
                       1.0 / (double)s.N);
}

void launch_kin(const System& s, double* kin, const int* d_mill, int npw, int npw_pad, const double* p,
                hipStream_t st) {
    const double* B = s.recip;
    TM_LAUNCH(k_kin, dim3((npw_pad + 255) / 256), dim3(256), 0, st, kin, d_mill, npw, npw_pad,
                       make_double3(p[0], p[1], p[2]), make_double3(B[0], B[1], B[2]),
                       make_double3(B[3], B[4], B[5]), make_double3(B[6], B[7], B[8]));
}

}  // namespace tml

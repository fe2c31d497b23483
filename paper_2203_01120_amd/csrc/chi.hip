// Susceptibility from the Lanczos tridiagonal matrix (Eqs.
// resolvent_Liouvillian_Lanczos_q and post_processing):
//   chi_l(w) = n1 sum_i z_l[i] eta_i,   ((w + i eta) I - T) eta = e_1.
// One thread per frequency solves its tridiagonal system by Gaussian
// elimination with partial pivoting (row interchanges create a second
// superdiagonal), then back-substitutes and contracts with z.  Per-frequency
// work arrays live in global memory laid out [i][frequency] so neighbouring
// threads touch neighbouring addresses.
#include "tm_internal.h"

namespace tml {

namespace {

__device__ inline double2 cdiv(double2 a, double2 b) {
    // Smith's algorithm for a / b
    if (fabs(b.x) >= fabs(b.y)) {
        double r = b.y / b.x, d = b.x + b.y * r;
        return cmk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
    }
    double r = b.x / b.y, d = b.x * r + b.y;
    return cmk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}

__device__ inline double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }

__global__ void k_chi(const double2* alpha, const double* beta, const double2* gamma, const double2* z, int nz,
                      int cap, int M, double n1, const double* omega, int nw, double eta, double2* wd, double2* wdu,
                      double2* wdu2, double2* wb, double2* chi, int* status) {
    int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nw) return;
    auto D = [&](int i) -> double2& { return wd[(long long)i * nw + w]; };
    auto DU = [&](int i) -> double2& { return wdu[(long long)i * nw + w]; };
    auto DU2 = [&](int i) -> double2& { return wdu2[(long long)i * nw + w]; };
    auto Bv = [&](int i) -> double2& { return wb[(long long)i * nw + w]; };
    const double2 wc = cmk(omega[w], eta);
    for (int i = 0; i < M; ++i) {
        D(i) = csub(wc, alpha[i]);
        DU(i) = i + 1 < M ? cmk(-gamma[i].x, -gamma[i].y) : cmk(0.0, 0.0);
        DU2(i) = cmk(0.0, 0.0);
        Bv(i) = i == 0 ? cmk(1.0, 0.0) : cmk(0.0, 0.0);
    }
    int bad = 0;
    for (int i = 0; i + 1 < M; ++i) {
        double2 dl = cmk(-beta[i], 0.0);  // A[i+1][i]
        double2 di = D(i);
        if (cabs1(di) >= cabs1(dl)) {
            if (cabs1(di) == 0.0) { bad = 1; break; }
            double2 f = cdiv(dl, di);
            D(i + 1) = csub(D(i + 1), cmul(f, DU(i)));
            Bv(i + 1) = csub(Bv(i + 1), cmul(f, Bv(i)));
        } else {
            double2 f = cdiv(di, dl);
            D(i) = dl;
            double2 tmp = D(i + 1);
            D(i + 1) = csub(DU(i), cmul(f, tmp));
            if (i + 2 < M) {
                DU2(i) = DU(i + 1);
                DU(i + 1) = cmk(-(f.x * DU2(i).x - f.y * DU2(i).y), -(f.x * DU2(i).y + f.y * DU2(i).x));
            }
            DU(i) = tmp;
            double2 bi = Bv(i);
            Bv(i) = Bv(i + 1);
            Bv(i + 1) = csub(bi, cmul(f, Bv(i + 1)));
        }
    }
    if (!bad && cabs1(D(M - 1)) == 0.0) bad = 1;
    double2 acc[4] = {cmk(0, 0), cmk(0, 0), cmk(0, 0), cmk(0, 0)};
    if (!bad) {
        double2 x1 = cmk(0, 0), x2 = cmk(0, 0);  // x[i+1], x[i+2]
        for (int i = M - 1; i >= 0; --i) {
            double2 r = Bv(i);
            if (i + 1 < M) r = csub(r, cmul(DU(i), x1));
            if (i + 2 < M) r = csub(r, cmul(DU2(i), x2));
            double2 xi = cdiv(r, D(i));
            for (int l = 0; l < 4; ++l)
                if (l < nz) acc[l] = cadd(acc[l], cmul(z[(long long)l * cap + i], xi));
            x2 = x1;
            x1 = xi;
        }
    } else {
        atomicOr(status, 1);
    }
    for (int l = 0; l < nz; ++l) chi[(long long)l * nw + w] = cscale(acc[l], n1);
}

}  // namespace

void launch_chi(const double2* alpha, const double* beta, const double2* gamma, const double2* z, int nz, int cap,
                int M, double n1, const double* omega, int nw, double eta, double2* work, double2* chi, int* status,
                hipStream_t st) {
    TM_CHECK(nz >= 1 && nz <= 4, TM_EINVAL, "1 to 4 measure rows");
    long long per = (long long)M * nw;
    TM_LAUNCH(k_chi, dim3((nw + 63) / 64), dim3(64), 0, st, alpha, beta, gamma, z, nz, cap, M, n1, omega, nw,
                       eta, work, work + per, work + 2 * per, work + 3 * per, chi, status);
}

}  // namespace tml

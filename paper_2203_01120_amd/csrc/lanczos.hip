// Lanczos recursions on the device (Sec. 2.5).
//
// Vectors are kept unnormalised ("raw") with their scale factors in a small
// device struct, so a step never rescales a vector in memory: the update
// kernel forms the new residual from scaled inputs and, in the same pass,
// accumulates the inner products the next coefficients need.  A one-thread
// control kernel turns the reduced inner products into alpha, beta, gamma and
// z, applies the breakdown rule and updates the scales; nothing returns to
// the host until the chain ends.
//
// Pseudo-Hermitian step (metric S = JL, one apply):
//   r = Lq - alpha q - beta q_prev;  Lr = L r;
//   beta' = sqrt(r^dag J Lr),  alpha' = (Lr)^dag J Lr / beta'^2,  z' = (u, r) / beta'.
// Non-Hermitian step (two applies, L^dag = J L J):
//   alpha = (p, Lq);  qh = Lq - alpha q - gamma q_prev;
//   ph = L^dag p - conj(alpha) p - conj(beta) p_prev;  s = (ph, qh);
//   beta' = sqrt|s|,  gamma' = s / beta',  q' = qh / beta',  p' = ph / conj(gamma').
// Inner products (a, b) = (1/nk) sum conj(a) b; J negates the Y half.
#include "lanczos_dev.h"

namespace tml {

namespace {

constexpr int kRedThreads = 256;
constexpr int kRedBlocks = kPartBlocks;

__device__ inline double2 wave_sum(double2 v) {
    for (int off = 32; off > 0; off >>= 1) {
        v.x += __shfl_down(v.x, off, 64);
        v.y += __shfl_down(v.y, off, 64);
    }
    return v;
}

// block reduction of ND complex values; result valid in thread 0
template <int ND>
__device__ inline void block_sum(double2 (&v)[ND]) {
    __shared__ double2 sh[ND][kRedThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        double2 s = wave_sum(v[d]);
        if (lane == 0) sh[d][w] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            double2 s = cmk(0.0, 0.0);
            for (int i = 0; i < kRedThreads / 64; ++i) s = cadd(s, sh[d][i]);
            v[d] = s;
        }
    }
}

struct Dot {
    const double2* a;
    const double2* b;
    int jsign;  // 1: negate the contribution of the Y half
};

// lane blockIdx.y
template <int ND>
__global__ void __launch_bounds__(kRedThreads) k_multidot(DotSet<ND> ds, long long n, long long half, double2* part) {
    const int lane = blockIdx.y;
    const double2* A[ND];
    const double2* B[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        A[d] = ds.a[d] + lane * ds.sa[d];
        B[d] = ds.b[d] + lane * ds.sb[d];
    }
    part += (long long)lane * gridDim.x * ND;
    double2 acc[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) acc[d] = cmk(0.0, 0.0);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const bool y = i >= half;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            double2 t = cmulc(A[d][i], B[d][i]);
            if (y && ds.jsign[d]) t = cmk(-t.x, -t.y);
            acc[d] = cadd(acc[d], t);
        }
    }
    block_sum<ND>(acc);
    if (threadIdx.x == 0)
#pragma unroll
        for (int d = 0; d < ND; ++d) part[(long long)blockIdx.x * ND + d] = acc[d];
}

// deterministic final sum of the block partials, times the 1/nk weight (lane
// blockIdx.x): wave d sums value d, each of its lanes a fixed stride of blocks,
// then the wave's lanes in a fixed tree
__global__ void k_dot_final(const double2* part, int nblk, int nd, double w, double2* out) {
    const int d = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (d >= nd) return;  // whole waves
    part += (long long)blockIdx.x * nblk * nd;
    out += blockIdx.x * kDotStride;
    double2 s = cmk(0.0, 0.0);
    for (int b = l; b < nblk; b += 64) s = cadd(s, part[(long long)b * nd + d]);
    s = wave_sum(s);
    if (l == 0) out[d] = cscale(s, w);
}

// pH residual: r = slq Lq - alpha sq q - beta sprev qprev; partials of (u_l, r)
// for the measure vectors l = x, y, z, n (lane blockIdx.y's at u_l + lane ustride)
__global__ void __launch_bounds__(kRedThreads) k_ph_update(const ChainState* cs, const double2* Lq, const double2* q,
                                                            const double2* qp, double2* r, const double2* u0,
                                                            const double2* u1, const double2* u2,
                                                            const double2* u3, long long ustride, long long n,
                                                            double2* part) {
    const long long lo = (long long)blockIdx.y * n;  // lane blockIdx.y
    const long long uo = (long long)blockIdx.y * ustride;
    u0 += uo;
    u1 += uo;
    u2 += uo;
    u3 += uo;
    cs += blockIdx.y;
    Lq += lo;
    q += lo;
    qp += lo;
    r += lo;
    part += (long long)blockIdx.y * gridDim.x * 4;
    const double slq = cs->slq.x, sq = cs->sq.x, sp = cs->sprev.x;
    const double a = cs->alpha.x, bp = cs->beta_prev;
    const bool live = !cs->broken;
    double2 acc[4] = {cmk(0, 0), cmk(0, 0), cmk(0, 0), cmk(0, 0)};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        double2 v = cmk(0.0, 0.0);
        if (live) {
            double2 lq = Lq[i], qq = q[i], pq = qp[i];
            v.x = slq * lq.x - a * sq * qq.x - bp * sp * pq.x;
            v.y = slq * lq.y - a * sq * qq.y - bp * sp * pq.y;
        }
        r[i] = v;
        acc[0] = cadd(acc[0], cmulc(u0[i], v));
        acc[1] = cadd(acc[1], cmulc(u1[i], v));
        acc[2] = cadd(acc[2], cmulc(u2[i], v));
        acc[3] = cadd(acc[3], cmulc(u3[i], v));
    }
    block_sum<4>(acc);
    if (threadIdx.x == 0)
        for (int d = 0; d < 4; ++d) part[(long long)blockIdx.x * 4 + d] = acc[d];
}

// nH residuals: qh = sq Lq - alpha sq q - gamma_p sqp qp,
//               ph = sp J Ltp - conj(alpha) sp p - conj(beta_p) spp pp;
// partials of (ph, qh), (qh, qh), (ph, ph), (u_l, qh) for l = x, y, z, n
__global__ void __launch_bounds__(kRedThreads) k_nh_update(const ChainState* cs, const double2* Lq, const double2* q,
                                                            const double2* qp, const double2* Ltp, const double2* p,
                                                            const double2* pp, double2* qh, double2* ph,
                                                            const double2* u0, const double2* u1, const double2* u2,
                                                            const double2* u3, long long ustride, long long n,
                                                            long long half, double2* part) {
    const long long lo = (long long)blockIdx.y * n;  // lane blockIdx.y
    const long long uo = (long long)blockIdx.y * ustride;
    u0 += uo;
    u1 += uo;
    u2 += uo;
    u3 += uo;
    cs += blockIdx.y;
    Lq += lo;
    q += lo;
    qp += lo;
    Ltp += lo;
    p += lo;
    pp += lo;
    qh += lo;
    ph += lo;
    part += (long long)blockIdx.y * gridDim.x * 7;
    const double2 sq = cs->sq, sqp = cs->sprev, sp = cs->sp, spp = cs->spprev;
    const double2 a = cs->alpha;
    const double2 g = cs->gamma_prev;
    const double bpv = cs->beta_prev;
    const bool live = !cs->broken;
    const double2 c_q = cmul(a, sq), c_qp = cmul(g, sqp);
    const double2 c_p = cmul(cconj(a), sp), c_pp = cscale(spp, bpv);  // conj(beta) = beta (real)
    double2 acc[7];
#pragma unroll
    for (int d = 0; d < 7; ++d) acc[d] = cmk(0.0, 0.0);
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        double2 vq = cmk(0.0, 0.0), vp = cmk(0.0, 0.0);
        if (live) {
            vq = csub(csub(cmul(sq, Lq[i]), cmul(c_q, q[i])), cmul(c_qp, qp[i]));
            double2 lt = Ltp[i];
            if (i >= half) lt = cmk(-lt.x, -lt.y);
            vp = csub(csub(cmul(sp, lt), cmul(c_p, p[i])), cmul(c_pp, pp[i]));
        }
        qh[i] = vq;
        ph[i] = vp;
        acc[0] = cadd(acc[0], cmulc(vp, vq));
        acc[1] = cadd(acc[1], cmulc(vq, vq));
        acc[2] = cadd(acc[2], cmulc(vp, vp));
        acc[3] = cadd(acc[3], cmulc(u0[i], vq));
        acc[4] = cadd(acc[4], cmulc(u1[i], vq));
        acc[5] = cadd(acc[5], cmulc(u2[i], vq));
        acc[6] = cadd(acc[6], cmulc(u3[i], vq));
    }
    block_sum<7>(acc);
    if (threadIdx.x == 0)
        for (int d = 0; d < 7; ++d) part[(long long)blockIdx.x * 7 + d] = acc[d];
}

__global__ void k_jcopy(const double2* src, double2* dst, long long n, long long half) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    src += (long long)blockIdx.y * n;
    dst += (long long)blockIdx.y * n;
    double2 v = src[i];
    dst[i] = i >= half ? cmk(-v.x, -v.y) : v;
}

// ---- control kernels (one thread per lane) ------------------------------------------

// pH start; dots: (v, J Lv), (v, v), (Lv, J Lv), (u_l, v) l = 0..3
__global__ void k_ph_start(ChainState* cs, const double2* d, Coeffs co) {
    cs += threadIdx.x;
    d += threadIdx.x * kDotStride;
    co = co.lane(threadIdx.x);
    const double n1sq = d[0].x, vv = d[1].x;
    cs->broken = 0;
    cs->step = 0;
    if (!(n1sq > kBreakdownTol * cs->lam * vv)) {
        cs->broken = 1;
        cs->n1 = 0.0;
        return;
    }
    const double n1 = sqrt(n1sq);
    cs->n1 = n1;
    cs->sq = cs->slq = cmk(1.0 / n1, 0.0);
    cs->sprev = cmk(0.0, 0.0);
    cs->beta_prev = 0.0;
    cs->alpha = cmk(d[2].x / n1sq, 0.0);
    cs->qq = vv / n1sq;
    co.alpha[0] = cs->alpha;
    for (int l = 0; l < kNMeasure; ++l) co.z[l * co.cap] = cscale(d[3 + l], 1.0 / n1);
}

// pH after the apply, one lane; d: (r, J Lr), (r, r), (Lr, J Lr); zu: (u_l, r)
__device__ void ph_step_lane(ChainState* cs, const double2* d, const double2* zu, Coeffs co) {
    const int j = cs->step;
    if (cs->broken || j >= co.cap) return;
    const double b2 = d[0].x, rr = d[1].x, ll = d[2].x;
    const double lam = cs->lam, eps = kBreakdownTol;
    cs->step = j + 1;
    if (!(b2 > eps * lam * rr && rr > eps * eps * lam * lam * cs->qq)) {
        cs->broken = 1;
        return;
    }
    const double b = sqrt(b2);
    co.beta[j] = b;
    co.gamma[j] = cmk(b, 0.0);
    cs->sprev = cs->sq;
    cs->sq = cs->slq = cmk(1.0 / b, 0.0);
    cs->beta_prev = b;
    cs->alpha = cmk(ll / b2, 0.0);
    cs->qq = rr / b2;
    for (int l = 0; l < kNMeasure; ++l) cs->znext[l] = cscale(zu[l], 1.0 / b);
    if (j + 1 < co.cap) {
        co.alpha[j + 1] = cs->alpha;
        for (int l = 0; l < kNMeasure; ++l) co.z[l * co.cap + j + 1] = cs->znext[l];
    }
}

// nH start; dots: (v, v), (u_l, v)
__global__ void k_nh_start(ChainState* cs, const double2* d, Coeffs co) {
    cs += threadIdx.x;
    d += threadIdx.x * kDotStride;
    co = co.lane(threadIdx.x);
    const double vv = d[0].x;
    cs->broken = 0;
    cs->step = 0;
    if (!(vv > 0.0)) {
        cs->broken = 1;
        cs->n1 = 0.0;
        return;
    }
    const double n1 = sqrt(vv);
    cs->n1 = n1;
    cs->sq = cs->sp = cmk(1.0 / n1, 0.0);
    cs->sprev = cs->spprev = cmk(0.0, 0.0);
    cs->beta_prev = 0.0;
    cs->gamma_prev = cmk(0.0, 0.0);
    cs->qq = cs->pp = 1.0;
    for (int l = 0; l < kNMeasure; ++l) co.z[l * co.cap] = cscale(d[1 + l], 1.0 / n1);
}

// nH alpha from (P_raw, LQ_raw), one lane
__device__ void nh_alpha_lane(ChainState* cs, const double2* d, Coeffs co) {
    const int j = cs->step;
    if (cs->broken || j >= co.cap) return;
    cs->alpha = cmul(cmul(cconj(cs->sp), cs->sq), d[0]);
    co.alpha[j] = cs->alpha;
}

// nH after the update, one lane; d: (ph, qh), (qh, qh), (ph, ph), (u_l, qh)
__device__ void nh_step_lane(ChainState* cs, const double2* d, Coeffs co) {
    const int j = cs->step;
    if (cs->broken || j >= co.cap) return;
    const double2 s = d[0];
    const double qq = d[1].x, pp = d[2].x;
    const double lam = cs->lam, eps = kBreakdownTol;
    cs->step = j + 1;
    const double as = sqrt(cabs2(s));
    if (!(as > eps * lam * lam * sqrt(cs->pp * cs->qq))) {
        cs->broken = 1;
        return;
    }
    const double b = sqrt(as);
    const double2 g = cscale(s, 1.0 / b);
    co.beta[j] = b;
    co.gamma[j] = g;
    cs->sprev = cs->sq;
    cs->spprev = cs->sp;
    cs->sq = cmk(1.0 / b, 0.0);
    // 1 / conj(g)
    const double gg = cabs2(g);
    cs->sp = cmk(g.x / gg, g.y / gg);
    cs->qq = qq / (b * b);
    cs->pp = pp / gg;
    cs->beta_prev = b;
    cs->gamma_prev = g;
    for (int l = 0; l < kNMeasure; ++l) cs->znext[l] = cscale(d[3 + l], 1.0 / b);
    if (j + 1 < co.cap)
        for (int l = 0; l < kNMeasure; ++l) co.z[l * co.cap + j + 1] = cs->znext[l];
}

// The final sums of the block partials (as k_dot_final) folded into the
// control step that consumes them: block = lane blockIdx.x, wave v sums
// value v; the sums also go to the inner-product array (out + lane kDotStride).
__device__ inline void final_into(const double2* part, int nblk, int nd, int v, double w, double2* out,
                                  double2* sh) {
    const int l = threadIdx.x & 63, r = blockIdx.x;
    part += (long long)r * nblk * nd;
    double2 s = cmk(0.0, 0.0);
    for (int b = l; b < nblk; b += 64) s = cadd(s, part[(long long)b * nd + v]);
    s = wave_sum(s);
    if (l == 0) {
        s = cscale(s, w);
        out[r * kDotStride + v] = s;
        sh[v] = s;
    }
}

// pH: waves 0-2 the multidot (r, J Lr), (r, r), (Lr, J Lr); waves 3-6 the
// update's (u_l, r); then the step
__global__ void __launch_bounds__(64 * (3 + kNMeasure)) k_ph_step_sums(ChainState* cs, const double2* part_md,
                                                                        const double2* part_up, int nblk, double w,
                                                                        double2* d, double2* zu, Coeffs co) {
    __shared__ double2 sh[3 + kNMeasure];
    const int v = threadIdx.x >> 6;
    if (v < 3) final_into(part_md, nblk, 3, v, w, d, sh);
    else final_into(part_up, nblk, kNMeasure, v - 3, w, zu, sh + 3);
    __syncthreads();
    if (threadIdx.x == 0) ph_step_lane(cs + blockIdx.x, sh, sh + 3, co.lane(blockIdx.x));
}

__global__ void __launch_bounds__(64) k_nh_alpha_sums(ChainState* cs, const double2* part, int nblk, double w,
                                                      double2* d, Coeffs co) {
    __shared__ double2 sh[1];
    final_into(part, nblk, 1, 0, w, d, sh);
    __syncthreads();
    if (threadIdx.x == 0) nh_alpha_lane(cs + blockIdx.x, sh, co.lane(blockIdx.x));
}

__global__ void __launch_bounds__(64 * (3 + kNMeasure)) k_nh_step_sums(ChainState* cs, const double2* part,
                                                                        int nblk, double w, double2* d, Coeffs co) {
    __shared__ double2 sh[3 + kNMeasure];
    final_into(part, nblk, 3 + kNMeasure, threadIdx.x >> 6, w, d, sh);
    __syncthreads();
    if (threadIdx.x == 0) nh_step_lane(cs + blockIdx.x, sh, co.lane(blockIdx.x));
}

}  // namespace

// ---- host-side launch helpers ----------------------------------------------------

template <int ND>
void run_multidot(const DotSet<ND>& ds, long long n, long long half, double w, double2* part, double2* out,
                  hipStream_t st, int lanes, bool final) {
    int nblk = (int)std::min<long long>(kRedBlocks, (n + kRedThreads - 1) / kRedThreads);
    TM_LAUNCH(k_multidot<ND>, dim3(nblk, lanes), dim3(kRedThreads), 0, st, ds, n, half, part);
    if (final) TM_LAUNCH(k_dot_final, dim3(lanes), dim3(64 * ND), 0, st, part, nblk, ND, w, out);
}
template void run_multidot<1>(const DotSet<1>&, long long, long long, double, double2*, double2*, hipStream_t,
                                  int, bool);
template void run_multidot<3>(const DotSet<3>&, long long, long long, double, double2*, double2*, hipStream_t,
                                  int, bool);
template void run_multidot<5>(const DotSet<5>&, long long, long long, double, double2*, double2*, hipStream_t,
                                  int, bool);
template void run_multidot<7>(const DotSet<7>&, long long, long long, double, double2*, double2*, hipStream_t,
                                  int, bool);

static int red_blocks(long long n) {
    return (int)std::min<long long>(kRedBlocks, (n + kRedThreads - 1) / kRedThreads);
}

void run_ph_update(const ChainState* cs, const double2* Lq, const double2* q, const double2* qp, double2* r,
                   const double2* const* u, long long ustride, long long n, double2* part, hipStream_t st,
                   int lanes) {
    int nblk = red_blocks(n);
    TM_LAUNCH(k_ph_update, dim3(nblk, lanes), dim3(kRedThreads), 0, st, cs, Lq, q, qp, r, u[0], u[1], u[2], u[3],
              ustride, n, part);
}

void run_nh_update(const ChainState* cs, const double2* Lq, const double2* q, const double2* qp, const double2* Ltp,
                   const double2* p, const double2* pp, double2* qh, double2* ph, const double2* const* u,
                   long long ustride, long long n, long long half, double2* part, hipStream_t st, int lanes) {
    int nblk = red_blocks(n);
    TM_LAUNCH(k_nh_update, dim3(nblk, lanes), dim3(kRedThreads), 0, st, cs, Lq, q, qp, Ltp, p, pp, qh, ph, u[0],
              u[1], u[2], u[3], ustride, n, half, part);
}

void run_jcopy(const double2* src, double2* dst, long long n, long long half, hipStream_t st, int lanes) {
    TM_LAUNCH(k_jcopy, dim3((unsigned)((n + 255) / 256), lanes), dim3(256), 0, st, src, dst, n, half);
}

void ctl_ph_start(ChainState* cs, const double2* d, const Coeffs& co, hipStream_t st, int lanes) {
    TM_LAUNCH(k_ph_start, dim3(1), dim3(lanes), 0, st, cs, d, co);
}
void ctl_ph_step_sums(ChainState* cs, const double2* part_md, const double2* part_up, long long n, double w,
                      double2* d, double2* zu, const Coeffs& co, hipStream_t st, int lanes) {
    TM_LAUNCH(k_ph_step_sums, dim3(lanes), dim3(64 * (3 + kNMeasure)), 0, st, cs, part_md, part_up, red_blocks(n), w,
              d, zu, co);
}
void ctl_nh_start(ChainState* cs, const double2* d, const Coeffs& co, hipStream_t st, int lanes) {
    TM_LAUNCH(k_nh_start, dim3(1), dim3(lanes), 0, st, cs, d, co);
}
void ctl_nh_alpha_sums(ChainState* cs, const double2* part, long long n, double w, double2* d, const Coeffs& co,
                       hipStream_t st, int lanes) {
    TM_LAUNCH(k_nh_alpha_sums, dim3(lanes), dim3(64), 0, st, cs, part, red_blocks(n), w, d, co);
}
void ctl_nh_step_sums(ChainState* cs, const double2* part, long long n, double w, double2* d, const Coeffs& co,
                      hipStream_t st, int lanes) {
    TM_LAUNCH(k_nh_step_sums, dim3(lanes), dim3(64 * (3 + kNMeasure)), 0, st, cs, part, red_blocks(n), w, d, co);
}

}  // namespace tml

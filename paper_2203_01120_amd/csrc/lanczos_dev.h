// Device-side state of one Lanczos chain and the launch helpers of lanczos.hip.
#pragma once

#include "tm_internal.h"

namespace tml {

// breakdown tolerance of the chains (see tm.h for the rule it enters)
constexpr double kBreakdownTol = 1e-10;

// measure vectors u^l of a chain: l = x, y, z (spin) and n (charge)
constexpr int kNMeasure = 4;
// field directions one chain can run together on one q set (lanes)
constexpr int kMaxLanes = 4;
// lanes of a chain whose lanes carry their own q sets (a lane group)
constexpr int kMaxChainLanes = 96;
// reduced inner products kept per lane (a lane is one recursion of a chain
// that runs several field directions together)
constexpr int kDotStride = 16;
// blocks of an inner-product kernel, at most (one partial per block and value)
constexpr int kPartBlocks = 1024;

// one lane's scalars; true vector = scale * raw vector
struct ChainState {
    double2 sq, slq, sprev;     // q, Lq, q_prev (pH: real)
    double2 sp, spprev;         // p, p_prev (nH)
    double2 alpha;
    double2 gamma_prev;
    double beta_prev;
    double qq, pp;              // (q_i, q_i), (p_i, p_i)
    double lam;
    double n1;
    double2 znext[kNMeasure];   // z of the next index, kept when it falls past the capacity
    int step;
    int broken;
};

// coefficient arrays of all lanes: lane r at alpha + r cap, ..., z + r kNMeasure cap
struct Coeffs {
    double2* alpha;   // [lanes][cap]
    double* beta;     // [lanes][cap]
    double2* gamma;   // [lanes][cap]
    double2* z;       // [lanes][kNMeasure][cap]
    int cap;
    __host__ __device__ Coeffs lane(int r) const {
        return Coeffs{alpha + (size_t)r * cap, beta + (size_t)r * cap, gamma + (size_t)r * cap,
                      z + (size_t)r * kNMeasure * cap, cap};
    }
};

// Inner products (a_d, b_d), d < ND, for each of `lanes` lanes: lane r reads
// a_d + r sa_d and b_d + r sb_d (stride 0 for a vector the lanes share).
template <int ND>
struct DotSet {
    const double2* a[ND];
    const double2* b[ND];
    int jsign[ND];
    long long sa[ND];
    long long sb[ND];
};

// All helpers below work on `lanes` lanes at once: lane r's vectors at + r n,
// its state at cs + r, its inner products at out + r kDotStride, its partial
// sums at part + r (blocks x values); the measure vectors u are shared.
// final = false: only the block partials (a *_sums control step adds them)
template <int ND>
void run_multidot(const DotSet<ND>& ds, long long n, long long half, double w, double2* part, double2* out,
                  hipStream_t st, int lanes = 1, bool final = true);
// the updates write the block partials of their inner products to part
// u: the four measure vectors; lane r's are at u[l] + r ustride (0: shared by the lanes)
void run_ph_update(const ChainState* cs, const double2* Lq, const double2* q, const double2* qp, double2* r,
                   const double2* const* u, long long ustride, long long n, double2* part, hipStream_t st,
                   int lanes = 1);
void run_nh_update(const ChainState* cs, const double2* Lq, const double2* q, const double2* qp, const double2* Ltp,
                   const double2* p, const double2* pp, double2* qh, double2* ph, const double2* const* u,
                   long long ustride, long long n, long long half, double2* part, hipStream_t st, int lanes = 1);
void run_jcopy(const double2* src, double2* dst, long long n, long long half, hipStream_t st, int lanes = 1);
void ctl_ph_start(ChainState* cs, const double2* d, const Coeffs& co, hipStream_t st, int lanes = 1);
// The step controls add the block partials of their inner products (over
// vectors of n elements, weight w) in a fixed order, store the sums at
// d (zu) + lane kDotStride, and update the state.  The step index comes from
// cs->step (device side), so step sequences can be replayed from a graph;
// steps past co.cap are ignored.
void ctl_ph_step_sums(ChainState* cs, const double2* part_md, const double2* part_up, long long n, double w,
                      double2* d, double2* zu, const Coeffs& co, hipStream_t st, int lanes = 1);
void ctl_nh_start(ChainState* cs, const double2* d, const Coeffs& co, hipStream_t st, int lanes = 1);
void ctl_nh_alpha_sums(ChainState* cs, const double2* part, long long n, double w, double2* d, const Coeffs& co,
                       hipStream_t st, int lanes = 1);
void ctl_nh_step_sums(ChainState* cs, const double2* part, long long n, double w, double2* d, const Coeffs& co,
                      hipStream_t st, int lanes = 1);

}  // namespace tml

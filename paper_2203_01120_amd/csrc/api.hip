// C ABI of libtm: system set-up, the Liouvillian apply, the Lanczos driver and
// the susceptibility.  See include/tm.h for the contract of every call.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <set>
#include <unordered_map>

#include "lanczos_dev.h"
#include "plane.h"

namespace tml {

void launch_kin(const System& s, double* kin, const int* d_mill, int npw, int npw_pad, const double* p, hipStream_t st);
size_t gemm_partial_elems(int nbatch, int M, int Nn, int K);
void launch_chi(const double2* alpha, const double* beta, const double2* gamma, const double2* z, int nz, int cap,
                int M, double n1, const double* omega, int nw, double eta, double2* work, double2* chi, int* status,
                hipStream_t st);

static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }

// ---- kernel timing ----------------------------------------------------------------
namespace {
struct ProfRec {
    const char* name;
    hipEvent_t a, b;
};
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;
struct ProfAgg {
    std::string name;
    double ms = 0;
    long long n = 0;
};
std::vector<ProfAgg> g_prof_agg;

hipEvent_t prof_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    TM_HIP(hipEventCreate(&e));
    return e;
}

void prof_fold() {
    if (g_prof_pending.empty()) return;
    TM_HIP(hipDeviceSynchronize());
    for (auto& r : g_prof_pending) {
        float ms = 0;
        TM_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        auto it = std::find_if(g_prof_agg.begin(), g_prof_agg.end(), [&](const ProfAgg& x) { return x.name == r.name; });
        if (it == g_prof_agg.end()) {
            g_prof_agg.push_back(ProfAgg{r.name, 0, 0});
            it = g_prof_agg.end() - 1;
        }
        it->ms += ms;
        it->n += 1;
        g_prof_pool.push_back(r.a);
        g_prof_pool.push_back(r.b);
    }
    g_prof_pending.clear();
}
}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t s) : slot(-1), st(s) {
    if (!g_prof_on) return;
    if (g_prof_pending.size() > 200000) prof_fold();
    ProfRec r{name, prof_event(), prof_event()};
    TM_HIP(hipEventRecord(r.a, st));
    g_prof_pending.push_back(r);
    slot = (int)g_prof_pending.size() - 1;
}

ProfScope::~ProfScope() {
    if (slot >= 0) (void)hipEventRecord(g_prof_pending[slot].b, st);
}

// ---- autotuning registry -----------------------------------------------------------
namespace {
struct TuneEntry {
    int op;
    long long key;
    int nvariants = 0;
    int chosen = 0;
    std::vector<float> us;      // timed microseconds per variant
    std::string shape;          // human-readable shape
};
std::mutex g_tune_mu;
std::map<std::pair<int, long long>, TuneEntry> g_tuned;
int g_force[kTuneOps] = {-1, -1, -1, -1, -1, -1};
int g_trial[kTuneOps] = {-1, -1, -1, -1, -1, -1};   // the variant being timed
long long g_seen_key[kTuneOps];
int g_seen_n[kTuneOps];
bool g_autotune = true;
const char* const kTuneNames[kTuneOps] = {"plane_density", "plane_apply", "zpass_inverse", "zpass_forward",
                                           "contraction", "update"};
}  // namespace

int tune_pick(int op, long long key, int nvariants) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_seen_key[op] = key;
    g_seen_n[op] = nvariants;
    int v = 0;
    if (g_force[op] >= 0) {
        v = g_force[op];
    } else if (g_trial[op] >= 0) {
        v = g_trial[op];
    } else {
        auto it = g_tuned.find({op, key});
        if (it != g_tuned.end()) v = it->second.chosen;
    }
    TM_CHECK(v >= 0 && v < nvariants, TM_EINVAL,
             std::string("variant ") + std::to_string(v) + " of " + kTuneNames[op] + " out of range (" +
                 std::to_string(nvariants) + " variants for this shape)");
    return v;
}

void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{TM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

bool make_radices(int n, FFTPlan& p) {
    p.n = n;
    p.nrad = 0;
    int m = n;
    const int order[4] = {4, 5, 3, 2};
    for (int r : order) {
        while (m % r == 0) {
            if (p.nrad >= kMaxRadices) return false;
            p.rad[p.nrad++] = r;
            m /= r;
        }
    }
    return m == 1 && n > 0;
}

namespace {

// Grid lengths the kernels take (host check, no device needed): positive,
// products of 2, 3 and 5, and planes of at most 4096 points.
void check_grid(const int* fft) {
    for (int i = 0; i < 3; ++i) {
        TM_CHECK(fft[i] > 0, TM_EINVAL, "FFT lengths must be positive");
        FFTPlan p;
        TM_CHECK(make_radices(fft[i], p), TM_EUNSUPPORTED, "FFT length must factor into 2, 3, 5");
    }
    TM_CHECK((long long)fft[0] * fft[1] <= 4 * 1024, TM_EUNSUPPORTED,
             "n1*n2 above 4096 is not supported by the plane kernels");
}

inline long long mkey(int a, int b, int c) {
    return ((long long)(a + (1 << 20)) << 42) | ((long long)(b + (1 << 20)) << 21) | (long long)(c + (1 << 20));
}

// start vectors: su = sigma^dir (U~_k) on side 0, sigma^dir (T U~_-k) on side 1
__global__ void k_start(const double2* const* ucoef, const int* npw_u, const int* const* maps, int nk, int nb,
                        int npw_pad, int dir, double usign_y, double vsign_y, double2* u, double2* v) {
    const int b = blockIdx.z;
    const int n = blockIdx.y;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npw_pad) return;
    const int side = b >= nk;
    const int* map = maps[b];
    const double2* U = ucoef[b];
    const int nu = npw_u[b];
    double2 a = cmk(0, 0), c = cmk(0, 0);
    int j = map[g];
    if (j >= 0) {
        double2 up = U[((long long)n * 2 + 0) * nu + j], dn = U[((long long)n * 2 + 1) * nu + j];
        if (side == 0) {
            a = up;
            c = dn;
        } else {  // T = i sigma_y K at -G: (conj dn, -conj up)
            a = cconj(dn);
            c = cmk(-up.x, up.y);
        }
    }
    double2 ra, rc;
    switch (dir) {
        case TM_DIR_X: ra = c; rc = a; break;
        case TM_DIR_Y: ra = cmk(c.y, -c.x); rc = cmk(-a.y, a.x); break;  // (-i c, i a)
        case TM_DIR_Z: ra = a; rc = cmk(-c.x, -c.y); break;
        case TM_DIR_PLUS: ra = cscale(c, 2.0); rc = cmk(0, 0); break;
        case TM_DIR_MINUS: ra = cmk(0, 0); rc = cscale(a, 2.0); break;
        default: ra = a; rc = c; break;  // TM_DIR_N: sigma_0
    }
    long long off = (((long long)b * nb + n) * 2) * npw_pad + g;
    if (v) {
        double sg = side ? vsign_y : 1.0;
        v[off] = cscale(ra, sg);
        v[off + npw_pad] = cscale(rc, sg);
    }
    if (u) {
        double sg = side ? usign_y : 1.0;
        u[off] = cscale(ra, sg);
        u[off + npw_pad] = cscale(rc, sg);
    }
}

// occupied partner on the k+q sphere: side 0 copies U_{k+q}, side 1 builds T U_{-k-q} at -G
__global__ void k_occ(const double2* src, int npw_src, const int* map, int npw, int npw_pad, int nb, int tr,
                      double2* dst) {
    const int n = blockIdx.y;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npw_pad) return;
    double2 a = cmk(0, 0), c = cmk(0, 0);
    if (g < npw) {
        int j = map ? map[g] : g;
        double2 up = src[((long long)n * 2) * npw_src + j], dn = src[((long long)n * 2 + 1) * npw_src + j];
        if (tr) {
            a = cconj(dn);
            c = cmk(-up.x, up.y);
        } else {
            a = up;
            c = dn;
        }
    }
    dst[((long long)n * 2) * npw_pad + g] = a;
    dst[((long long)n * 2 + 1) * npw_pad + g] = c;
}

__global__ void k_pad_copy(const double2* src, int npw, int npw_pad, int rows, double2* dst) {
    const int r = blockIdx.y;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npw_pad || r >= rows) return;
    dst[(long long)r * npw_pad + g] = g < npw ? src[(long long)r * npw + g] : cmk(0, 0);
}

void build_sphere_map(System& s, SphereMap& m, const std::vector<int>& mill3, int npw) {
    m.npw = npw;
    std::unordered_map<int, int> colid;
    std::vector<int> colpos;
    std::vector<std::vector<int>> ents;
    std::unordered_map<long long, int> seen;
    for (int g = 0; g < npw; ++g) {
        int m1 = mill3[3 * g], m2 = mill3[3 * g + 1], m3 = mill3[3 * g + 2];
        TM_CHECK(2 * std::abs(m1) < s.n1 && 2 * std::abs(m2) < s.n2 && 2 * std::abs(m3) < s.n3, TM_EINVAL,
                 "a plane-wave sphere does not fit inside the FFT grid");
        int i1 = ((m1 % s.n1) + s.n1) % s.n1, i2 = ((m2 % s.n2) + s.n2) % s.n2;
        int pos = i1 * s.n2 + i2;
        TM_CHECK(seen.emplace(mkey(m1, m2, m3), g).second, TM_EINVAL, "duplicate Miller index in a sphere");
        auto it = colid.find(pos);
        int c;
        if (it == colid.end()) {
            c = (int)colpos.size();
            colid[pos] = c;
            colpos.push_back(pos);
            ents.emplace_back();
        } else {
            c = it->second;
        }
        ents[c].push_back(g);
    }
    m.ncol = (int)colpos.size();
    // columns in plane order (row-major in (i1, i2)) so each plane row is one contiguous run
    std::vector<int> order(m.ncol);
    for (int c = 0; c < m.ncol; ++c) order[c] = c;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return colpos[x] < colpos[y]; });
    std::vector<int> ptr(m.ncol + 1, 0), eg, ei, cpos(m.ncol), rows;
    eg.reserve(npw);
    ei.reserve(npw);
    m.rmask = 0;
    for (int c = 0; c < m.ncol; ++c) {
        const int oc = order[c];
        cpos[c] = colpos[oc];
        ptr[c + 1] = ptr[c] + (int)ents[oc].size();
        for (int g : ents[oc]) {
            eg.push_back(g);
            ei.push_back(((mill3[3 * g + 2] % s.n3) + s.n3) % s.n3);
        }
        const int i1 = cpos[c] / s.n2;
        if (rows.empty() || rows.back() != i1) rows.push_back(i1);
        if (i1 < 64) m.rmask |= 1ULL << i1;
    }
    m.col_ptr = dev_upload(s, ptr.data(), ptr.size());
    m.ent_g = dev_upload(s, eg.data(), eg.size());
    m.ent_i3 = dev_upload(s, ei.data(), ei.size());
    m.col_pos = dev_upload(s, cpos.data(), cpos.size());
    m.h_col_pos = cpos;
    m.nrows = (int)rows.size();
    m.rows = dev_upload(s, rows.data(), rows.size());
}

std::vector<int> shifted(const std::vector<int>& mill, int npw, const int* g) {
    std::vector<int> out(3 * (size_t)npw);
    for (int i = 0; i < npw; ++i)
        for (int c = 0; c < 3; ++c) out[3 * i + c] = mill[3 * i + c] - (g ? g[c] : 0);
    return out;
}

template <typename T>
T** upload_table(System& s, const std::vector<T*>& v) {
    return dev_upload(s, const_cast<T**>(v.data()), v.size());
}

void transpose_to_planes(const System& s, const double* src, std::vector<double>& dst, int ncomp) {
    // C order [n1][n2][n3] -> plane-major [i3][i1][i2]
    dst.resize((size_t)ncomp * s.N);
    for (int c = 0; c < ncomp; ++c)
        for (int i1 = 0; i1 < s.n1; ++i1)
            for (int i2 = 0; i2 < s.n2; ++i2)
                for (int i3 = 0; i3 < s.n3; ++i3)
                    dst[(size_t)c * s.N + ((size_t)i3 * s.n1 + i1) * s.n2 + i2] =
                        src[(size_t)c * s.N + ((size_t)i1 * s.n2 + i2) * s.n3 + i3];
}

// Column stride of the z-transformed column buffers: the most columns of any
// k+q sphere, rounded up to 8 so that a run of 8 columns (128 bytes in FP64)
// starting at a multiple of 8 fills whole cache lines (the forward z pass
// reads 8-column runs).
static int col_stride(int ncol) { return (ncol + 7) / 8 * 8; }

// The padded sphere length of every q set of a system: the largest k+q sphere
// over all of them, rounded up to 16, so that the BR vectors of all q sets
// share one layout and the lanes of one chain may carry different q sets.
int system_npw_pad(const tm_system_desc* d) {
    int npw_max = 0;
    for (int iq = 0; iq < d->nq; ++iq)
        for (int ik = 0; ik < d->nk; ++ik) {
            const int* r = d->roles + ((size_t)iq * d->nk + ik) * 4;
            for (int t = 0; t < 4; ++t) TM_CHECK(r[t] >= 0 && r[t] < d->npts, TM_EINVAL, "role index out of range");
            npw_max = std::max(npw_max, d->npw[r[2]]);
        }
    return (npw_max + 15) / 16 * 16;
}

void build_qset(System& s, const tm_system_desc* d, int iq, int npw_pad, QSet& q) {
    const int nk = d->nk;
    q.nk = nk;
    q.tmod = 2 * nk;
    for (int c = 0; c < 3; ++c) q.xq[c] = d->xq[3 * iq + c];
    q.kb.resize(nk);
    q.npw_pad = npw_pad;
    const int P = q.npw_pad, nb = s.nbnd;
    hipStream_t st = nullptr;
    q.ncol_max = 0;
    q.ncol_u_max = 0;
    q.lam = 0.0;
    std::vector<int*> t_colptr_kq(2 * nk), t_entg_kq(2 * nk), t_enti3_kq(2 * nk), t_colpos_kq(2 * nk);
    std::vector<int*> t_colptr_u(2 * nk), t_entg_u(2 * nk), t_enti3_u(2 * nk), t_colpos_u(2 * nk);
    std::vector<int> t_ncol_kq(2 * nk), t_npw_kq(2 * nk), t_ncol_u(2 * nk), t_npw_u(2 * nk);
    std::vector<const double2*> t_ucoef(2 * nk);
    std::vector<double*> t_kin(2 * nk), t_eps(2 * nk);
    std::vector<double2*> t_occ(2 * nk), t_vkb(2 * nk);
    std::vector<int*> t_maps(2 * nk);
    std::vector<int*> t_rows_kq(2 * nk), t_rows_u(2 * nk);
    std::vector<int> t_nrows_kq(2 * nk), t_nrows_u(2 * nk);
    std::vector<unsigned long long> t_rmask_kq(2 * nk), t_rmask_u(2 * nk);
    std::vector<int> t_uslot(2 * nk);
    std::vector<short*> t_colidx(2 * nk);
    for (int ik = 0; ik < nk; ++ik) {
        KBlock& kb = q.kb[ik];
        const int* r = d->roles + ((size_t)iq * nk + ik) * 4;
        const int* sh = d->shifts ? d->shifts + ((size_t)iq * nk + ik) * 12 : nullptr;
        const int pk = r[0], pmk = r[1], pkq = r[2], pmkq = r[3];
        const int npw = d->npw[pkq];
        kb.npw = npw;
        std::vector<int> m_kq = shifted(s.mill[pkq], npw, sh ? sh + 6 : nullptr);
        std::vector<int> m_k = shifted(s.mill[pk], d->npw[pk], sh ? sh + 0 : nullptr);
        std::vector<int> m_mk = shifted(s.mill[pmk], d->npw[pmk], sh ? sh + 3 : nullptr);
        std::vector<int> m_mkq = shifted(s.mill[pmkq], d->npw[pmkq], sh ? sh + 9 : nullptr);
        for (int c = 0; c < 3; ++c) {
            double g = 0;
            for (int t = 0; t < 3; ++t) g += (sh ? sh[6 + t] : 0) * s.recip[3 * t + c];
            kb.kq[c] = d->xk[3 * pkq + c] + g;
        }
        build_sphere_map(s, kb.sph_kq, m_kq, npw);
        build_sphere_map(s, kb.sph_u[0], m_k, d->npw[pk]);
        build_sphere_map(s, kb.sph_u[1], m_mk, d->npw[pmk]);
        kb.u_coef[0] = s.evc[pk];
        kb.u_coef[1] = s.evc[pmk];
        kb.npw_u[0] = d->npw[pk];
        kb.npw_u[1] = d->npw[pmk];
        q.ncol_max = std::max(q.ncol_max, kb.sph_kq.ncol);
        q.ncol_u_max = std::max({q.ncol_u_max, kb.sph_u[0].ncol, kb.sph_u[1].ncol});
        // lookup tables
        std::unordered_map<long long, int> lk, lmk, lmkq;
        for (int g = 0; g < d->npw[pk]; ++g) lk[mkey(m_k[3 * g], m_k[3 * g + 1], m_k[3 * g + 2])] = g;
        for (int g = 0; g < d->npw[pmk]; ++g) lmk[mkey(m_mk[3 * g], m_mk[3 * g + 1], m_mk[3 * g + 2])] = g;
        for (int g = 0; g < d->npw[pmkq]; ++g)
            lmkq[mkey(m_mkq[3 * g], m_mkq[3 * g + 1], m_mkq[3 * g + 2])] = g;
        TM_CHECK(d->npw[pmkq] == npw, TM_EINVAL, "the -k-q sphere is not the negative of the k+q sphere");
        std::vector<int> map_k(P, -1), map_mk(P, -1), map_mkq(npw, -1);
        for (int g = 0; g < npw; ++g) {
            int a = m_kq[3 * g], b = m_kq[3 * g + 1], c = m_kq[3 * g + 2];
            auto i1 = lk.find(mkey(a, b, c));
            if (i1 != lk.end()) map_k[g] = i1->second;
            auto i2 = lmk.find(mkey(-a, -b, -c));
            if (i2 != lmk.end()) map_mk[g] = i2->second;
            auto i3 = lmkq.find(mkey(-a, -b, -c));
            TM_CHECK(i3 != lmkq.end(), TM_EINVAL, "the -k-q sphere is not the negative of the k+q sphere");
            map_mkq[g] = i3->second;
        }
        kb.map_k = dev_upload(s, map_k.data(), map_k.size());
        kb.map_mk = dev_upload(s, map_mk.data(), map_mk.size());
        int* d_map_mkq = dev_upload(s, map_mkq.data(), map_mkq.size());
        // kinetic energies from the k+q point's own Miller indices
        int* d_mill = dev_upload(s, s.mill[pkq].data(), s.mill[pkq].size());
        kb.kin = dev_alloc<double>(s, P);
        launch_kin(s, kb.kin, d_mill, npw, P, d->xk + 3 * pkq, st);
        for (int g = 0; g < npw; ++g) {
            double x[3];
            for (int c = 0; c < 3; ++c) {
                x[c] = d->xk[3 * pkq + c];
                for (int t = 0; t < 3; ++t) x[c] += s.mill[pkq][3 * g + t] * s.recip[3 * t + c];
            }
            q.lam = std::max(q.lam, 0.5 * (x[0] * x[0] + x[1] * x[1] + x[2] * x[2]));
        }
        kb.eps[0] = dev_upload(s, s.et[pk].data(), nb);
        kb.eps[1] = dev_upload(s, s.et[pmk].data(), nb);
        kb.occ[0] = dev_alloc<double2>(s, (size_t)nb * 2 * P);
        kb.occ[1] = dev_alloc<double2>(s, (size_t)nb * 2 * P);
        dim3 gr((P + 127) / 128, nb);
        TM_LAUNCH(k_occ, gr, dim3(128), 0, st, s.evc[pkq], npw, (const int*)nullptr, npw, P, nb, 0, kb.occ[0]);
        TM_LAUNCH(k_occ, gr, dim3(128), 0, st, s.evc[pmkq], npw, d_map_mkq, npw, P, nb, 1, kb.occ[1]);
        if (s.nproj > 0) {
            double2* vk = dev_upload(s, s.h_vkb[pkq].data(), s.h_vkb[pkq].size());
            kb.vkb = dev_alloc<double2>(s, (size_t)s.nproj * P);
            TM_LAUNCH(k_pad_copy, dim3((P + 127) / 128, s.nproj), dim3(128), 0, st, vk, npw, P, s.nproj,
                               kb.vkb);
        }
        // plane position -> column of the k+q sphere (wave-local plane kernels)
        std::vector<short> ci((size_t)s.n1 * s.n2, (short)-1);
        for (int c = 0; c < kb.sph_kq.ncol; ++c) ci[kb.sph_kq.h_col_pos[c]] = (short)c;
        short* d_ci = dev_upload(s, ci.data(), ci.size());
        for (int side = 0; side < 2; ++side) {
            int b = side * nk + ik;
            t_colidx[b] = d_ci;
            t_colptr_kq[b] = kb.sph_kq.col_ptr;
            t_entg_kq[b] = kb.sph_kq.ent_g;
            t_enti3_kq[b] = kb.sph_kq.ent_i3;
            t_colpos_kq[b] = kb.sph_kq.col_pos;
            t_ncol_kq[b] = kb.sph_kq.ncol;
            t_npw_kq[b] = npw;
            t_colptr_u[b] = kb.sph_u[side].col_ptr;
            t_entg_u[b] = kb.sph_u[side].ent_g;
            t_enti3_u[b] = kb.sph_u[side].ent_i3;
            t_colpos_u[b] = kb.sph_u[side].col_pos;
            t_ncol_u[b] = kb.sph_u[side].ncol;
            t_npw_u[b] = kb.npw_u[side];
            t_ucoef[b] = kb.u_coef[side];
            t_kin[b] = kb.kin;
            t_eps[b] = kb.eps[side];
            t_occ[b] = kb.occ[side];
            t_vkb[b] = kb.vkb;
            t_maps[b] = side == 0 ? kb.map_k : kb.map_mk;
            t_rows_kq[b] = kb.sph_kq.rows;
            t_nrows_kq[b] = kb.sph_kq.nrows;
            t_rmask_kq[b] = kb.sph_kq.rmask;
            t_rows_u[b] = kb.sph_u[side].rows;
            t_nrows_u[b] = kb.sph_u[side].nrows;
            t_rmask_u[b] = kb.sph_u[side].rmask;
            // the real-space ground state of a batch depends only on its point,
            // its G shift and the side (time reversal on the y side)
            const int* gs = sh ? sh + 3 * side : nullptr;
            std::array<int, 5> key{side == 0 ? pk : pmk, gs ? gs[0] : 0, gs ? gs[1] : 0, gs ? gs[2] : 0, side};
            auto it = s.uslot_of.find(key);
            if (it == s.uslot_of.end()) it = s.uslot_of.emplace(key, (int)s.uslot_of.size()).first;
            t_uslot[b] = it->second;
        }
    }
    q.ncol_max = col_stride(q.ncol_max);
    q.d_uslot = dev_upload(s, t_uslot.data(), t_uslot.size());
    q.d_colidx_kq = upload_table(s, t_colidx);
    q.d_rows_kq = upload_table(s, t_rows_kq);
    q.d_rows_u = upload_table(s, t_rows_u);
    q.d_nrows_kq = dev_upload(s, t_nrows_kq.data(), t_nrows_kq.size());
    q.d_nrows_u = dev_upload(s, t_nrows_u.data(), t_nrows_u.size());
    q.d_rmask_kq = dev_upload(s, t_rmask_kq.data(), t_rmask_kq.size());
    q.d_rmask_u = dev_upload(s, t_rmask_u.data(), t_rmask_u.size());
    q.d_colptr_kq = upload_table(s, t_colptr_kq);
    q.d_entg_kq = upload_table(s, t_entg_kq);
    q.d_enti3_kq = upload_table(s, t_enti3_kq);
    q.d_colpos_kq = upload_table(s, t_colpos_kq);
    q.d_ncol_kq = dev_upload(s, t_ncol_kq.data(), t_ncol_kq.size());
    q.d_npw_kq = dev_upload(s, t_npw_kq.data(), t_npw_kq.size());
    q.d_colptr_u = upload_table(s, t_colptr_u);
    q.d_entg_u = upload_table(s, t_entg_u);
    q.d_enti3_u = upload_table(s, t_enti3_u);
    q.d_colpos_u = upload_table(s, t_colpos_u);
    q.d_ncol_u = dev_upload(s, t_ncol_u.data(), t_ncol_u.size());
    q.d_npw_u = dev_upload(s, t_npw_u.data(), t_npw_u.size());
    q.d_ucoef = dev_upload(s, t_ucoef.data(), t_ucoef.size());
    q.d_kin = upload_table(s, t_kin);
    q.d_eps = upload_table(s, t_eps);
    q.d_occ = upload_table(s, t_occ);
    q.d_vkb = upload_table(s, t_vkb);
    q.d_maps = upload_table(s, t_maps);
    q.hq = dev_alloc<double>(s, s.N);
    launch_coulomb_setup(s, q, st);
    const double* hq = q.hq;
    q.d_hqt = dev_upload(s, &hq, 1);
    q.hmod = 1;
}

}  // namespace

// Workspace of the apply, sized once for every q set of the system: captured
// chain graphs keep its pointers, so it is never reallocated afterwards.
static void free_workspace(Workspace& w) {
    void* wp[] = {w.xcols, w.rho_part, w.rho, w.W, w.work, w.gpart, w.gsmall, w.dots, w.dotpart, w.fields};
    for (void* p : wp)
        if (p) (void)hipFree(p);
    w = Workspace{};
}

// Makes slot j's workspace the one the launches use (see System::ws).
static void select_slot(System& s, int j) {
    if ((int)s.wslot.size() <= j) s.wslot.resize(j + 1);
    if (j == s.wcur) return;
    s.wslot[s.wcur] = s.ws;
    s.ws = s.wslot[j];
    s.wcur = j;
}

// Buffer sizes of a workspace for nrhs right-hand sides over all q sets
// (element counts in w.cap_*, w.nchunk); returns the device bytes it holds.
static size_t plan_workspace(const System& s, int nrhs, Workspace& w) {
    const int nb = s.nbnd;
    int nb2 = 0, ncol_max = 0, npw_pad = 0;
    for (const QSet& q : s.qs) {
        nb2 = std::max(nb2, 2 * q.nk);
        ncol_max = std::max(ncol_max, q.ncol_max);
        npw_pad = std::max(npw_pad, q.npw_pad);
    }
    long long blocks_per_chunk = (long long)s.n3 * nb2;
    // band chunks of the plane kernels: about 2048 blocks per right-hand side,
    // but at least two bands per chunk (a block's set-up is then shared; on the
    // 20^3 system 4 chunks of 2 bands: 7515 applies/s, 8 of 1: 7219); grids
    // with many planes and sides get one chunk
    w.nchunk = (int)std::min<long long>(std::max(1, nb / 2),
                                        std::max<long long>(1, (2048 + blocks_per_chunk - 1) / blocks_per_chunk));
    const size_t R = (size_t)nrhs;
    w.cap_xcols = R * nb2 * 2 * nb * s.n3 * ncol_max;
    w.cap_rho_part = R * nb2 * w.nchunk * 4 * s.N;
    w.cap_gpart = R * std::max(gemm_partial_elems(nb2, nb, nb, 2 * npw_pad),
                               gemm_partial_elems(nb2, std::max(s.nproj, 1), 2 * nb, npw_pad));
    w.cap_gsmall = R * std::max((size_t)nb2 * nb * nb, (size_t)2 * nb2 * std::max(s.nproj, 1) * 2 * nb);
    w.bytes = (w.cap_xcols + w.cap_rho_part + w.cap_gpart + w.cap_gsmall + R * 9 * s.N) * sizeof(double2);
    size_t all = w.bytes + (64 + kPartBlocks * 8) * sizeof(double2);
    if (plane_fixed_supported(s.n1, s.n2)) all += R * 6 * s.N * sizeof(double2);
    return all;
}

// Sized for nrhs right-hand sides over all q sets.  Growing it frees the old
// buffers (after the device is idle) and bumps the epoch, so chains re-capture
// their step graphs, which hold its pointers.
void ensure_workspace(System& s, const QSet&, int nrhs) {
    Workspace& w = s.ws;
    if (w.rho && w.width >= nrhs) return;
    if (w.rho) {
        TM_HIP(hipDeviceSynchronize());
        const int epoch = w.epoch;
        free_workspace(w);
        w.epoch = epoch + 1;
    }
    w.width = nrhs;
    const size_t R = (size_t)nrhs;
    const size_t all = plan_workspace(s, nrhs, w);
    auto grab = [&](void** p, size_t bytes) {
        if (hipMalloc(p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            throw Error{TM_ENOMEM, "hipMalloc of the apply workspace failed"};
        }
    };
    grab((void**)&w.xcols, w.cap_xcols * sizeof(double2));
    grab((void**)&w.rho_part, w.cap_rho_part * sizeof(double2));
    grab((void**)&w.gpart, w.cap_gpart * sizeof(double2));
    grab((void**)&w.gsmall, w.cap_gsmall * sizeof(double2));
    grab((void**)&w.W, R * 4 * s.N * sizeof(double2));
    grab((void**)&w.work, R * s.N * sizeof(double2));
    grab((void**)&w.dots, 64 * sizeof(double2));
    grab((void**)&w.dotpart, kPartBlocks * 8 * sizeof(double2));
    if (plane_fixed_supported(s.n1, s.n2)) grab((void**)&w.fields, R * 6 * s.N * sizeof(double2));
    w.alloc_bytes = all;
    grab((void**)&w.rho, R * 4 * s.N * sizeof(double2));  // last: marks the workspace complete
}

// Ground-state planes for the plane kernels.  With fixed-size plane kernels
// and enough device memory the bands are kept in real space (one inverse
// transform per band for the lifetime of the system instead of one per
// apply); otherwise their z-transformed columns are kept and the plane
// kernels finish the inverse transform on every apply.
static void ensure_ground(System& s, QSet& q, hipStream_t st) {
    if (q.ground_ready) return;
    const size_t NP = (size_t)s.n1 * s.n2;
    if (s.ureal_mode == 0) {
        const size_t need = s.uslot_of.size() * (size_t)s.nbnd * s.n3 * 2 * NP * sizeof(double2);
        size_t limit = 0;
        if (s.resident_limit < 0) {
            size_t fr = 0, tot = 0;
            TM_HIP(hipMemGetInfo(&fr, &tot));
            // leave room for the column caches built on the way and for chains
            const size_t ucol = (size_t)2 * q.nk * 2 * s.nbnd * s.n3 * q.ncol_u_max * sizeof(double2);
            limit = fr > ucol ? (size_t)(0.8 * (double)(fr - ucol)) : 0;
        } else {
            limit = (size_t)s.resident_limit;
        }
        const bool res = plane_fixed_supported(s.n1, s.n2) && need > 0 && need <= limit;
        if (res) {
            void* p = nullptr;
            if (hipMalloc(&p, need) == hipSuccess) {
                s.ureal = static_cast<double2*>(p);
                s.ureal_bytes = need;
            } else {
                (void)hipGetLastError();
            }
        }
        s.ureal_mode = s.ureal ? 1 : 2;
    }
    if (!q.ucols) {
        const size_t need = (size_t)2 * q.nk * 2 * s.nbnd * s.n3 * q.ncol_u_max;
        TM_HIP(hipMalloc(&q.ucols, need * sizeof(double2)));
        q.ucols_bytes = need * sizeof(double2);
        launch_zpass_inv(s, q, true, nullptr, 0, 2 * s.nbnd, 0, q.ucols, st);
    }
    if (s.ureal_mode == 1) {
        launch_ureal(s, q, st);
        TM_HIP(hipStreamSynchronize(st));
        TM_HIP(hipFree(q.ucols));
        q.ucols = nullptr;
        q.ucols_bytes = 0;
    }
    q.ground_ready = true;
}

// The batch tables of a lane group: a chain whose lane r carries q set
// iqs[r].  Every per-batch table the resident apply reads (spheres, columns,
// kinetic energies and eigenvalues, occupied partners, projectors, plane rows
// and resident slots) is laid out lane after lane, so that batch b of the
// group (lane b / 2nk, side and k point b % 2nk) finds its row at b; the
// Coulomb multiplier is per lane.  Built once per distinct list of q sets and
// kept with the system.
template <class T>
static T* cat_table(System& s, const std::vector<int>& iqs, T* QSet::*f, int nb2) {
    std::vector<T> h(iqs.size() * (size_t)nb2);
    for (size_t r = 0; r < iqs.size(); ++r)
        TM_HIP(hipMemcpy(h.data() + r * nb2, s.qs[iqs[r]].*f, nb2 * sizeof(T), hipMemcpyDeviceToHost));
    return dev_upload(s, h.data(), h.size());
}

static QSet& lane_group(System& s, const std::vector<int>& iqs) {
    auto it = s.groups.find(iqs);
    if (it != s.groups.end()) return *it->second;
    auto g = std::make_unique<QSet>();
    const QSet& q0 = s.qs[iqs[0]];
    const int nb2 = 2 * q0.nk;
    g->nk = q0.nk;
    g->npw_pad = q0.npw_pad;
    g->tmod = (int)iqs.size() * nb2;
    g->members = iqs;
    g->ncol_max = 0;
    g->ncol_u_max = 0;
    g->lam = 0.0;
    for (int iq : iqs) {
        g->ncol_max = std::max(g->ncol_max, s.qs[iq].ncol_max);
        g->ncol_u_max = std::max(g->ncol_u_max, s.qs[iq].ncol_u_max);
    }
    g->d_colptr_kq = cat_table(s, iqs, &QSet::d_colptr_kq, nb2);
    g->d_entg_kq = cat_table(s, iqs, &QSet::d_entg_kq, nb2);
    g->d_enti3_kq = cat_table(s, iqs, &QSet::d_enti3_kq, nb2);
    g->d_colpos_kq = cat_table(s, iqs, &QSet::d_colpos_kq, nb2);
    g->d_ncol_kq = cat_table(s, iqs, &QSet::d_ncol_kq, nb2);
    g->d_npw_kq = cat_table(s, iqs, &QSet::d_npw_kq, nb2);
    g->d_kin = cat_table(s, iqs, &QSet::d_kin, nb2);
    g->d_eps = cat_table(s, iqs, &QSet::d_eps, nb2);
    g->d_occ = cat_table(s, iqs, &QSet::d_occ, nb2);
    g->d_vkb = cat_table(s, iqs, &QSet::d_vkb, nb2);
    g->d_nrows_kq = cat_table(s, iqs, &QSet::d_nrows_kq, nb2);
    g->d_rmask_kq = cat_table(s, iqs, &QSet::d_rmask_kq, nb2);
    g->d_rows_kq = cat_table(s, iqs, &QSet::d_rows_kq, nb2);
    g->d_colidx_kq = cat_table(s, iqs, &QSet::d_colidx_kq, nb2);
    g->d_uslot = cat_table(s, iqs, &QSet::d_uslot, nb2);
    std::vector<const double*> hq(iqs.size());
    for (size_t r = 0; r < iqs.size(); ++r) hq[r] = s.qs[iqs[r]].hq;
    g->d_hqt = dev_upload(s, hq.data(), hq.size());
    g->hmod = (int)iqs.size();
    QSet& ref = *g;
    s.groups.emplace(iqs, std::move(g));
    return ref;
}

// the ground-state caches an apply on q needs (a lane group: those of its
// q sets, which must be resident)
static void ensure_ground_q(System& s, QSet& q, hipStream_t st) {
    if (q.members.empty()) return ensure_ground(s, q, st);
    for (int iq : q.members) ensure_ground(s, s.qs[iq], st);
    TM_CHECK(s.ureal_mode == 1, TM_EUNSUPPORTED,
             "lanes with different q sets need the resident real-space ground state (fixed-size plane kernels "
             "and room for it on the device)");
}

// index of a q set of the system; a lane group: that of its first lane
static int qset_index(const System& s, const QSet& q) {
    return q.members.empty() ? (int)(&q - s.qs.data()) : q.members[0];
}

// drops the resident real-space ground state (the next apply decides again)
static void reset_ground(System& s) {
    if (s.ureal) {
        TM_HIP(hipDeviceSynchronize());
        TM_HIP(hipFree(s.ureal));
    }
    s.ureal = nullptr;
    s.ureal_bytes = 0;
    s.ureal_mode = 0;
    for (QSet& q : s.qs) q.ground_ready = false;
}

// ---- the allocation-free apply ---------------------------------------------------
// Apply workspace of tm_liouvillian_apply_noalloc: a static device array, one copy
// per device (each GPU the library runs on holds it until the process ends).
// Host code never uses its name as an address: the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::unordered_map<int, char*> g_scratch_ptr;  // device -> address of its scratch copy

char* scratch_address(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) return it->second;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        throw Error{TM_EDEVICE, std::string("hipGetSymbolAddress of the apply scratch failed: ") +
                                    hipGetErrorString(e)};
    g_scratch_ptr[device] = static_cast<char*>(ptr);
    return static_cast<char*>(ptr);
}

// a one-right-hand-side workspace carved out of `base` (256-byte aligned pieces)
Workspace scratch_workspace(const System& s, char* base, size_t cap) {
    Workspace w;
    plan_workspace(s, 1, w);
    size_t off = 0;
    auto take = [&](size_t elems) {
        double2* p = reinterpret_cast<double2*>(base + off);
        off += (elems * sizeof(double2) + 255) / 256 * 256;
        return p;
    };
    w.xcols = take(w.cap_xcols);
    w.rho_part = take(w.cap_rho_part);
    w.gpart = take(w.cap_gpart);
    w.gsmall = take(w.cap_gsmall);
    w.W = take(4 * (size_t)s.N);
    w.work = take((size_t)s.N);
    w.dots = take(64);
    w.dotpart = take(kPartBlocks * 8);
    if (plane_fixed_supported(s.n1, s.n2)) w.fields = take(6 * (size_t)s.N);
    w.rho = take(4 * (size_t)s.N);
    w.width = 1;
    w.alloc_bytes = off;
    TM_CHECK(off <= cap, TM_EUNSUPPORTED,
             "the system's apply workspace (" + std::to_string(off) + " bytes) exceeds the " +
                 std::to_string(cap) + "-byte scratch of the allocation-free apply");
    return w;
}
}  // namespace

static void apply_l_ready(System& s, QSet& q, const double2* in, double2* out, bool fp32, hipStream_t st,
                          int nrhs);

// ---- the autotuner ---------------------------------------------------------------
// Times every compiled variant of each tunable launch of one FP64 apply on the
// system's own data (after a warm-up, at least three runs each and about 2 ms
// of runs for short launches; HIP events on the apply's stream) and keeps the
// fastest per shape, once per shape and process:
// plane density and apply kernels, the two z passes, the projector and P_c
// contractions.  `out` (one right-hand side) is scratch here; the caller's
// apply recomputes it with the chosen variants.
// nrhs > 1 (a chain's first apply with that many lanes): the plane and
// z-pass launches of that many right-hand sides, whose best shapes differ
// from one right-hand side's once the grid fills the device; the
// contractions keep the one-right-hand-side choice (their K split decides
// the rounding, and a lane must round as its chain alone does).
static void autotune(System& s, QSet& q, const double2* in, double2* out, hipStream_t st, int nrhs) {
    hipEvent_t e0, e1;
    TM_HIP(hipEventCreate(&e0));
    TM_HIP(hipEventCreate(&e1));
    struct Ev {
        hipEvent_t a, b;
        ~Ev() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } ev{e0, e1};
    apply_l_ready(s, q, in, out, false, st, nrhs);  // every buffer holds this system's data
    const long long bstride = (long long)s.nbnd * 2 * q.npw_pad;
    struct Op {
        int op;
        const char* what;
        std::function<void()> run;
    };
    const Op ops[] = {
        {kTuneZInv, "z inverse",
         [&] { launch_zpass_inv(s, q, false, in, bstride, 2 * s.nbnd, q.npw_pad, s.ws.xcols, st, false, nrhs); }},
        {kTuneDensity, "density planes", [&] { launch_density(s, q, st, false, nrhs); }},
        {kTuneApply, "apply planes", [&] { launch_apply_planes(s, q, st, false, nrhs); }},
        {kTuneZFwd, "z forward", [&] { launch_zpass_fwd(s, q, s.ws.xcols, in, out, st, false, nrhs); }},
        {kTuneGemm, "P_c contraction", [&] { launch_project(s, q, out, st); }},
        {kTuneGemm, "projector contraction", [&] { launch_nonlocal(s, q, in, out, st); }},
        {kTuneUpd, "P_c update", [&] { launch_project(s, q, out, st); }},
        {kTuneUpd, "projector update", [&] { launch_nonlocal(s, q, in, out, st); }},
    };
    for (const Op& o : ops) {
        if (nrhs > 1 && (o.op == kTuneGemm || o.op == kTuneUpd)) continue;
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            g_seen_n[o.op] = 0;
        }
        o.run();  // the default variant; records the launch's shape key and variant count
        long long key;
        int n;
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            key = g_seen_key[o.op];
            n = g_seen_n[o.op];
            if (n <= 1 || g_force[o.op] >= 0 || g_tuned.count({o.op, key})) continue;
        }
        std::vector<float> us(n);
        // runs per variant: at least 3, and for short launches enough for about
        // 2 ms, so that launch gaps and timer resolution do not decide
        auto timed = [&](int reps) {
            TM_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r) o.run();
            TM_HIP(hipEventRecord(e1, st));
            TM_HIP(hipEventSynchronize(e1));
            float ms = 0;
            TM_HIP(hipEventElapsedTime(&ms, e0, e1));
            return ms * 1000.0f / (float)reps;
        };
        try {
            g_trial[o.op] = 0;
            const float t1 = timed(1);
            const int reps = (int)std::min(200.0f, std::max(3.0f, 2000.0f / std::max(t1, 1.0f)));
            for (int v = 0; v < n; ++v) {
                g_trial[o.op] = v;
                o.run();
                us[v] = timed(reps);
            }
        } catch (...) {
            g_trial[o.op] = -1;
            throw;
        }
        g_trial[o.op] = -1;
        TuneEntry t;
        t.op = o.op;
        t.key = key;
        t.nvariants = n;
        t.chosen = (int)(std::min_element(us.begin(), us.end()) - us.begin());
        t.us = us;
        t.shape = std::string(o.what) + " grid " + std::to_string(s.n1) + "x" + std::to_string(s.n2) + "x" +
                  std::to_string(s.n3) + ", " + std::to_string(s.nbnd) + " bands, " + std::to_string(q.nk) + " k" +
                  (nrhs > 1 ? ", " + std::to_string(nrhs) + " right-hand sides" : "");
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[{o.op, key}] = t;
    }
}

static void start_vectors_raw(System& s, int iq, int dir, double2* u, double2* v, hipStream_t st);

// Runs the autotuner on the system (once; FP64; never inside a graph capture,
// where nothing can be timed) before any tunable launch of it produces a
// result: the start vectors' projection, the first apply, a chain's first
// step.  Every result of a tuned system then comes from the same launch
// variants, so it does not depend on which call happened to come first.
// in/out: one right-hand side to time on (out is overwritten), or null for
// scratch vectors allocated here and freed before returning.
static void ensure_tuned(System& s, int iq, hipStream_t st, const double2* in = nullptr, double2* out = nullptr) {
    if (s.tuned || !g_autotune) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    TM_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) return;
    QSet& q = s.qs[iq];
    ensure_workspace(s, q, 1);
    ensure_ground(s, q, st);
    if (in && out) {
        autotune(s, q, in, out, st, 1);
        s.tuned = true;
        return;
    }
    const size_t bytes = (size_t)2 * q.nk * s.nbnd * 2 * q.npw_pad * sizeof(double2);
    struct Scratch {
        double2* p[2] = {nullptr, nullptr};
        hipStream_t st;
        ~Scratch() {
            (void)hipStreamSynchronize(st);
            for (double2* x : p)
                if (x) (void)hipFree(x);
        }
    } sc{{nullptr, nullptr}, st};
    for (double2*& x : sc.p)
        if (hipMalloc((void**)&x, bytes) != hipSuccess) {
            (void)hipGetLastError();
            x = nullptr;
            throw Error{TM_ENOMEM, "hipMalloc of the autotuner's vectors failed"};
        }
    start_vectors_raw(s, iq, TM_DIR_Z, nullptr, sc.p[0], st);
    autotune(s, q, sc.p[0], sc.p[1], st, 1);
    s.tuned = true;
}

// the launch shapes of nrhs right-hand sides, timed at the system's first
// FP64 apply of that many (one size class per power of two), on the caller's
// vectors (out is recomputed by the caller's apply)
static void ensure_tuned_rhs(System& s, QSet& q, const double2* in, double2* out, hipStream_t st, int nrhs) {
    if (nrhs <= 1 || !g_autotune || s.tuned_rhs.count(rhs_class(nrhs))) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    TM_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) return;
    autotune(s, q, in, out, st, nrhs);
    s.tuned_rhs.insert(rhs_class(nrhs));
}

// out = L_q in.  fp32: the FFTs, densities, point-wise products and the
// nonlocal/projector contractions run in single precision (FP32 MFMA, FP32
// accumulation); the potential (Hartree + kernel), the kinetic term and the
// vectors stay FP64.  Needs the fixed-size kernels and the resident ground state.
// q: a q set of the system (every right-hand side on it) or a lane group
// (right-hand side r on q set q.members[r])
static void apply_l(System& s, QSet& q, const double2* in, double2* out, bool fp32, hipStream_t st, int nrhs) {
    ensure_workspace(s, q, nrhs);
    ensure_ground_q(s, q, st);
    if (fp32)
        TM_CHECK(s.ureal_mode == 1 && zpass_fixed_supported(s.n3), TM_EUNSUPPORTED,
                 "TM_FP32 needs fixed-size plane and z kernels and the resident ground state");
    else {
        ensure_tuned(s, qset_index(s, q), st, in, out);
        ensure_tuned_rhs(s, q, in, out, st, nrhs);
    }
    apply_l_ready(s, q, in, out, fp32, st, nrhs);
}

void apply_l(System& s, int iq, const double2* in, double2* out, bool fp32, hipStream_t st, int nrhs) {
    apply_l(s, s.qs[iq], in, out, fp32, st, nrhs);
}

// the launches of one apply; the workspace (s.ws) and the ground-state caches
// of the q set are in place (nothing is allocated here)
static void apply_l_ready(System& s, QSet& q, const double2* in, double2* out, bool fp32, hipStream_t st,
                          int nrhs) {
    const long long bstride = (long long)s.nbnd * 2 * q.npw_pad;
    launch_zpass_inv(s, q, false, in, bstride, 2 * s.nbnd, q.npw_pad, s.ws.xcols, st, fp32, nrhs);
    launch_density(s, q, st, fp32, nrhs);
    launch_potential(s, q, st, nrhs);
    launch_apply_planes(s, q, st, fp32, nrhs);
    launch_zpass_fwd(s, q, s.ws.xcols, in, out, st, fp32, nrhs);
    launch_nonlocal(s, q, in, out, st, fp32, nrhs);
    launch_project(s, q, out, st, fp32, nrhs);
}

static void start_vectors_raw(System& s, int iq, int dir, double2* u, double2* v, hipStream_t st) {
    QSet& q = s.qs[iq];
    ensure_workspace(s, q);
    dim3 gr((q.npw_pad + 127) / 128, s.nbnd, 2 * q.nk);
    // lower-side signs: u^l = (s U, t_l s T U), v^m = (P s U, -t_m P+ s T U) with the
    // time-reversal parity t = -1 of the spin matrices and +1 of sigma_0
    const double t = dir == TM_DIR_N ? 1.0 : -1.0;
    TM_LAUNCH(k_start, gr, dim3(128), 0, st, q.d_ucoef, q.d_npw_u, (const int* const*)q.d_maps, q.nk,
                       s.nbnd, q.npw_pad, dir, t, -t, u, v);
    if (v) launch_project_signed(s, q, v, 1.0, 1.0, st);
}

void start_vectors(System& s, int iq, int dir, double2* u, double2* v, hipStream_t st) {
    if (v) ensure_tuned(s, iq, st);  // the projection of v is a tuned contraction
    start_vectors_raw(s, iq, dir, u, v, st);
}

// Steps after which the vector roles of a chain return to their initial
// assignment (pH: q_prev, q, r rotate in 3, Lq, Lr in 2; nH: two 3-cycles).
constexpr int kPeriodPH = 6, kPeriodNH = 3;

// One Lanczos chain (Sec. 2.5) resident on the device: its vectors, the four
// measure vectors u^lambda, the coefficient arrays and the scale/step state.
// A chain may carry several lanes: independent recursions for several field
// directions (the columns of the susceptibility tensor) that step together,
// so that every application of L runs on all of them at once (the plane,
// z-pass and contraction kernels take the lanes as extra batches and read the
// ground state and the projectors once for all).  Work vector i of lane r
// sits at vec[i] + r n.  Steps are issued asynchronously; step indices and
// breakdown flags live on the device, so a chain never returns to the host
// until its coefficients are read.
struct Chain {
    System* s = nullptr;
    int iq = 0, flavour = 0, cap = 0;  // iq: the q set of lane 0
    int lanes = 1;
    int dir[kMaxChainLanes] = {};
    int lane_iq[kMaxChainLanes] = {};  // the q set of each lane
    QSet* qa = nullptr;        // what the applies run on: the lanes' q set, or their lane group
    long long ustride = 0;     // 0: measure vectors shared by the lanes (one q set); n: one per lane
    bool fp32 = false;         // single-precision applies (recurrence and dots stay FP64)
    long long n = 0, half = 0;
    double w = 1.0;
    std::vector<double2*> vec;  // work vectors (5 pH, 9 nH), each [lanes][n]
    int ix[9] = {0, 1, 2, 3, 4, 5, 6, 7, 8};  // current role -> vector
    double2* u[kNMeasure] = {};  // measure vectors u^l, l = x, y, z, n (lane r's at u[l] + r ustride)
    Coeffs co{};               // [lanes] coefficient arrays
    ChainState* cs = nullptr;  // [lanes]
    double2* dots = nullptr;   // [lanes][kDotStride] reduced inner products
    double2* part = nullptr;   // [lanes][blocks x values] partial sums
    int issued = 0;            // steps issued so far
    int broken_seen = 0;       // breakdown observed on the host
    hipStream_t last = nullptr;
    hipGraphExec_t gexec = nullptr;  // one period of steps, captured
    int gepoch = -1;                 // workspace epoch the graph was captured against
    int slot = 0;                    // the system's workspace slot (and stream inside tm_chains_step)
    std::vector<void*> mem;

    void* alloc(size_t bytes) {
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            throw Error{TM_ENOMEM, "hipMalloc failed for a Lanczos chain"};
        }
        mem.push_back(p);
        return p;
    }
    ~Chain() {
        if (!mem.empty()) (void)hipStreamSynchronize(last);
        if (gexec) (void)hipGraphExecDestroy(gexec);
        for (void* p : mem) (void)hipFree(p);
    }
    // steps after which the vector roles return to their initial assignment
    int period() const { return flavour == TM_PSEUDOHERMITIAN ? kPeriodPH : kPeriodNH; }
    int nvec() const { return flavour == TM_PSEUDOHERMITIAN ? 5 : 9; }
    double2* V(int role) const { return vec[ix[role]]; }
};

// device memory of a chain: vectors, coefficients and state
static void chain_alloc(Chain& c) {
    const size_t L = (size_t)c.lanes, cap = (size_t)c.cap;
    for (int i = 0; i < c.nvec(); ++i) c.vec.push_back(static_cast<double2*>(c.alloc(L * c.n * sizeof(double2))));
    const size_t UL = c.ustride ? L : 1;
    for (int l = 0; l < kNMeasure; ++l) c.u[l] = static_cast<double2*>(c.alloc(UL * c.n * sizeof(double2)));
    c.co.cap = c.cap;
    c.co.alpha = static_cast<double2*>(c.alloc(L * cap * sizeof(double2)));
    c.co.beta = static_cast<double*>(c.alloc(L * cap * sizeof(double)));
    c.co.gamma = static_cast<double2*>(c.alloc(L * cap * sizeof(double2)));
    c.co.z = static_cast<double2*>(c.alloc(L * kNMeasure * cap * sizeof(double2)));
    c.cs = static_cast<ChainState*>(c.alloc(L * sizeof(ChainState)));
    c.dots = static_cast<double2*>(c.alloc(L * kDotStride * sizeof(double2)));
    c.part = static_cast<double2*>(c.alloc(L * kPartBlocks * 8 * sizeof(double2)));
}

static void chain_clear_coeffs(Chain& c, hipStream_t st) {
    const size_t L = (size_t)c.lanes, cap = (size_t)c.cap;
    TM_HIP(hipMemsetAsync(c.co.alpha, 0, L * cap * sizeof(double2), st));
    TM_HIP(hipMemsetAsync(c.co.beta, 0, L * cap * sizeof(double), st));
    TM_HIP(hipMemsetAsync(c.co.gamma, 0, L * cap * sizeof(double2), st));
    TM_HIP(hipMemsetAsync(c.co.z, 0, L * kNMeasure * cap * sizeof(double2), st));
}

// Chains of a system whose workspace is small are spread over up to
// slot_cap workspace slots, which run concurrently inside tm_chains_step (a
// small system's step leaves most of the device idle); others keep one.
constexpr size_t kSlotBytes = 256u << 20;

static void chain_bind_slot(Chain& c, const QSet& q) {
    System& s = *c.s;
    if (s.nslots == 0) {
        select_slot(s, 0);
        ensure_workspace(s, q, c.lanes);
        s.nslots = s.ws.bytes <= kSlotBytes ? s.slot_cap : 1;
    }
    c.slot = s.next_slot++ % s.nslots;
    select_slot(s, c.slot);
    ensure_workspace(s, q, c.lanes);
}

// Lane q sets of a chain (c.lane_iq, c.lanes set): the q set of lane 0, the
// vector length, and what the applies run on -- the lanes' common q set, or
// the lane group of their q sets (then each lane has its own measure vectors)
static void chain_qsets(Chain& c) {
    System& s = *c.s;
    TM_CHECK(c.lanes >= 1 && c.lanes <= kMaxChainLanes, TM_EINVAL,
             "1 to " + std::to_string(kMaxChainLanes) + " lanes per chain");
    bool mixed = false;
    for (int r = 0; r < c.lanes; ++r) {
        TM_CHECK(c.lane_iq[r] >= 0 && c.lane_iq[r] < (int)s.qs.size(), TM_EINVAL, "lane q set out of range");
        mixed |= c.lane_iq[r] != c.lane_iq[0];
    }
    c.iq = c.lane_iq[0];
    const QSet& q = s.qs[c.iq];
    c.n = 2LL * q.nk * s.nbnd * 2 * q.npw_pad;  // the same for every q set of the system
    c.half = c.n / 2;
    c.w = 1.0 / q.nk;
    c.qa = mixed ? &lane_group(s, std::vector<int>(c.lane_iq, c.lane_iq + c.lanes)) : &s.qs[c.iq];
    c.ustride = mixed ? c.n : 0;
}

static void chain_begin(Chain& c, hipStream_t st) {
    System& s = *c.s;
    chain_qsets(c);
    QSet& q = s.qs[c.iq];
    chain_bind_slot(c, q);
    ensure_ground_q(s, *c.qa, st);  // before any step, so steps never allocate or synchronise
    if (!c.fp32) ensure_tuned(s, c.iq, st);  // before the chain's vectors exist (its scratch is freed)
    chain_alloc(c);
    c.last = st;
    chain_clear_coeffs(c, st);
    std::vector<ChainState> h(c.lanes);
    for (int r = 0; r < c.lanes; ++r) h[r].lam = s.qs[c.lane_iq[r]].lam;
    TM_HIP(hipMemcpyAsync(c.cs, h.data(), h.size() * sizeof(ChainState), hipMemcpyHostToDevice, st));
    TM_HIP(hipStreamSynchronize(st));  // h is released on return
    const int mdir[kNMeasure] = {TM_DIR_X, TM_DIR_Y, TM_DIR_Z, TM_DIR_N};
    for (int l = 0; l < kNMeasure; ++l) {
        if (c.ustride == 0) {
            start_vectors(s, c.iq, mdir[l], c.u[l], nullptr, st);
        } else {
            for (int r = 0; r < c.lanes; ++r)
                start_vectors(s, c.lane_iq[r], mdir[l], c.u[l] + r * c.ustride, nullptr, st);
        }
    }
    const long long n = c.n, half = c.half, L = c.lanes, us = c.ustride;
    double2* d = c.dots;
    if (c.flavour == TM_PSEUDOHERMITIAN) {
        // roles: 0 q_prev, 1 q, 2 Lq, 3 r, 4 Lr
        TM_HIP(hipMemsetAsync(c.V(0), 0, L * n * sizeof(double2), st));
        for (int r = 0; r < c.lanes; ++r) start_vectors(s, c.lane_iq[r], c.dir[r], nullptr, c.V(1) + r * n, st);
        apply_l(s, *c.qa, c.V(1), c.V(2), c.fp32, st, c.lanes);
        DotSet<7> ds0{{c.V(1), c.V(1), c.V(2), c.u[0], c.u[1], c.u[2], c.u[3]},
                      {c.V(2), c.V(1), c.V(2), c.V(1), c.V(1), c.V(1), c.V(1)},
                      {1, 0, 1, 0, 0, 0, 0},
                      {n, n, n, us, us, us, us},
                      {n, n, n, n, n, n, n}};
        run_multidot<7>(ds0, n, half, c.w, c.part, d, st, c.lanes);
        ctl_ph_start(c.cs, d, c.co, st, c.lanes);
    } else {
        // roles: 0 q_prev, 1 q, 2 p_prev, 3 p, 4 Lq, 5 L^dag p, 6 J p, 7 q^, 8 p^
        TM_HIP(hipMemsetAsync(c.V(0), 0, L * n * sizeof(double2), st));
        TM_HIP(hipMemsetAsync(c.V(2), 0, L * n * sizeof(double2), st));
        for (int r = 0; r < c.lanes; ++r) start_vectors(s, c.lane_iq[r], c.dir[r], nullptr, c.V(1) + r * n, st);
        TM_HIP(hipMemcpyAsync(c.V(3), c.V(1), L * n * sizeof(double2), hipMemcpyDeviceToDevice, st));
        DotSet<5> ds0{{c.V(1), c.u[0], c.u[1], c.u[2], c.u[3]},
                      {c.V(1), c.V(1), c.V(1), c.V(1), c.V(1)},
                      {0, 0, 0, 0, 0},
                      {n, us, us, us, us},
                      {n, n, n, n, n}};
        run_multidot<5>(ds0, n, half, c.w, c.part, d, st, c.lanes);
        ctl_nh_start(c.cs, d, c.co, st, c.lanes);
    }
}

// one step of the chain (all lanes) on stream st
static void chain_step(Chain& c, hipStream_t st) {
    System& s = *c.s;
    const long long n = c.n, half = c.half;
    const int L = c.lanes;
    double2* d = c.dots;
    const double2* uc[kNMeasure] = {c.u[0], c.u[1], c.u[2], c.u[3]};
    if (c.flavour == TM_PSEUDOHERMITIAN) {
        double2 *QP = c.V(0), *Q = c.V(1), *LQ = c.V(2), *R = c.V(3), *LR = c.V(4);
        // block partials of the update's (u_l, r) and, further on, of the
        // multidot, side by side in c.part; both summed by the step control
        double2* part_up = c.part;
        double2* part_md = c.part + (size_t)L * kPartBlocks * kNMeasure;
        run_ph_update(c.cs, LQ, Q, QP, R, uc, c.ustride, n, part_up, st, L);
        // back onto the empty manifold: removes rounding-level occupied parts
        // that the metric JL cannot see (identity in exact arithmetic)
        launch_project_signed(s, *c.qa, R, 1.0, 1.0, st, false, L);
        apply_l(s, *c.qa, R, LR, c.fp32, st, L);
        DotSet<3> ds{{R, R, LR}, {LR, R, LR}, {1, 0, 1}, {n, n, n}, {n, n, n}};
        run_multidot<3>(ds, n, half, c.w, part_md, d, st, L, false);
        ctl_ph_step_sums(c.cs, part_md, part_up, n, c.w, d, d + 8, c.co, st, L);
        // q_prev <- q, q <- r, Lq <- Lr; the old q_prev and Lq become scratch
        const int oqp = c.ix[0], olq = c.ix[2];
        c.ix[0] = c.ix[1];
        c.ix[1] = c.ix[3];
        c.ix[2] = c.ix[4];
        c.ix[3] = oqp;
        c.ix[4] = olq;
    } else {
        double2 *QP = c.V(0), *Q = c.V(1), *PP = c.V(2), *Pv = c.V(3), *LQ = c.V(4), *LTP = c.V(5),
                *TMP = c.V(6), *QH = c.V(7), *PH = c.V(8);
        // q_i, p_i back onto the empty manifold (see the pH step)
        launch_project_signed(s, *c.qa, Q, 1.0, 1.0, st, false, L);
        launch_project_signed(s, *c.qa, Pv, 1.0, 1.0, st, false, L);
        apply_l(s, *c.qa, Q, LQ, c.fp32, st, L);
        run_jcopy(Pv, TMP, n, half, st, L);
        apply_l(s, *c.qa, TMP, LTP, c.fp32, st, L);
        DotSet<1> da{{Pv}, {LQ}, {0}, {n}, {n}};
        run_multidot<1>(da, n, half, c.w, c.part, d, st, L, false);
        ctl_nh_alpha_sums(c.cs, c.part, n, c.w, d, c.co, st, L);
        run_nh_update(c.cs, LQ, Q, QP, LTP, Pv, PP, QH, PH, uc, c.ustride, n, half, c.part, st, L);
        ctl_nh_step_sums(c.cs, c.part, n, c.w, d + 8, c.co, st, L);
        // q_prev <- q, q <- q^, p_prev <- p, p <- p^
        const int oqp = c.ix[0], opp = c.ix[2];
        c.ix[0] = c.ix[1];
        c.ix[1] = c.ix[7];
        c.ix[2] = c.ix[3];
        c.ix[3] = c.ix[8];
        c.ix[7] = oqp;
        c.ix[8] = opp;
    }
}

// Graph replay of a period of steps.  Small systems spend most of a step in
// launch gaps (about 25 kernels per step); a captured period replays with the
// gaps of a graph.  The step index and the breakdown flag are device state, so
// the replayed kernels need no new arguments; the capture stream is private to
// the system and the replay goes to the caller's stream.
bool g_use_graphs = true;

static void chain_capture(Chain& c) {
    System& s = *c.s;
    if (!s.cap_stream) TM_HIP(hipStreamCreateWithFlags(&s.cap_stream, hipStreamNonBlocking));
    int saved[9];
    std::copy(c.ix, c.ix + 9, saved);
    hipGraph_t g = nullptr;
    TM_HIP(hipStreamBeginCapture(s.cap_stream, hipStreamCaptureModeRelaxed));
    try {
        for (int i = 0; i < c.period(); ++i) chain_step(c, s.cap_stream);
    } catch (...) {
        (void)hipStreamEndCapture(s.cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        std::copy(saved, saved + 9, c.ix);
        throw;
    }
    TM_HIP(hipStreamEndCapture(s.cap_stream, &g));
    TM_CHECK(std::equal(saved, saved + 9, c.ix), TM_EDEVICE, "vector roles did not return after a period");
    hipError_t e = hipGraphInstantiate(&c.gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c.gexec = nullptr;
        throw Error{TM_EDEVICE, std::string("graph instantiation failed: ") + hipGetErrorString(e)};
    }
    c.gepoch = s.ws.epoch;
}

// up to k steps of one chain (never past its capacity)
static void chain_steps(Chain& c, int k, hipStream_t st) {
    select_slot(*c.s, c.slot);
    k = std::min(k, c.cap - c.issued);
    const int P = c.period();
    while (k > 0) {
        if (g_use_graphs && !g_prof_on && c.issued % P == 0 && k >= P) {
            if (c.gexec && c.gepoch != c.s->ws.epoch) {  // the workspace moved since the capture
                (void)hipGraphExecDestroy(c.gexec);
                c.gexec = nullptr;
            }
            if (!c.gexec) chain_capture(c);
            const int r = k / P;
            for (int i = 0; i < r; ++i) TM_HIP(hipGraphLaunch(c.gexec, st));
            c.issued += r * P;
            k -= r * P;
        } else {
            chain_step(c, st);
            ++c.issued;
            --k;
        }
    }
    c.last = st;
}

static std::vector<ChainState> chain_states(Chain& c) {
    std::vector<ChainState> h(c.lanes);
    TM_HIP(hipMemcpyAsync(h.data(), c.cs, h.size() * sizeof(ChainState), hipMemcpyDeviceToHost, c.last));
    TM_HIP(hipStreamSynchronize(c.last));
    return h;
}

// reads the device state; returns 1 once every lane has broken down (a
// broken lane idles: its kernels skip it while the others go on)
static int chain_poll(Chain& c) {
    int all = 1;
    for (const ChainState& h : chain_states(c)) all &= h.broken != 0;
    c.broken_seen = all;
    return all;
}

// out: one tm_coeffs per lane
static int chain_coeffs(Chain& c, tm_coeffs* out) {
    const std::vector<ChainState> hs = chain_states(c);
    const int cap = c.cap;
    const size_t L = (size_t)c.lanes;
    std::vector<double2> ha(L * cap), hg(L * cap), hz(L * kNMeasure * (size_t)cap);
    std::vector<double> hb(L * cap);
    TM_HIP(hipMemcpy(ha.data(), c.co.alpha, ha.size() * sizeof(double2), hipMemcpyDeviceToHost));
    TM_HIP(hipMemcpy(hb.data(), c.co.beta, hb.size() * sizeof(double), hipMemcpyDeviceToHost));
    TM_HIP(hipMemcpy(hg.data(), c.co.gamma, hg.size() * sizeof(double2), hipMemcpyDeviceToHost));
    TM_HIP(hipMemcpy(hz.data(), c.co.z, hz.size() * sizeof(double2), hipMemcpyDeviceToHost));
    int broken = 0, all = 1;
    for (size_t r = 0; r < L; ++r) {
        tm_coeffs* o = out + r;
        const ChainState& h = hs[r];
        broken |= h.broken;
        all &= h.broken != 0;
        o->steps_done = h.step;
        o->n1 = h.n1;
        const int m = std::min(cap, o->capacity);
        const double2* a = ha.data() + r * cap;
        const double* b = hb.data() + r * cap;
        const double2* g = hg.data() + r * cap;
        const double2* z = hz.data() + r * kNMeasure * cap;
        for (int j = 0; j < m; ++j) {
            o->alpha[2 * j] = a[j].x;
            o->alpha[2 * j + 1] = a[j].y;
            o->beta[j] = b[j];
            o->gamma[2 * j] = g[j].x;
            o->gamma[2 * j + 1] = g[j].y;
            for (int l = 0; l < 3; ++l) {
                o->z[2 * ((size_t)l * o->capacity + j)] = z[l * (size_t)cap + j].x;
                o->z[2 * ((size_t)l * o->capacity + j) + 1] = z[l * (size_t)cap + j].y;
            }
            if (o->zn) {
                o->zn[2 * j] = z[3 * (size_t)cap + j].x;
                o->zn[2 * j + 1] = z[3 * (size_t)cap + j].y;
            }
        }
    }
    c.broken_seen = all;
    return broken ? TM_EBREAKDOWN : TM_OK;
}

// ---- checkpoint: header, per-lane device state, coefficients, vectors
struct ChainBlobHeader {
    char magic[8];       // "TMCHAIN4"
    int iq, flavour, fp32, cap, issued, nvec, lanes;
    int dir[kMaxChainLanes];
    int lane_iq[kMaxChainLanes];
    int ix[9];
    long long n;
};

// ulanes: measure vector sets saved (1 shared, or one per lane)
static size_t blob_bytes(int lanes, int cap, int nvec, long long n, int ulanes) {
    const size_t L = (size_t)lanes;
    return sizeof(ChainBlobHeader) + L * sizeof(ChainState) +
           L * (size_t)cap * (2 * sizeof(double2) + sizeof(double) + kNMeasure * sizeof(double2)) +
           (L * nvec + (size_t)kNMeasure * ulanes) * (size_t)n * sizeof(double2);
}

static int ulanes_of(const int* lane_iq, int lanes) {
    for (int r = 1; r < lanes; ++r)
        if (lane_iq[r] != lane_iq[0]) return lanes;
    return 1;
}

static size_t chain_blob_bytes(const Chain& c) {
    return blob_bytes(c.lanes, c.cap, c.nvec(), c.n, c.ustride ? c.lanes : 1);
}

static void chain_save(Chain& c, char* out) {
    TM_HIP(hipStreamSynchronize(c.last));
    ChainBlobHeader h{};
    std::memcpy(h.magic, "TMCHAIN4", 8);
    h.iq = c.iq;
    h.flavour = c.flavour;
    h.fp32 = c.fp32 ? 1 : 0;
    h.cap = c.cap;
    h.issued = c.issued;
    h.nvec = c.nvec();
    h.lanes = c.lanes;
    std::copy(c.dir, c.dir + kMaxChainLanes, h.dir);
    std::copy(c.lane_iq, c.lane_iq + kMaxChainLanes, h.lane_iq);
    std::copy(c.ix, c.ix + 9, h.ix);
    h.n = c.n;
    const size_t L = (size_t)c.lanes, cap = (size_t)c.cap;
    char* p = out;
    auto put = [&](const void* dev, size_t bytes) {
        TM_HIP(hipMemcpy(p, dev, bytes, hipMemcpyDeviceToHost));
        p += bytes;
    };
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    put(c.cs, L * sizeof(ChainState));
    put(c.co.alpha, L * cap * sizeof(double2));
    put(c.co.beta, L * cap * sizeof(double));
    put(c.co.gamma, L * cap * sizeof(double2));
    put(c.co.z, L * kNMeasure * cap * sizeof(double2));
    for (double2* v : c.vec) put(v, L * c.n * sizeof(double2));
    const size_t UL = c.ustride ? L : 1;
    for (int l = 0; l < kNMeasure; ++l) put(c.u[l], UL * c.n * sizeof(double2));
}

// rebuilds a chain from a checkpoint of a chain of the same system; capacity
// may grow (more steps than the original run was sized for)
static void chain_restore(Chain& c, const char* in, size_t bytes, int capacity, hipStream_t st) {
    ChainBlobHeader h{};
    TM_CHECK(bytes >= sizeof(h), TM_EINVAL, "checkpoint too short");
    std::memcpy(&h, in, sizeof(h));
    TM_CHECK(std::memcmp(h.magic, "TMCHAIN4", 8) == 0, TM_EINVAL, "not a chain checkpoint");
    System& s = *c.s;
    TM_CHECK(h.iq >= 0 && h.iq < (int)s.qs.size(), TM_EINVAL, "checkpoint q set not in this system");
    const QSet& q = s.qs[h.iq];
    TM_CHECK(h.n == 2LL * q.nk * s.nbnd * 2 * q.npw_pad, TM_EINVAL, "checkpoint vectors do not fit this system");
    TM_CHECK(h.flavour == TM_PSEUDOHERMITIAN || h.flavour == TM_NONHERMITIAN, TM_EINVAL, "bad flavour");
    TM_CHECK(h.nvec == (h.flavour == TM_PSEUDOHERMITIAN ? 5 : 9), TM_EINVAL, "bad vector count");
    TM_CHECK(h.lanes >= 1 && h.lanes <= kMaxChainLanes, TM_EINVAL, "bad lane count");
    for (int r = 0; r < h.lanes; ++r) {
        TM_CHECK(h.dir[r] >= TM_DIR_X && h.dir[r] <= TM_DIR_N, TM_EINVAL, "bad direction");
        TM_CHECK(h.lane_iq[r] >= 0 && h.lane_iq[r] < (int)s.qs.size(), TM_EINVAL,
                 "checkpoint lane q set not in this system");
    }
    TM_CHECK(h.lane_iq[0] == h.iq, TM_EINVAL, "checkpoint lane q sets inconsistent");
    TM_CHECK(h.cap >= 1 && capacity >= 0, TM_EINVAL, "bad capacity");
    TM_CHECK(h.issued >= 0 && h.issued <= h.cap, TM_EINVAL, "bad step count");
    {
        int seen = 0;
        for (int i = 0; i < h.nvec; ++i) {
            TM_CHECK(h.ix[i] >= 0 && h.ix[i] < h.nvec && !(seen >> h.ix[i] & 1), TM_EINVAL, "bad vector roles");
            seen |= 1 << h.ix[i];
        }
    }
    TM_CHECK(bytes >= blob_bytes(h.lanes, h.cap, h.nvec, h.n, ulanes_of(h.lane_iq, h.lanes)), TM_EINVAL,
             "checkpoint truncated");
    c.flavour = h.flavour;
    c.fp32 = h.fp32 != 0;
    c.lanes = h.lanes;
    std::copy(h.dir, h.dir + kMaxChainLanes, c.dir);
    std::copy(h.lane_iq, h.lane_iq + kMaxChainLanes, c.lane_iq);
    c.cap = std::max(capacity, h.cap);
    chain_qsets(c);
    QSet& qm = s.qs[c.iq];
    chain_bind_slot(c, qm);
    ensure_ground_q(s, *c.qa, st);
    if (!c.fp32) ensure_tuned(s, c.iq, st);  // the first step's projection is a tuned contraction
    chain_alloc(c);
    c.last = st;
    std::copy(h.ix, h.ix + 9, c.ix);
    c.issued = h.issued;
    chain_clear_coeffs(c, st);
    const size_t L = (size_t)c.lanes, hcap = (size_t)h.cap, ccap = (size_t)c.cap;
    const char* p = in + sizeof(h);
    std::vector<ChainState> hs(L);
    std::memcpy(hs.data(), p, L * sizeof(ChainState));
    auto get = [&](void* dev, size_t nbytes) {
        TM_HIP(hipMemcpyAsync(dev, p, nbytes, hipMemcpyHostToDevice, st));
        p += nbytes;
    };
    get(c.cs, L * sizeof(ChainState));
    // coefficient rows move to the (possibly larger) new capacity
    for (size_t r = 0; r < L; ++r) get(c.co.alpha + r * ccap, hcap * sizeof(double2));
    for (size_t r = 0; r < L; ++r) get(c.co.beta + r * ccap, hcap * sizeof(double));
    for (size_t r = 0; r < L; ++r) get(c.co.gamma + r * ccap, hcap * sizeof(double2));
    for (size_t r = 0; r < L; ++r)
        for (int l = 0; l < kNMeasure; ++l) get(c.co.z + (r * kNMeasure + l) * ccap, hcap * sizeof(double2));
    for (double2* v : c.vec) get(v, L * c.n * sizeof(double2));
    const size_t UL = c.ustride ? L : 1;
    for (int l = 0; l < kNMeasure; ++l) get(c.u[l], UL * c.n * sizeof(double2));
    // a lane saved at its capacity holds the coefficients of its next index
    // only in the state struct (alpha for pH; z for both): grown capacity gets them
    if (ccap > hcap && h.issued == h.cap) {
        for (size_t r = 0; r < L; ++r) {
            const ChainState& x = hs[r];
            if (x.step != h.cap || x.broken) continue;
            if (c.flavour == TM_PSEUDOHERMITIAN)
                TM_HIP(hipMemcpyAsync(c.co.alpha + r * ccap + hcap, &x.alpha, sizeof(double2), hipMemcpyHostToDevice,
                                      st));
            for (int l = 0; l < kNMeasure; ++l)
                TM_HIP(hipMemcpyAsync(c.co.z + (r * kNMeasure + l) * ccap + hcap, &x.znext[l], sizeof(double2),
                                      hipMemcpyHostToDevice, st));
        }
    }
    // the host blob (and hs) may be released as soon as the call returns
    TM_HIP(hipStreamSynchronize(st));
}

static int run_chain(System& s, int iq, int lanes, const int* dirs, int flavour, bool fp32, int nsteps,
                     tm_coeffs* out, hipStream_t st) {
    Chain c;
    c.s = &s;
    c.fp32 = fp32;
    c.iq = iq;
    c.lanes = lanes;
    std::copy(dirs, dirs + lanes, c.dir);
    std::fill(c.lane_iq, c.lane_iq + lanes, iq);
    c.flavour = flavour;
    c.cap = nsteps;
    chain_begin(c, st);
    while (c.issued < nsteps) {
        chain_steps(c, 66, st);
        if (c.issued < nsteps && chain_poll(c)) break;
    }
    return chain_coeffs(c, out);
}

}  // namespace tml

using namespace tml;

struct tm_system {
    System s;
};

struct tm_chain {
    Chain c;
};

template <typename F>
static int guarded(F&& f) {
    try {
        set_error("");
        return f();
    } catch (const Error& e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception& e) {
        set_error(e.what());
        return TM_EINVAL;
    }
}

extern "C" {

const char* tm_last_error(void) { return g_err.c_str(); }

int tm_profile_enable(int on) {
    return guarded([&]() -> int {
        if (!on) prof_fold();
        g_prof_on = on != 0;
        return TM_OK;
    });
}

int tm_profile_reset(void) {
    return guarded([&]() -> int {
        prof_fold();
        g_prof_agg.clear();
        return TM_OK;
    });
}

int tm_profile_count(void) {
    return guarded([&]() -> int {
        prof_fold();
        return (int)g_prof_agg.size();
    });
}

int tm_profile_get(int i, char* name, int name_cap, double* total_ms, long long* launches) {
    return guarded([&]() -> int {
        TM_CHECK(i >= 0 && i < (int)g_prof_agg.size(), TM_EINVAL, "profile index out of range");
        const ProfAgg& a = g_prof_agg[i];
        if (name && name_cap > 0) {
            std::strncpy(name, a.name.c_str(), name_cap - 1);
            name[name_cap - 1] = 0;
        }
        if (total_ms) *total_ms = a.ms;
        if (launches) *launches = a.n;
        return TM_OK;
    });
}

static bool all_finite(const double* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// every floating-point input of the description is finite (NaN or Inf -> TM_EINVAL)
static void check_finite(const tm_system_desc* d) {
    const size_t N = (size_t)d->fft[0] * d->fft[1] * d->fft[2];
    TM_CHECK(all_finite(d->cell, 9), TM_EINVAL, "non-finite cell");
    TM_CHECK(d->xk && all_finite(d->xk, 3 * (size_t)d->npts), TM_EINVAL, "non-finite point vectors");
    for (int p = 0; p < d->npts; ++p) {
        const size_t npw = (size_t)std::max(d->npw[p], 0);
        TM_CHECK(!d->evc[p] || all_finite(d->evc[p], 4 * (size_t)d->nbnd * npw), TM_EINVAL,
                 "non-finite ground-state spinors");
        TM_CHECK(!d->et[p] || all_finite(d->et[p], d->nbnd), TM_EINVAL, "non-finite eigenvalues");
        if (d->nproj > 0 && d->vkb && d->vkb[p])
            TM_CHECK(all_finite(d->vkb[p], 2 * (size_t)d->nproj * npw), TM_EINVAL, "non-finite projectors");
    }
    if (d->nproj > 0 && d->dvan)
        TM_CHECK(all_finite(d->dvan, 8 * (size_t)d->nproj * d->nproj), TM_EINVAL, "non-finite D matrix");
    if (d->vrs) TM_CHECK(all_finite(d->vrs, 4 * N), TM_EINVAL, "non-finite potential");
    if (d->rho) TM_CHECK(all_finite(d->rho, 4 * N), TM_EINVAL, "non-finite ground-state density");
    if (d->nq > 0) TM_CHECK(d->xq && all_finite(d->xq, 3 * (size_t)d->nq), TM_EINVAL, "non-finite q");
}

int tm_system_create(const tm_system_desc* d, tm_system** out) {
    return guarded([&]() -> int {
        TM_CHECK(d && out, TM_EINVAL, "null argument");
        *out = nullptr;
        // host-side validation first: it needs no device
        TM_CHECK(d->nbnd > 0 && d->npts > 0 && d->nq >= 0 && d->nk > 0, TM_EINVAL, "bad sizes");
        TM_CHECK(d->fft[0] > 0 && d->fft[1] > 0 && d->fft[2] > 0, TM_EINVAL, "bad FFT grid");
        check_grid(d->fft);
        TM_CHECK(d->nproj >= 0, TM_EINVAL, "bad nproj");
        TM_CHECK(d->npw && d->mill && d->evc && d->et, TM_EINVAL, "missing ground-state points");
        check_finite(d);
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) throw Error{TM_EDEVICE, "no HIP device"};
        std::unique_ptr<tm_system> ts(new tm_system());
        System& s = ts->s;
        TM_HIP(hipGetDevice(&s.device));
        std::memcpy(s.cell, d->cell, sizeof(s.cell));
        const double* a = d->cell;
        double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                     a[2] * (a[3] * a[7] - a[4] * a[6]);
        TM_CHECK(std::fabs(det) > 1e-12, TM_EINVAL, "singular cell");
        s.omega = std::fabs(det);
        // b_i = 2 pi (a_j x a_k) / det
        auto cross = [](const double* u, const double* v, double* w) {
            w[0] = u[1] * v[2] - u[2] * v[1];
            w[1] = u[2] * v[0] - u[0] * v[2];
            w[2] = u[0] * v[1] - u[1] * v[0];
        };
        cross(a + 3, a + 6, s.recip + 0);
        cross(a + 6, a + 0, s.recip + 3);
        cross(a + 0, a + 3, s.recip + 6);
        for (int i = 0; i < 9; ++i) s.recip[i] *= 2 * M_PI / det;
        s.n1 = d->fft[0];
        s.n2 = d->fft[1];
        s.n3 = d->fft[2];
        s.N = (long long)s.n1 * s.n2 * s.n3;
        s.nbnd = d->nbnd;
        s.nproj = d->nproj;
        const int ns[3] = {s.n1, s.n2, s.n3};
        for (int i = 0; i < 3; ++i) {
            TM_CHECK(make_radices(ns[i], s.plan[i]), TM_EUNSUPPORTED, "FFT length must factor into 2, 3, 5");
            std::vector<double2> tw(ns[i]);
            for (int j = 0; j < ns[i]; ++j) {
                double ang = -2.0 * M_PI * (double)j / (double)ns[i];
                tw[j] = cmk(std::cos(ang), std::sin(ang));
            }
            s.tw[i] = dev_upload(s, tw.data(), tw.size());
            s.plan[i].tw = s.tw[i];
            std::vector<float2> twf(ns[i]);
            for (int j = 0; j < ns[i]; ++j) twf[j] = make_float2((float)tw[j].x, (float)tw[j].y);
            s.twf[i] = dev_upload(s, twf.data(), twf.size());
            std::vector<int> pr = digit_reversal(ns[i]);
            s.perm[i] = dev_upload(s, pr.data(), pr.size());
        }
        TM_CHECK(s.n1 * s.n2 <= 4 * 1024, TM_EUNSUPPORTED, "n1*n2 above 4096 is not supported by the plane kernels");
        // ground-state points
        s.evc.resize(d->npts);
        s.npw.resize(d->npts);
        s.mill.resize(d->npts);
        s.et.resize(d->npts);
        s.h_vkb.resize(d->npts);
        for (int p = 0; p < d->npts; ++p) {
            int npw = d->npw[p];
            TM_CHECK(npw > 0 && d->mill[p] && d->evc[p] && d->et[p], TM_EINVAL, "bad ground-state point");
            TM_CHECK(npw * 2 >= d->nbnd, TM_EINVAL, "sphere smaller than the number of bands");
            s.npw[p] = npw;
            s.mill[p].assign(d->mill[p], d->mill[p] + 3 * (size_t)npw);
            s.et[p].assign(d->et[p], d->et[p] + d->nbnd);
            s.evc[p] = dev_upload(s, reinterpret_cast<const double2*>(d->evc[p]), (size_t)d->nbnd * 2 * npw);
            if (d->nproj > 0) {
                TM_CHECK(d->vkb && d->vkb[p], TM_EINVAL, "missing projector table");
                const double2* v = reinterpret_cast<const double2*>(d->vkb[p]);
                s.h_vkb[p].assign(v, v + (size_t)d->nproj * npw);
            }
        }
        if (d->nproj > 0) {
            TM_CHECK(d->dvan != nullptr, TM_EINVAL, "missing D matrix");
            s.dvan = dev_upload(s, reinterpret_cast<const double2*>(d->dvan), (size_t)d->nproj * d->nproj * 4);
        }
        // fields
        TM_CHECK(d->vrs && d->rho, TM_EINVAL, "missing fields");
        std::vector<double> tmp;
        transpose_to_planes(s, d->vrs, tmp, 4);
        s.vrs = dev_upload(s, tmp.data(), tmp.size());
        transpose_to_planes(s, d->rho, tmp, 4);
        double* rho_d = dev_upload(s, tmp.data(), tmp.size());
        s.fxc = dev_alloc<double>(s, 10 * (size_t)s.N);
        launch_fxc_setup(s, rho_d, nullptr);
        // q-sets
        s.qs.resize(d->nq);
        const int npw_pad = system_npw_pad(d);
        for (int iq = 0; iq < d->nq; ++iq) build_qset(s, d, iq, npw_pad, s.qs[iq]);
        TM_HIP(hipDeviceSynchronize());
        *out = ts.release();
        return TM_OK;
    });
}

int tm_system_destroy(tm_system* sys) {
    if (!sys) return TM_OK;
    return guarded([&]() -> int {
        System& s = sys->s;
        TM_CHECK(s.nchains == 0, TM_EINVAL, "end the system's chains before destroying it");
        (void)hipDeviceSynchronize();
        for (void* p : s.allocs) (void)hipFree(p);
        for (QSet& q : s.qs)
            if (q.ucols) (void)hipFree(q.ucols);
        if (s.cap_stream) (void)hipStreamDestroy(s.cap_stream);
        for (hipStream_t x : s.slot_stream) (void)hipStreamDestroy(x);
        for (hipEvent_t e : s.slot_event) (void)hipEventDestroy(e);
        if (s.fork_event) (void)hipEventDestroy(s.fork_event);
        if (s.ureal) (void)hipFree(s.ureal);
        if (s.wslot.empty()) s.wslot.push_back(s.ws);
        else s.wslot[s.wcur] = s.ws;
        for (Workspace& w : s.wslot) free_workspace(w);
        delete sys;
        return TM_OK;
    });
}

int tm_qset_info_get(const tm_system* sys, int iq, tm_qset_info* info) {
    return guarded([&]() -> int {
        TM_CHECK(sys && info, TM_EINVAL, "null argument");
        const System& s = sys->s;
        TM_CHECK(iq >= 0 && iq < (int)s.qs.size(), TM_EINVAL, "q-set index out of range");
        const QSet& q = s.qs[iq];
        info->nk = q.nk;
        info->nbnd = s.nbnd;
        info->npw_pad = q.npw_pad;
        info->nelem = 2LL * q.nk * s.nbnd * 2 * q.npw_pad;
        info->lam = q.lam;
        return TM_OK;
    });
}

int tm_system_set_resident_limit(tm_system* sys, long long bytes) {
    return guarded([&]() -> int {
        TM_CHECK(sys, TM_EINVAL, "null system");
        TM_CHECK(sys->s.nchains == 0, TM_EINVAL, "the residency limit cannot change while chains exist");
        reset_ground(sys->s);
        sys->s.resident_limit = bytes < 0 ? -1 : bytes;
        return TM_OK;
    });
}

int tm_system_set_chain_slots(tm_system* sys, int nslots) {
    return guarded([&]() -> int {
        TM_CHECK(sys, TM_EINVAL, "null system");
        TM_CHECK(nslots >= 1 && nslots <= 16, TM_EINVAL, "1 to 16 chain slots");
        System& s = sys->s;
        TM_CHECK(s.nchains == 0, TM_EINVAL, "the chain slots cannot change while chains exist");
        s.slot_cap = nslots;
        s.nslots = 0;  // decided again at the next chain
        s.next_slot = 0;
        return TM_OK;
    });
}

int tm_system_resident_bytes(const tm_system* sys, long long* bytes) {
    return guarded([&]() -> int {
        TM_CHECK(sys && bytes, TM_EINVAL, "null argument");
        *bytes = (long long)sys->s.ureal_bytes;
        return TM_OK;
    });
}

int tm_system_memory(const tm_system* sys, tm_memory_info* out) {
    return guarded([&]() -> int {
        TM_CHECK(sys && out, TM_EINVAL, "null argument");
        const System& s = sys->s;
        tm_memory_info m{};
        m.tables = (long long)s.table_bytes;
        m.resident = (long long)s.ureal_bytes;
        const size_t NP = (size_t)s.n1 * s.n2;
        m.resident_full = plane_fixed_supported(s.n1, s.n2)
                              ? (long long)(s.uslot_of.size() * (size_t)s.nbnd * s.n3 * 2 * NP * sizeof(double2))
                              : 0;
        for (const QSet& q : s.qs) {
            m.columns += (long long)q.ucols_bytes;
            m.columns_full = std::max(m.columns_full,
                                      (long long)((size_t)2 * q.nk * 2 * s.nbnd * s.n3 * q.ncol_u_max * sizeof(double2)));
        }
        for (int j = 0; j < (int)s.wslot.size(); ++j)
            if (j != s.wcur) m.workspace += (long long)s.wslot[j].alloc_bytes;
        m.workspace += (long long)s.ws.alloc_bytes;
        Workspace one;
        m.workspace_per_rhs = (long long)plan_workspace(s, 1, one);
        m.chain_slots = s.nslots > 0 ? s.nslots : s.slot_cap;
        *out = m;
        return TM_OK;
    });
}

// Device bytes a system will hold, from its descriptor alone (nothing is
// allocated): the workspace uses the same sizing as the real allocation; the
// tables sum their large items (bands, occupied partners, projector tables,
// sphere maps, fields) with a small allowance for the rest.
int tm_system_footprint(const tm_system_desc* d, tm_memory_info* out) {
    return guarded([&]() -> int {
        TM_CHECK(d && out, TM_EINVAL, "null argument");
        TM_CHECK(d->nbnd > 0 && d->npts > 0 && d->nq > 0 && d->nk > 0, TM_EINVAL, "empty system");
        check_grid(d->fft);
        System s;
        s.n1 = d->fft[0];
        s.n2 = d->fft[1];
        s.n3 = d->fft[2];
        s.N = (long long)s.n1 * s.n2 * s.n3;
        s.nbnd = d->nbnd;
        s.nproj = d->nproj;
        const size_t nb = (size_t)d->nbnd, NP = (size_t)s.n1 * s.n2;
        // distinct (m1, m2) columns of each point's sphere (a G shift moves them all alike)
        std::vector<int> ncol(d->npts);
        double tables = 0;
        for (int p = 0; p < d->npts; ++p) {
            std::unordered_map<long long, int> cols;
            for (int g = 0; g < d->npw[p]; ++g) cols.emplace(mkey(d->mill[p][3 * g], d->mill[p][3 * g + 1], 0), 0);
            ncol[p] = (int)cols.size();
            tables += (double)nb * 2 * d->npw[p] * sizeof(double2) + (double)d->nproj * d->npw[p] * sizeof(double2) +
                      3.0 * d->npw[p] * sizeof(int) + nb * sizeof(double);
        }
        std::set<std::array<int, 5>> uslots;
        s.qs.resize(d->nq);
        const int npw_pad = system_npw_pad(d);
        for (int iq = 0; iq < d->nq; ++iq) {
            QSet& q = s.qs[iq];
            q.nk = d->nk;
            q.ncol_max = q.ncol_u_max = 0;
            for (int ik = 0; ik < d->nk; ++ik) {
                const int* r = d->roles + ((size_t)iq * d->nk + ik) * 4;
                const int* sh = d->shifts ? d->shifts + ((size_t)iq * d->nk + ik) * 12 : nullptr;
                q.ncol_max = std::max(q.ncol_max, ncol[r[2]]);
                q.ncol_u_max = std::max({q.ncol_u_max, ncol[r[0]], ncol[r[1]]});
                for (int side = 0; side < 2; ++side) {
                    const int* gsh = sh ? sh + 3 * side : nullptr;
                    uslots.insert({r[side], gsh ? gsh[0] : 0, gsh ? gsh[1] : 0, gsh ? gsh[2] : 0, side});
                }
            }
            q.ncol_max = col_stride(q.ncol_max);
            q.npw_pad = npw_pad;
            const double P = q.npw_pad;
            // per k: occupied partners of both sides, padded projectors, maps and kinetic
            // energies, three sphere maps, the plane-position column index
            for (int ik = 0; ik < d->nk; ++ik) {
                const int* r = d->roles + ((size_t)iq * d->nk + ik) * 4;
                const double npw = d->npw[r[2]];
                // occupied partners, projector tables (the point's and the padded copy),
                // restriction maps, kinetic energies, Miller indices, eigenvalues,
                // plane-position column index, three sphere maps
                tables += 2.0 * nb * 2 * P * sizeof(double2) + (double)d->nproj * (P + npw) * sizeof(double2) +
                          (2 * P + npw) * sizeof(int) + P * sizeof(double) + 3 * npw * sizeof(int) +
                          2.0 * nb * sizeof(double) + NP * sizeof(short) +
                          2.0 * (npw + d->npw[r[0]] + d->npw[r[1]] + ncol[r[2]] + ncol[r[0]] + ncol[r[1]] + 3) *
                              sizeof(int);
            }
            tables += (double)s.N * sizeof(double);  // Coulomb multiplier
        }
        // potentials, density and magnetisation, kernel fields; twiddles and permutations
        tables += (double)s.N * (4 + 4 + 10) * sizeof(double) +
                  (double)(s.n1 + s.n2 + s.n3) * (sizeof(double2) + sizeof(float2) + sizeof(int));
        tables = tables * 1.05 + (1 << 20);
        tm_memory_info m{};
        m.tables = (long long)tables;
        m.resident_full = plane_fixed_supported(s.n1, s.n2)
                              ? (long long)(uslots.size() * nb * s.n3 * 2 * NP * sizeof(double2))
                              : 0;
        for (const QSet& q : s.qs)
            m.columns_full = std::max(m.columns_full,
                                      (long long)((size_t)2 * q.nk * 2 * nb * s.n3 * q.ncol_u_max * sizeof(double2)));
        Workspace one;
        m.workspace_per_rhs = (long long)plan_workspace(s, 1, one);
        m.chain_slots = 0;
        *out = m;
        return TM_OK;
    });
}

int tm_liouvillian_apply_multi(tm_system* sys, int iq, int nrhs, const void* xy_in, void* xy_out,
                               tm_precision prec, void* stream) {
    return guarded([&]() -> int {
        TM_CHECK(sys && xy_in && xy_out, TM_EINVAL, "null argument");
        System& s = sys->s;
        TM_CHECK(iq >= 0 && iq < (int)s.qs.size(), TM_EINVAL, "q-set index out of range");
        TM_CHECK(prec == TM_FP64 || prec == TM_FP32, TM_EINVAL, "bad precision");
        TM_CHECK(nrhs >= 1 && nrhs <= kMaxLanes, TM_EINVAL, "1 to 4 right-hand sides");
        const QSet& q = s.qs[iq];
        const size_t bytes = (size_t)nrhs * 2 * q.nk * s.nbnd * 2 * q.npw_pad * sizeof(double2);
        const char* a = static_cast<const char*>(xy_in);
        const char* b = static_cast<const char*>(xy_out);
        TM_CHECK(a + bytes <= b || b + bytes <= a, TM_EINVAL, "xy_in and xy_out overlap");
        apply_l(s, iq, static_cast<const double2*>(xy_in), static_cast<double2*>(xy_out), prec == TM_FP32,
                static_cast<hipStream_t>(stream), nrhs);
        return TM_OK;
    });
}

int tm_liouvillian_apply(tm_system* sys, int iq, const void* xy_in, void* xy_out, tm_precision prec,
                         void* stream) {
    return tm_liouvillian_apply_multi(sys, iq, 1, xy_in, xy_out, prec, stream);
}

int tm_autotune_enable(int on) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_autotune = on != 0;
    return TM_OK;
}

int tm_autotune_force(int op, int variant) {
    return guarded([&]() -> int {
        TM_CHECK(op >= 0 && op < kTuneOps, TM_EINVAL, "unknown tunable operation");
        TM_CHECK(variant >= -1, TM_EINVAL, "variant must be -1 (tuned) or an index");
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_force[op] = variant;
        return TM_OK;
    });
}

int tm_autotune_report(char* buf, size_t cap, size_t* needed) {
    return guarded([&]() -> int {
        TM_CHECK(needed != nullptr, TM_EINVAL, "null argument");
        std::string r;
        std::lock_guard<std::mutex> lock(g_tune_mu);
        for (const auto& kv : g_tuned) {
            const TuneEntry& t = kv.second;
            r += std::string(kTuneNames[t.op]) + "\t" + t.shape + "\tvariants " + std::to_string(t.nvariants) +
                 "\tchosen " + std::to_string(t.chosen) + "\tus";
            for (float u : t.us) r += " " + std::to_string(u);
            r += "\n";
        }
        *needed = r.size() + 1;
        if (buf && cap > 0) {
            const size_t n = std::min(cap - 1, r.size());
            std::memcpy(buf, r.data(), n);
            buf[n] = 0;
        }
        return TM_OK;
    });
}

int tm_liouvillian_apply_noalloc(tm_system* sys, int iq, const void* xy_in, void* xy_out, tm_precision prec,
                                 void* stream) {
    return guarded([&]() -> int {
        TM_CHECK(sys && xy_in && xy_out, TM_EINVAL, "null argument");
        System& s = sys->s;
        TM_CHECK(iq >= 0 && iq < (int)s.qs.size(), TM_EINVAL, "q-set index out of range");
        TM_CHECK(prec == TM_FP64 || prec == TM_FP32, TM_EINVAL, "bad precision");
        QSet& q = s.qs[iq];
        const size_t bytes = (size_t)2 * q.nk * s.nbnd * 2 * q.npw_pad * sizeof(double2);
        const char* a = static_cast<const char*>(xy_in);
        const char* b = static_cast<const char*>(xy_out);
        TM_CHECK(a + bytes <= b || b + bytes <= a, TM_EINVAL, "xy_in and xy_out overlap");
        int dev = -1;
        TM_HIP(hipGetDevice(&dev));
        TM_CHECK(dev == s.device, TM_EINVAL, "the current device is not the system's device");
        // the ground-state caches are built (and allocated) by an ordinary apply
        TM_CHECK(q.ground_ready && (s.ureal_mode == 1 || q.ucols), TM_EINVAL,
                 "the q set's ground-state caches are not built: call tm_liouvillian_apply once first");
        if (prec == TM_FP32)
            TM_CHECK(s.ureal_mode == 1 && zpass_fixed_supported(s.n3), TM_EUNSUPPORTED,
                     "TM_FP32 needs fixed-size plane and z kernels and the resident ground state");
        Workspace w = scratch_workspace(s, scratch_address(dev), kNoallocScratchBytes);
        w.epoch = s.ws.epoch;
        const Workspace saved = s.ws;
        s.ws = w;
        try {
            apply_l_ready(s, q, static_cast<const double2*>(xy_in), static_cast<double2*>(xy_out),
                          prec == TM_FP32, static_cast<hipStream_t>(stream), 1);
        } catch (...) {
            s.ws = saved;
            throw;
        }
        s.ws = saved;
        return TM_OK;
    });
}

int tm_start_vectors(tm_system* sys, int iq, tm_dir dir, void* u, void* v, void* stream) {
    return guarded([&]() -> int {
        TM_CHECK(sys, TM_EINVAL, "null argument");
        System& s = sys->s;
        TM_CHECK(iq >= 0 && iq < (int)s.qs.size(), TM_EINVAL, "q-set index out of range");
        TM_CHECK(dir >= TM_DIR_X && dir <= TM_DIR_N, TM_EINVAL, "bad direction");
        start_vectors(s, iq, (int)dir, static_cast<double2*>(u), static_cast<double2*>(v),
                      static_cast<hipStream_t>(stream));
        return TM_OK;
    });
}

int tm_lanczos_run(tm_system* sys, int iq, tm_dir dir, tm_flavour f, int nsteps, tm_precision prec,
                   tm_coeffs* out) {
    return guarded([&]() -> int {
        TM_CHECK(sys && out, TM_EINVAL, "null argument");
        System& s = sys->s;
        TM_CHECK(iq >= 0 && iq < (int)s.qs.size(), TM_EINVAL, "q-set index out of range");
        TM_CHECK(dir >= TM_DIR_X && dir <= TM_DIR_N, TM_EINVAL, "bad direction");
        TM_CHECK(f == TM_NONHERMITIAN || f == TM_PSEUDOHERMITIAN, TM_EINVAL, "bad flavour");
        TM_CHECK(nsteps >= 1 && nsteps <= out->capacity, TM_EINVAL, "nsteps must be in [1, capacity]");
        TM_CHECK(out->alpha && out->beta && out->gamma && out->z, TM_EINVAL, "null coefficient array");
        TM_CHECK(prec == TM_FP64 || prec == TM_FP32, TM_EINVAL, "bad precision");
        const int d = (int)dir;
        int rc = run_chain(s, iq, 1, &d, (int)f, prec == TM_FP32, nsteps, out, nullptr);
        if (rc == TM_EBREAKDOWN) set_error("Lanczos breakdown");
        return rc;
    });
}

int tm_tensor_run(tm_system* sys, int iq, int ndir, const tm_dir* dirs, tm_flavour f, int nsteps,
                  tm_precision prec, tm_coeffs* out) {
    return guarded([&]() -> int {
        TM_CHECK(sys && dirs && out, TM_EINVAL, "null argument");
        System& s = sys->s;
        TM_CHECK(iq >= 0 && iq < (int)s.qs.size(), TM_EINVAL, "q-set index out of range");
        TM_CHECK(ndir >= 1 && ndir <= kMaxLanes, TM_EINVAL, "1 to 4 directions");
        int d[kMaxLanes];
        for (int r = 0; r < ndir; ++r) {
            TM_CHECK(dirs[r] >= TM_DIR_X && dirs[r] <= TM_DIR_N, TM_EINVAL, "bad direction");
            TM_CHECK(nsteps >= 1 && nsteps <= out[r].capacity, TM_EINVAL, "nsteps must be in [1, capacity]");
            TM_CHECK(out[r].alpha && out[r].beta && out[r].gamma && out[r].z, TM_EINVAL,
                     "null coefficient array");
            d[r] = (int)dirs[r];
        }
        TM_CHECK(f == TM_NONHERMITIAN || f == TM_PSEUDOHERMITIAN, TM_EINVAL, "bad flavour");
        TM_CHECK(prec == TM_FP64 || prec == TM_FP32, TM_EINVAL, "bad precision");
        int rc = run_chain(s, iq, ndir, d, (int)f, prec == TM_FP32, nsteps, out, nullptr);
        if (rc == TM_EBREAKDOWN) set_error("Lanczos breakdown");
        return rc;
    });
}

int tm_chain_begin_lanes(tm_system* sys, int nlanes, const int* iqs, const tm_dir* dirs, tm_flavour f,
                         tm_precision prec, int capacity, void* stream, tm_chain** out) {
    return guarded([&]() -> int {
        TM_CHECK(sys && out && dirs && iqs, TM_EINVAL, "null argument");
        *out = nullptr;
        System& s = sys->s;
        TM_CHECK(nlanes >= 1 && nlanes <= kMaxChainLanes, TM_EINVAL,
                 "1 to " + std::to_string(kMaxChainLanes) + " lanes");
        for (int r = 0; r < nlanes; ++r) {
            TM_CHECK(iqs[r] >= 0 && iqs[r] < (int)s.qs.size(), TM_EINVAL, "q-set index out of range");
            TM_CHECK(dirs[r] >= TM_DIR_X && dirs[r] <= TM_DIR_N, TM_EINVAL, "bad direction");
        }
        TM_CHECK(f == TM_NONHERMITIAN || f == TM_PSEUDOHERMITIAN, TM_EINVAL, "bad flavour");
        TM_CHECK(capacity >= 1, TM_EINVAL, "capacity must be >= 1");
        TM_CHECK(prec == TM_FP64 || prec == TM_FP32, TM_EINVAL, "bad precision");
        std::unique_ptr<tm_chain> h(new tm_chain());
        Chain& c = h->c;
        c.s = &s;
        c.lanes = nlanes;
        for (int r = 0; r < nlanes; ++r) {
            c.dir[r] = (int)dirs[r];
            c.lane_iq[r] = iqs[r];
        }
        c.iq = iqs[0];
        c.flavour = (int)f;
        c.cap = capacity;
        c.fp32 = prec == TM_FP32;
        chain_begin(c, static_cast<hipStream_t>(stream));
        ++s.nchains;
        *out = h.release();
        return TM_OK;
    });
}

int tm_chain_begin_multi(tm_system* sys, int iq, int ndir, const tm_dir* dirs, tm_flavour f, tm_precision prec,
                         int capacity, void* stream, tm_chain** out) {
    if (ndir < 1 || ndir > kMaxLanes) {
        set_error("1 to 4 directions");
        return TM_EINVAL;
    }
    int iqs[kMaxLanes];
    std::fill(iqs, iqs + ndir, iq);
    return tm_chain_begin_lanes(sys, ndir, iqs, dirs, f, prec, capacity, stream, out);
}

int tm_chain_begin(tm_system* sys, int iq, tm_dir dir, tm_flavour f, tm_precision prec, int capacity, void* stream,
                   tm_chain** out) {
    return tm_chain_begin_multi(sys, iq, 1, &dir, f, prec, capacity, stream, out);
}

int tm_chain_lanes(const tm_chain* chain, int* lanes) {
    return guarded([&]() -> int {
        TM_CHECK(chain && lanes, TM_EINVAL, "null argument");
        *lanes = chain->c.lanes;
        return TM_OK;
    });
}

// Slot 0 runs on st itself; slots 1 .. nslots-1 on streams of their own,
// which wait for the work issued so far on st.
static void fork_slots(System& s, hipStream_t st) {
    if (!s.fork_event) TM_HIP(hipEventCreateWithFlags(&s.fork_event, hipEventDisableTiming));
    while ((int)s.slot_stream.size() < s.nslots - 1) {
        hipStream_t x = nullptr;
        hipEvent_t e = nullptr;
        TM_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        s.slot_stream.push_back(x);
        TM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        s.slot_event.push_back(e);
    }
    TM_HIP(hipEventRecord(s.fork_event, st));
    for (int j = 0; j + 1 < s.nslots; ++j) TM_HIP(hipStreamWaitEvent(s.slot_stream[j], s.fork_event, 0));
}

// st waits for everything issued on the slot streams
static void join_slots(System& s, hipStream_t st) {
    for (int j = 0; j + 1 < s.nslots; ++j) {
        TM_HIP(hipEventRecord(s.slot_event[j], s.slot_stream[j]));
        TM_HIP(hipStreamWaitEvent(st, s.slot_event[j], 0));
    }
}

// the stream of chain c inside tm_chains_step
static hipStream_t chain_stream(const Chain& c, hipStream_t st) {
    return c.slot == 0 || c.s->nslots <= 1 ? st : c.s->slot_stream[c.slot - 1];
}

int tm_chains_step(tm_chain* const* chains, int n, int k_steps, void* stream) {
    return guarded([&]() -> int {
        TM_CHECK(n >= 0 && k_steps >= 0, TM_EINVAL, "negative count");
        TM_CHECK(n == 0 || chains, TM_EINVAL, "null chain array");
        for (int i = 0; i < n; ++i) TM_CHECK(chains[i] != nullptr, TM_EINVAL, "null chain");
        hipStream_t st = static_cast<hipStream_t>(stream);
        // Systems with several workspace slots: each slot's chains go to the
        // slot's stream, forked from st and joined back into it, so that work
        // issued on st afterwards comes after them.
        std::vector<System*> forked;
        for (int i = 0; i < n; ++i) {
            System* s = chains[i]->c.s;
            if (s->nslots > 1 && std::find(forked.begin(), forked.end(), s) == forked.end()) forked.push_back(s);
        }
        for (System* s : forked) fork_slots(*s, st);
        try {
            // round robin, one period of steps per chain and turn
            std::vector<int> left(n, k_steps);
            for (bool any = true; any;) {
                any = false;
                for (int i = 0; i < n; ++i) {
                    Chain& c = chains[i]->c;
                    if (left[i] <= 0 || c.issued >= c.cap || c.broken_seen) continue;
                    const int before = c.issued;
                    chain_steps(c, std::min(left[i], c.period()), chain_stream(c, st));
                    left[i] -= c.issued - before;
                    any = true;
                }
            }
        } catch (...) {
            for (System* s : forked) join_slots(*s, st);
            throw;
        }
        for (System* s : forked) join_slots(*s, st);
        for (int i = 0; i < n; ++i) chains[i]->c.last = st;
        return TM_OK;
    });
}

int tm_chains_use_graphs(int on) {
    g_use_graphs = on != 0;
    return TM_OK;
}

int tm_chain_coeffs(tm_chain* chain, tm_coeffs* out) {
    return guarded([&]() -> int {
        TM_CHECK(chain && out, TM_EINVAL, "null argument");
        for (int r = 0; r < chain->c.lanes; ++r)
            TM_CHECK(out[r].capacity >= 1 && out[r].alpha && out[r].beta && out[r].gamma && out[r].z, TM_EINVAL,
                     "bad coefficient arrays");
        int rc = chain_coeffs(chain->c, out);
        if (rc == TM_EBREAKDOWN) set_error("Lanczos breakdown");
        return rc;
    });
}

int tm_chain_state_size(const tm_chain* chain, size_t* bytes) {
    return guarded([&]() -> int {
        TM_CHECK(chain && bytes, TM_EINVAL, "null argument");
        *bytes = chain_blob_bytes(chain->c);
        return TM_OK;
    });
}

int tm_chain_save(tm_chain* chain, void* host, size_t bytes) {
    return guarded([&]() -> int {
        TM_CHECK(chain && host, TM_EINVAL, "null argument");
        TM_CHECK(bytes >= chain_blob_bytes(chain->c), TM_EINVAL, "buffer smaller than tm_chain_state_size");
        chain_save(chain->c, static_cast<char*>(host));
        return TM_OK;
    });
}

int tm_chain_restore(tm_system* sys, const void* host, size_t bytes, int capacity, void* stream, tm_chain** out) {
    return guarded([&]() -> int {
        TM_CHECK(sys && host && out, TM_EINVAL, "null argument");
        *out = nullptr;
        std::unique_ptr<tm_chain> h(new tm_chain());
        h->c.s = &sys->s;
        chain_restore(h->c, static_cast<const char*>(host), bytes, capacity, static_cast<hipStream_t>(stream));
        ++sys->s.nchains;
        *out = h.release();
        return TM_OK;
    });
}

int tm_chain_end(tm_chain* chain) {
    if (!chain) return TM_OK;
    return guarded([&]() -> int {
        System* s = chain->c.s;
        delete chain;
        if (s && s->nchains > 0) --s->nchains;
        return TM_OK;
    });
}

int tm_chi(const tm_coeffs* c, int m_use, const double* omega, int nomega, double eta, double* chi) {
    return tm_chi_extrapolated(c, m_use, m_use, TM_EXTRAP_NONE, omega, nomega, eta, chi);
}

// chi rows from the measure overlaps: the three spin rows (z), or with
// `tensor` the charge row (zn) first and then the spin rows
static int chi_rows(const tm_coeffs* c, int m_use, int m_total, tm_extrap mode, const double* omega, int nomega,
                    double eta, double* chi, bool tensor) {
    return guarded([&]() -> int {
        TM_CHECK(c && omega && chi, TM_EINVAL, "null argument");
        TM_CHECK(!tensor || c->zn, TM_EINVAL, "the 4 x 4 tensor needs the charge overlaps zn");
        TM_CHECK(m_use >= 1 && m_use <= c->steps_done && m_use <= c->capacity, TM_EINVAL,
                 "m_use must be in [1, steps_done]");
        TM_CHECK(mode == TM_EXTRAP_NONE || mode == TM_EXTRAP_CONSTANT || mode == TM_EXTRAP_OSC, TM_EINVAL,
                 "bad extrapolation mode");
        TM_CHECK(mode == TM_EXTRAP_NONE ? m_total == m_use : m_total >= m_use, TM_EINVAL,
                 "m_total must equal m_use without extrapolation and be >= m_use with it");
        TM_CHECK(mode == TM_EXTRAP_NONE || m_use >= 4, TM_EINVAL, "extrapolation needs at least 4 steps");
        TM_CHECK(nomega >= 0, TM_EINVAL, "negative nomega");
        if (nomega == 0) return TM_OK;
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) throw Error{TM_EDEVICE, "no HIP device"};
        const int M0 = m_use, M = m_total, cap = c->capacity;
        const int nz = tensor ? 4 : 3;
        auto zsrc = [&](int l, int j) -> double2 {
            const double* zr = tensor ? (l == 0 ? c->zn : c->z + 2 * (size_t)(l - 1) * cap) : c->z + 2 * (size_t)l * cap;
            return cmk(zr[2 * j], zr[2 * j + 1]);
        };
        // host coefficients, extended past M0: alpha, beta, gamma by their mean over
        // the second half of the computed ones (one mean: constant; one per parity
        // of the index: osc), z = 0 beyond M0 (no measured overlaps there)
        std::vector<double2> ha(M), hg(M), hz(nz * (size_t)M, cmk(0.0, 0.0));
        std::vector<double> hb(M);
        for (int j = 0; j < M0; ++j) {
            ha[j] = cmk(c->alpha[2 * j], c->alpha[2 * j + 1]);
            hb[j] = c->beta[j];
            hg[j] = cmk(c->gamma[2 * j], c->gamma[2 * j + 1]);
            for (int l = 0; l < nz; ++l) hz[(size_t)l * M + j] = zsrc(l, j);
        }
        if (M > M0) {
            const int np = mode == TM_EXTRAP_OSC ? 2 : 1;
            double2 ma[2] = {cmk(0, 0), cmk(0, 0)}, mg[2] = {cmk(0, 0), cmk(0, 0)};
            double mb[2] = {0, 0};
            int cnt[2] = {0, 0};
            for (int j = M0 / 2; j < M0; ++j) {
                const int p = j % np;
                ma[p] = cadd(ma[p], ha[j]);
                mg[p] = cadd(mg[p], hg[j]);
                mb[p] += hb[j];
                ++cnt[p];
            }
            for (int p = 0; p < np; ++p) {
                TM_CHECK(cnt[p] > 0, TM_EINVAL, "too few steps to extrapolate");
                ma[p] = cscale(ma[p], 1.0 / cnt[p]);
                mg[p] = cscale(mg[p], 1.0 / cnt[p]);
                mb[p] /= cnt[p];
            }
            for (int j = M0; j < M; ++j) {
                const int p = j % np;
                ha[j] = ma[p];
                hb[j] = mb[p];
                hg[j] = mg[p];
            }
        }
        std::vector<void*> mem;
        struct G {
            std::vector<void*>& m;
            ~G() {
                for (void* p : m) (void)hipFree(p);
            }
        } g{mem};
        auto al = [&](size_t b) {
            void* p = nullptr;
            if (hipMalloc(&p, b) != hipSuccess) throw Error{TM_ENOMEM, "hipMalloc failed in tm_chi"};
            mem.push_back(p);
            return p;
        };
        double2* da = (double2*)al(M * sizeof(double2));
        double* db = (double*)al(M * sizeof(double));
        double2* dg = (double2*)al(M * sizeof(double2));
        double2* dz = (double2*)al(nz * (size_t)M * sizeof(double2));
        double* dw = (double*)al(nomega * sizeof(double));
        double2* work = (double2*)al(4 * (size_t)M * nomega * sizeof(double2));
        double2* dchi = (double2*)al(nz * (size_t)nomega * sizeof(double2));
        int* dst = (int*)al(sizeof(int));
        TM_HIP(hipMemcpy(da, ha.data(), M * sizeof(double2), hipMemcpyHostToDevice));
        TM_HIP(hipMemcpy(db, hb.data(), M * sizeof(double), hipMemcpyHostToDevice));
        TM_HIP(hipMemcpy(dg, hg.data(), M * sizeof(double2), hipMemcpyHostToDevice));
        TM_HIP(hipMemcpy(dz, hz.data(), nz * (size_t)M * sizeof(double2), hipMemcpyHostToDevice));
        TM_HIP(hipMemcpy(dw, omega, nomega * sizeof(double), hipMemcpyHostToDevice));
        TM_HIP(hipMemset(dst, 0, sizeof(int)));
        launch_chi(da, db, dg, dz, nz, M, M, c->n1, dw, nomega, eta, work, dchi, dst, nullptr);
        int status = 0;
        TM_HIP(hipMemcpy(&status, dst, sizeof(int), hipMemcpyDeviceToHost));
        TM_HIP(hipMemcpy(chi, dchi, nz * (size_t)nomega * sizeof(double2), hipMemcpyDeviceToHost));
        TM_CHECK(status == 0, TM_EINVAL, "singular tridiagonal system (eta = 0 on a pole?)");
        return TM_OK;
    });
}

int tm_chi_extrapolated(const tm_coeffs* c, int m_use, int m_total, tm_extrap mode, const double* omega,
                        int nomega, double eta, double* chi) {
    return chi_rows(c, m_use, m_total, mode, omega, nomega, eta, chi, false);
}

int tm_chi_tensor(const tm_coeffs* c, int m_use, int m_total, tm_extrap mode, const double* omega, int nomega,
                  double eta, double* chi) {
    return chi_rows(c, m_use, m_total, mode, omega, nomega, eta, chi, true);
}

int tm_structure_factor(const double* q, const double* chi, int nomega, double* s) {
    return guarded([&]() -> int {
        TM_CHECK(q && chi && s && nomega >= 0, TM_EINVAL, "bad argument");
        const double q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
        TM_CHECK(q2 > 0.0, TM_EINVAL, "q = 0 has no transverse projector");
        // P_ab = delta_ab - q_a q_b / q^2;  S = -Im sum_ab P_ab chi_ba
        for (int w = 0; w < nomega; ++w) {
            double acc = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    const double p = (a == b ? 1.0 : 0.0) - q[a] * q[b] / q2;
                    acc += p * chi[2 * (((size_t)b * 3 + a) * nomega + w) + 1];
                }
            s[w] = -acc;
        }
        return TM_OK;
    });
}

}  // extern "C"

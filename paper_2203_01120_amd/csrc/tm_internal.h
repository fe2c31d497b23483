// Internal declarations of libtm: device helpers, the system object and the
// kernel launchers shared between translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <memory>
#include <string>
#include <array>
#include <map>
#include <set>
#include <vector>

#include "../../include/tm.h"

namespace tml {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
struct Error {
    int code;
    std::string msg;
};
#define TM_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            throw ::tml::Error{TM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)
#define TM_CHECK(cond, code, msg)                                                 \
    do {                                                                          \
        if (!(cond)) throw ::tml::Error{(code), (msg)};                           \
    } while (0)
void check_launch(const char* what);

// Kernel timing with HIP events (enabled by tm_profile_enable); a scope
// records an event before and after the launches it encloses.
struct ProfScope {
    ProfScope(const char* name, hipStream_t st);
    ~ProfScope();
    int slot;
    hipStream_t st;
};
#define TM_LAUNCH(kern, grid, block, shm, st, ...)                          \
    do {                                                                    \
        ::tml::ProfScope ps_(#kern, (st));                                  \
        hipLaunchKernelGGL(kern, grid, block, shm, st, __VA_ARGS__);       \
        ::tml::check_launch(#kern);                                         \
    } while (0)

// ---------------------------------------------------------------- autotuning
// Launch shapes picked per problem shape by timing.  A launcher with several
// compiled variants of one operation asks tune_pick(op, key, n) which of its
// n variants to use for shape `key`: a variant forced for tests, the one
// chosen by the last timing of that shape, or 0 (the hand-picked default).
// Variants of the plane kernels and z passes do the same arithmetic in the
// same order (only the work split differs), so their results are identical;
// the contraction's variants split K differently (rounding-level differences).
enum TuneOp { kTuneDensity = 0, kTuneApply = 1, kTuneZInv = 2, kTuneZFwd = 3, kTuneGemm = 4, kTuneUpd = 5, kTuneOps = 6 };
int tune_pick(int op, long long key, int nvariants);
// size class of a right-hand side count for the launch-shape keys: 0 for 1,
// 1 for 2-3, 2 for 4-7, ...
inline int rhs_class(int nrhs) {
    int c = 0;
    while (nrhs > 1) {
        nrhs >>= 1;
        ++c;
    }
    return c;
}
inline long long tune_key(long long a, long long b = 0, long long c = 0, long long d = 0) {
    unsigned long long h = 1469598103934665603ULL;  // FNV-1a over the four values
    for (long long v : {a, b, c, d}) {
        h ^= (unsigned long long)v;
        h *= 1099511628211ULL;
    }
    return (long long)(h >> 1);
}

// ---------------------------------------------------------------- complex
__host__ __device__ inline double2 cmk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return cmk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
    return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ inline double2 cmulc(double2 a, double2 b) {
    return cmk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 cconj(double2 a) { return cmk(a.x, -a.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return cmk(a.x * s, a.y * s); }
__host__ __device__ inline double2 cmuli(double2 a) { return cmk(-a.y, a.x); }  // i*a
__host__ __device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// the same for single precision (the FP32 bulk path)
__host__ __device__ inline float2 cmkf(float r, float i) { return make_float2(r, i); }
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return cmkf(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return cmkf(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cmul(float2 a, float2 b) {
    return cmkf(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline float2 cmulc(float2 a, float2 b) {
    return cmkf(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline float2 cconj(float2 a) { return cmkf(a.x, -a.y); }
__host__ __device__ inline float2 cscale(float2 a, float s) { return cmkf(a.x * s, a.y * s); }
__host__ __device__ inline float2 cmuli(float2 a) { return cmkf(-a.y, a.x); }

// complex type traits: real type, constructor, conversions
template <class T2>
struct Cx;
template <>
struct Cx<double2> {
    using R = double;
    __host__ __device__ static double2 mk(double r, double i) { return make_double2(r, i); }
    __host__ __device__ static double2 from(double2 a) { return a; }
    __host__ __device__ static double2 from(float2 a) { return make_double2(a.x, a.y); }
};
template <>
struct Cx<float2> {
    using R = float;
    __host__ __device__ static float2 mk(float r, float i) { return make_float2(r, i); }
    __host__ __device__ static float2 from(double2 a) { return make_float2((float)a.x, (float)a.y); }
    __host__ __device__ static float2 from(float2 a) { return a; }
};

// ---------------------------------------------------------------- FFT plans
constexpr int kMaxRadices = 8;
struct FFTPlan {
    int n;
    int nrad;
    int rad[kMaxRadices];
    const double2* tw;  // device table exp(-2 pi i j / n), j < n
};
// factor n into radices 4, 5, 3, 2 (returns false if another prime divides n)
bool make_radices(int n, FFTPlan& p);

// One plane-wave sphere as seen by the FFT: its (m1, m2) columns and, per
// column, the G entries with their i3 grid index.
struct SphereMap {
    int npw = 0;
    int ncol = 0;
    int* col_ptr = nullptr;   // [ncol+1] CSR over entries sorted by column
    int* ent_g = nullptr;     // [npw] sphere index of each entry
    int* ent_i3 = nullptr;    // [npw] grid i3 of each entry
    int* col_pos = nullptr;   // [ncol] plane position i1*n2 + i2 of each column (sorted)
    std::vector<int> h_col_pos;
    int nrows = 0;            // plane rows i1 holding at least one column
    int* rows = nullptr;      // [nrows] their i1
    unsigned long long rmask = 0;  // bit i1 set for every such row (n1 <= 64)
};

// Per q-set, per mesh point k: everything the apply needs.
struct KBlock {
    double kq[3];
    int npw;                      // sphere of k+q
    SphereMap sph_kq;             // response sphere
    SphereMap sph_u[2];           // spheres of U_k (side 0) and U_-k (side 1)
    const double2* u_coef[2];     // device coefficients of U_k, U_-k [nb][2][npw_u]
    int npw_u[2];
    double* kin = nullptr;        // [npw_pad] |k+q+G|^2/2 (0 in padding)
    double* eps[2];               // [nb] e_k, e_-k (device)
    double2* occ[2];              // [nb][2][npw_pad]: U_{k+q}, T U_{-k-q} on the k+q sphere
    double2* vkb = nullptr;       // [nproj][npw_pad] projectors at k+q
    int* map_k = nullptr;         // [npw] index of G in the U_k sphere or -1
    int* map_mk = nullptr;        // [npw] index of -G in the U_-k sphere or -1
};

struct QSet {
    double xq[3];
    int nk;
    int npw_pad;                  // the system's: every q set pads its spheres to the same length
    int tmod = 0;                 // table period of the batches: 2 nk (a lane group: 2 nk times its lanes)
    const double** d_hqt = nullptr;  // Coulomb multiplier of right-hand side r: d_hqt[r % hmod]
    int hmod = 1;
    std::vector<int> members;     // a lane group: the q set of each right-hand side (empty otherwise)
    int ncol_max;                 // max columns over the k+q spheres
    int ncol_u_max;               // max columns over the u spheres
    double lam;
    std::vector<KBlock> kb;
    double* hq = nullptr;         // [N] 4 pi/|G+q|^2 / N, plane-major
    // device pointer tables (one entry per batch b = side*nk + ik)
    int** d_colptr_kq = nullptr;
    int** d_entg_kq = nullptr;
    int** d_enti3_kq = nullptr;
    int** d_colpos_kq = nullptr;
    int* d_ncol_kq = nullptr;
    int* d_npw_kq = nullptr;
    int** d_colptr_u = nullptr;
    int** d_entg_u = nullptr;
    int** d_enti3_u = nullptr;
    int** d_colpos_u = nullptr;
    int* d_ncol_u = nullptr;
    const double2** d_ucoef = nullptr;
    int* d_npw_u = nullptr;
    double** d_kin = nullptr;
    double** d_eps = nullptr;
    double2** d_occ = nullptr;
    double2** d_vkb = nullptr;
    int** d_maps = nullptr;       // restriction maps for the start vectors (map_k, map_mk)
    int* d_nrows_kq = nullptr;    // occupied plane rows of each batch's spheres
    int* d_nrows_u = nullptr;
    unsigned long long* d_rmask_kq = nullptr;
    unsigned long long* d_rmask_u = nullptr;
    int** d_rows_kq = nullptr;
    int** d_rows_u = nullptr;
    int* d_uslot = nullptr;       // [2nk] slot of each batch in the resident real-space ground state
    short** d_colidx_kq = nullptr;  // [2nk] plane position -> column of the k+q sphere, or -1
    // lazily built caches
    double2* ucols = nullptr;     // z-transformed ground-state columns [b][nb*2][n3][ncol_u_max]
    size_t ucols_bytes = 0;
    bool ground_ready = false;    // ucols or the resident real-space slots of this set are built
};

struct Workspace {
    size_t bytes = 0;             // the large buffers (decides whether chains spread over slots)
    size_t alloc_bytes = 0;       // everything the workspace holds on the device
    int epoch = 0;                // bumped whenever the buffers are reallocated
    double2* xcols = nullptr;     // [2nk][nb*2][n3][ncol_max] (also reused for phi columns)
    double2* rho_part = nullptr;  // [nslot][4][N]
    double2* rho = nullptr;       // [4][N]
    double2* work = nullptr;      // [nrhs][N] Hartree scratch
    double2* W = nullptr;         // [4][N]
    double2* fields = nullptr;    // 6 fields per point, laid out for the wave plane kernels
    double2* gpart = nullptr;     // GEMM split-K partials
    double2* gsmall = nullptr;    // reduced small GEMM outputs
    double2* dots = nullptr;      // reduced inner products [64]
    double2* dotpart = nullptr;   // per-block partial inner products
    int nchunk = 0;
    int ksplit = 0;
    int width = 0;                // right-hand sides the buffers hold
    size_t cap_xcols = 0, cap_rho_part = 0, cap_gpart = 0, cap_gsmall = 0;
};

struct System {
    int device = 0;
    double cell[9];
    double recip[9];
    double omega;
    int n1, n2, n3;
    long long N;
    int nbnd;
    int nproj;
    FFTPlan plan[3];
    double2* tw[3] = {nullptr, nullptr, nullptr};
    float2* twf[3] = {nullptr, nullptr, nullptr};  // the same twiddles in single precision
    int* perm[3] = {nullptr, nullptr, nullptr};  // digit reversal of the in-place plane transforms
    // ground-state points (device)
    std::vector<double2*> evc;    // [npts] [nb][2][npw]
    std::vector<int> npw;
    std::vector<std::vector<int>> mill;   // host copies
    std::vector<std::vector<double>> et;
    std::vector<std::vector<double2>> h_vkb;
    std::vector<double2> dvan_h;
    double2* dvan = nullptr;      // [nproj][nproj][2][2]
    double* vrs = nullptr;        // [4][N] plane-major
    double* fxc = nullptr;        // [10][N] unique kernel entries, plane-major
    std::vector<QSet> qs;
    // resident real-space ground state: one slot per distinct (point, G shift,
    // side) over all q sets, [slot][nb][n3][2][n1*n2]
    std::map<std::array<int, 5>, int> uslot_of;
    long long resident_limit = -1;  // bytes; -1 = a share of the free device memory
    int ureal_mode = 0;             // 0 undecided, 1 resident, 2 columns
    double2* ureal = nullptr;
    size_t ureal_bytes = 0;
    hipStream_t cap_stream = nullptr;  // private stream for graph capture of chain steps
    int nchains = 0;                   // chains alive (tm_chain_begin .. tm_chain_end)
    // Workspaces of the apply: one per chain slot.  Chains of a small system
    // are spread over slots whose streams run concurrently inside
    // tm_chains_step; `ws` is the selected slot's (its copy in wslot is stale
    // while selected).
    Workspace ws;
    std::vector<Workspace> wslot;
    std::vector<hipStream_t> slot_stream;
    std::vector<hipEvent_t> slot_event;
    hipEvent_t fork_event = nullptr;
    int wcur = 0;
    int nslots = 0;                    // decided at the first chain
    int slot_cap = 3;                  // at most this many (tm_system_set_chain_slots)
    int next_slot = 0;
    std::vector<void*> allocs;
    size_t table_bytes = 0;            // device bytes of everything in `allocs`
    // lane groups: the batch tables of chains whose lanes have their own q
    // sets, one per distinct list of lane q sets (kept until the system ends)
    std::map<std::vector<int>, std::unique_ptr<QSet>> groups;
    bool tuned = false;                // the autotuner has timed this system's launches
    std::set<int> tuned_rhs;           // ... and those of these classes of right-hand side counts (rhs_class)
};

template <typename T>
T* dev_alloc(System& s, size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess)
        throw Error{TM_ENOMEM, std::string("hipMalloc of ") + std::to_string(count * sizeof(T)) +
                                   " bytes failed: " + hipGetErrorString(e)};
    s.allocs.push_back(p);
    s.table_bytes += count * sizeof(T);
    return static_cast<T*>(p);
}
template <typename T>
T* dev_upload(System& s, const T* h, size_t count) {
    T* d = dev_alloc<T>(s, count);
    if (count) TM_HIP(hipMemcpy(d, h, count * sizeof(T), hipMemcpyHostToDevice));
    return d;
}

// ---------------------------------------------------------------- launchers
// nrhs: right-hand sides applied together; their BR vectors sit back to back
// (batch b of the kernels = side and k point b % 2nk of right-hand side b / 2nk)
// fft.hip
// fp32: single-precision columns (stored in the same buffer, cast to float2)
void launch_zpass_inv(const System& s, const QSet& q, bool ucols, const double2* coef, long long coef_bstride,
                      int nitems, int item_stride, double2* cols, hipStream_t st, bool fp32 = false, int nrhs = 1);
void launch_zpass_fwd(const System& s, const QSet& q, const double2* cols, const double2* xin,
                      double2* out, hipStream_t st, bool fp32 = false, int nrhs = 1);
void launch_fft3d_full(const System& s, double2* data, int sign, hipStream_t st, int nrhs = 1);
// apply.hip
void launch_density(const System& s, const QSet& q, hipStream_t st, bool fp32 = false, int nrhs = 1);
void launch_potential(const System& s, const QSet& q, hipStream_t st, int nrhs = 1);
void launch_apply_planes(const System& s, const QSet& q, hipStream_t st, bool fp32 = false, int nrhs = 1);
void launch_ureal(const System& s, const QSet& q, hipStream_t st);
void launch_fxc_setup(System& s, const double* rho_plane, hipStream_t st);
void launch_coulomb_setup(const System& s, QSet& q, hipStream_t st);
// gemm.hip
void launch_nonlocal(const System& s, const QSet& q, const double2* x, double2* out, hipStream_t st,
                     bool f32 = false, int nrhs = 1);
void launch_project(const System& s, const QSet& q, double2* out, hipStream_t st, bool f32 = false,
                    int nrhs = 1);
void launch_project_signed(const System& s, const QSet& q, double2* phi, double osx, double osy, hipStream_t st,
                           bool f32 = false, int nrhs = 1);

// api.hip
void apply_l(System& s, int iq, const double2* in, double2* out, bool fp32, hipStream_t st, int nrhs = 1);
// sizes the apply workspace for nrhs right-hand sides (grows it when needed)
void ensure_workspace(System& s, const QSet& q, int nrhs = 1);

}  // namespace tml

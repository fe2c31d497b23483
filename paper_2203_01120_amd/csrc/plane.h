// Arguments of the plane kernels (generic ones in apply.hip, fixed-size ones in plane.hip).
#pragma once

#include "tm_internal.h"

namespace tml {

// Several right-hand sides run as one batch: batch b of the grid is side and
// k point b % nb2 of right-hand side b / nb2.  Sphere tables are per b % tmod
// (tmod = nb2 when every right-hand side has the same q set; nb2 times the
// right-hand sides when each has its own); columns, densities, fields and W
// are per b (or per right-hand side).
struct PlaneArgs {
    int n1, n2, n3, NP;
    int nk, nb, nitems, bpc, nchunk;
    int cpb;            // chunks of bands per block of the wave kernels (grid.y = nchunk / cpb, rounded up)
    int nb2;            // 2 nk: batches of one right-hand side
    int tmod;           // sphere and slot tables are per b % tmod
    long long wstride;  // elements between the W (and rho) of consecutive right-hand sides (4 N)
    long long fstride;  // elements between the local field tables of consecutive right-hand sides (6 N)
    double2* xcols;
    int ncol_max;
    const double2* ucols;
    int ncol_u_max;
    const int* const* colpos_kq;
    const int* ncol_kq;
    const int* const* colpos_u;
    const int* ncol_u;
    double2* rho_part;
    const double* vrs;
    const double2* W;
    // resident real-space ground state (fixed-size kernels only; null = use
    // ucols): [slot][nb][n3][2][n1*n2], plane points column-major over the
    // digit-reversed positions of the in-place transforms, time reversal
    // applied on the y side
    double2* ureal;
    const int* uslot;  // [2nk] slot of each batch
    double2* fields;   // [n3][n1*n2][6] local fields in the order of the resident planes
    // single-precision views of xcols, rho_part and fields (FP32 bulk path)
    float2* xcols32;
    float2* rho_part32;
    float2* fields32;
};

// rows of the (i1, i2) plane occupied by each sphere, per batch b
struct PlaneTabs {
    const int* nrows_kq;
    const int* nrows_u;
    const unsigned long long* rmask_kq;
    const unsigned long long* rmask_u;
    const int* const* rows_kq;
    const int* const* rows_u;
    const double2* tw1;  // exp(-2 pi i j / n1)
    const double2* tw2;  // exp(-2 pi i j / n2)
    const int* perm1;    // mixed-radix digit reversal of the in-place transforms along i1
    const int* perm2;    // and along i2
    const short* const* colidx_kq;  // [n1*n2] column of the k+q sphere at each plane position, or -1
    const float2* tw1f;  // single-precision twiddles (FP32 bulk path)
    const float2* tw2f;
};

// position p of an in-place decimation-in-frequency transform of length n holds
// output index perm[p] (radices 4, 5, 3, 2 in that order)
std::vector<int> digit_reversal(int n);

// arguments of the fixed-size z passes (sphere <-> columns along i3)
struct ZPassArgs {
    int nb2;                           // the table period: sphere and per-batch tables are per b % nb2
                                       // (2 nk, or 2 nk times the right-hand sides when each has its own q set)
    const double2* const* coef_table;  // inverse: per-batch coefficient base, or null
    const double2* coef_base;          //          else coef_base + b * coef_bstride
    long long coef_bstride;
    long long istride;                 // complex elements between items
    const int* istride_tab;            // per-batch item stride (overrides when non-null)
    const int* const* colptr;
    const int* const* entg;
    const int* const* enti3;
    const int* ncol;
    double2* cols;                     // [b][item][n3][ncol_stride]
    float2* cols32;                    // the same in single precision (FP32 bulk path)
    int ncol_stride;
    int nitems;
    const double2* tw;                 // exp(-2 pi i j / n3)
    const float2* tw32;
    const int* perm;                   // digit reversal along i3
    // forward only
    const int* npw;
    const double* const* kin;
    const double* const* eps;
    const double2* xin;
    double2* out;
    int npw_pad;
    double inv_n;
};

bool zpass_fixed_supported(int n3);
void launch_zpass_fixed(bool inverse, const ZPassArgs& a, int ncolmax, int nbatch, int n3, hipStream_t st,
                        bool fp32 = false);

bool plane_fixed_supported(int n1, int n2);
void launch_plane_fixed(bool density, const PlaneArgs& a, const PlaneTabs& t, dim3 grid, int n1, int n2,
                        hipStream_t st, bool fp32 = false);
// fills a.ureal for the batches of the grid from a.ucols
void launch_ureal_fixed(const PlaneArgs& a, const PlaneTabs& t, dim3 grid, int n1, int n2, hipStream_t st);

}  // namespace tml

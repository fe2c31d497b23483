// Batched mixed-radix (2, 3, 4, 5) complex FFT of lines held in LDS.
//
// Stockham autosort formulation: pass with radix R over length n after a
// sub-length p (product of the earlier radices) maps, for i < n/R,
//   u_t = x[i + t n/R] * w^{t k},  k = i mod p,  w = exp(sign 2 pi i / (p R)),
//   v = DFT_R(u),   y[(i - k) R + k + s p] = v_s.
// Every thread reads all inputs of its butterflies into registers, the block
// synchronises, then writes the outputs back in place, so one LDS buffer is
// enough.  The caller guarantees nlines * n / R <= kMaxBfly * blockDim.x for
// every radix of the plan.
#pragma once

#include "tm_internal.h"

namespace tml {

constexpr int kMaxBfly = 4;

// exp(sign * 2 pi i * idx / n) from the table exp(-2 pi i j / n)
__device__ inline double2 twiddle(const double2* tw, int idx, int sign) {
    double2 w = tw[idx];
    return sign < 0 ? w : cmk(w.x, -w.y);
}

// in-register DFT of length R on v[0..R), sign = -1 forward, +1 inverse;
// T2 = double2 or float2
template <int R, class T2>
__device__ inline void dft_small(T2* v, int sign) {
    using Re = typename Cx<T2>::R;
    if constexpr (R == 2) {
        T2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (R == 3) {
        const Re c = Re(-0.5), s = Re(0.86602540378443864676) * Re(sign);
        T2 a = v[0], b = v[1], d = v[2];
        T2 t = cadd(b, d);
        T2 m = Cx<T2>::mk(a.x + c * t.x, a.y + c * t.y);
        T2 df = csub(b, d);
        T2 r = Cx<T2>::mk(-s * df.y, s * df.x);  // i s (b - d)
        v[0] = cadd(a, t);
        v[1] = cadd(m, r);
        v[2] = csub(m, r);
    } else if constexpr (R == 4) {
        T2 a = v[0], b = v[1], c = v[2], d = v[3];
        T2 t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = csub(b, d);
        // sign * i * t3
        T2 it3 = sign < 0 ? Cx<T2>::mk(t3.y, -t3.x) : Cx<T2>::mk(-t3.y, t3.x);
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, it3);
        v[3] = csub(t1, it3);
    } else if constexpr (R == 5) {
        const Re c1 = Re(0.30901699437494742410), c2 = Re(-0.80901699437494742410);
        const Re s1 = Re(0.95105651629515357212) * Re(sign), s2 = Re(0.58778525229247312917) * Re(sign);
        T2 a = v[0];
        T2 b1 = cadd(v[1], v[4]), b2 = cadd(v[2], v[3]);
        T2 d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
        T2 m1 = Cx<T2>::mk(a.x + c1 * b1.x + c2 * b2.x, a.y + c1 * b1.y + c2 * b2.y);
        T2 m2 = Cx<T2>::mk(a.x + c2 * b1.x + c1 * b2.x, a.y + c2 * b1.y + c1 * b2.y);
        // i*(s1 d1 + s2 d2) and i*(s2 d1 - s1 d2)
        T2 e1 = Cx<T2>::mk(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y);
        T2 e2 = Cx<T2>::mk(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y);
        T2 ie1 = cmuli(e1), ie2 = cmuli(e2);
        v[0] = cadd(a, cadd(b1, b2));
        v[1] = cadd(m1, ie1);
        v[4] = csub(m1, ie1);
        v[2] = cadd(m2, ie2);
        v[3] = csub(m2, ie2);
    }
}

// line l at l * lstride
struct StrideLines {
    int lstride;
    __device__ int base(int l) const { return l * lstride; }
};

// line l = (o, i), o = l / inner, at o * ostride + i * istride
struct GridLines {
    int inner, ostride, istride;
    __device__ int base(int l) const {
        const int o = l / inner;
        return o * ostride + (l - o * inner) * istride;
    }
};

// BF: butterflies a thread takes, at most (nlines * n / R <= BF * blockDim.x)
template <int R, int BF = kMaxBfly, class LN>
__device__ inline void fft_pass(double2* lds, int nlines, const LN& ln, int estride, int n, int p,
                                const double2* tw, int sign) {
    const int T = n / R;
    const int nb = nlines * T;
    const int twstep = n / (p * R);
    double2 v[BF][R];
    int pos[BF];
#pragma unroll
    for (int bi = 0; bi < BF; ++bi) {
        int b = threadIdx.x + bi * blockDim.x;
        pos[bi] = -1;
        if (b < nb) {
            int line = b / T;
            int i = b - line * T;
            int k = i % p;
            const int lb = ln.base(line);
            double2* base = lds + lb;
#pragma unroll
            for (int t = 0; t < R; ++t) {
                double2 x = base[(i + t * T) * estride];
                v[bi][t] = (t == 0 || k == 0) ? x : cmul(x, twiddle(tw, t * k * twstep, sign));
            }
            pos[bi] = lb + ((i - k) * R + k) * estride;
        }
    }
    __syncthreads();
#pragma unroll
    for (int bi = 0; bi < BF; ++bi) {
        if (pos[bi] >= 0) {
            dft_small<R>(v[bi], sign);
#pragma unroll
            for (int s = 0; s < R; ++s) lds[pos[bi] + s * p * estride] = v[bi][s];
        }
    }
    __syncthreads();
}

// Full FFT of `nlines` lines: element t of line l is lds[ln.base(l) + t*estride].
// Unnormalised; sign = -1 forward, +1 inverse.  Ends with a barrier.
// (twiddles from tw, the plan's table or a copy of it)
template <class LN>
__device__ inline void lds_fft_lines(double2* lds, int nlines, const LN& ln, int estride, const FFTPlan& pl,
                                     const double2* tw, int sign) {
    int p = 1;
    for (int r = 0; r < pl.nrad; ++r) {
        int R = pl.rad[r];
        switch (R) {
            case 4: fft_pass<4>(lds, nlines, ln, estride, pl.n, p, tw, sign); break;
            case 5: fft_pass<5>(lds, nlines, ln, estride, pl.n, p, tw, sign); break;
            case 3: fft_pass<3>(lds, nlines, ln, estride, pl.n, p, tw, sign); break;
            default: fft_pass<2>(lds, nlines, ln, estride, pl.n, p, tw, sign); break;
        }
        p *= R;
    }
}

// lines l * lstride
__device__ inline void lds_fft(double2* lds, int nlines, int lstride, int estride, const FFTPlan& pl,
                               int sign) {
    lds_fft_lines(lds, nlines, StrideLines{lstride}, estride, pl, pl.tw, sign);
}

}  // namespace tml

// Complex tall-skinny contractions on the FP64 matrix cores (gfx950
// v_mfma_f64_16x16x4f64), used by the deflation projection (Eq. (4) of
// arXiv:2502.00152: coefficients V^H b, then x0 = V c) and by the
// eigensolver's Gram-Schmidt, Rayleigh-Ritz and basis rotation blocks.
//
// Vectors are columns of length N = 3*Vh complex, stored one after another
// (column j at offset j*N complex); each complex is (re, im) doubles, so a
// column is 2N reals.
//
//   gemm_tn:  C[j][i] = sum_s conj(V[i][s]) B[j][s]          (k x n, reduction over N)
//   gemm_nn:  X[j][s] = beta X[j][s] + sum_i V[i][s] C[j][i] (N x n, k summed)
//
// Real forms.  With v = V[i][s], b = B[j][s]:
//   Re conj(v) b = vr br + vi bi,   Im conj(v) b = vr bi - vi br
// so over the interleaved reals of the columns, Re C = V~^T B~ and
// Im C = V~^T B~' where B~' is B~ with each (re, im) pair mapped to (im, -re).
// gemm_tn therefore multiplies a k x 2N real matrix by a 2N x 2n one, the 2n
// columns being the n right-hand sides read twice.  The matrix core's K
// dimension (4 per instruction) runs over the 2N reals; each lane loads 4
// consecutive reals of one column and the instruction's K slots are assigned
// so that A and B use the same permutation of the reduction index.
//
// Output layout of v_mfma_f64_16x16x4f64 (checked on gfx950): lane l,
// accumulator register r holds C[4r + l/16][l%16]; lane l supplies
// A[l%16][l/16] and B[l/16][l%16].
#include <type_traits>

#include "device_util.h"
#include "hisq_internal.h"

namespace hisq {

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef double dvec4 __attribute__((ext_vector_type(4)));

// FP32 eigenvectors on the FP32 matrix cores: -1 automatic, 0 never, 1 always
// (hisq_set_tuning "gemm_fp32_mfma").
int64_t g_gemm_f32 = -1;

// The FP32 form is chosen automatically where the FP64 one would be bound by
// the FP64 matrix rate: 4 k n flops per reduction real against 4 k + 8 n
// bytes (FP32 V, FP64 B) exceed the FP64 ridge of about 10 flop/B.
bool use_f32_mfma(int k, int n) {
    if (g_gemm_f32 >= 0) return g_gemm_f32 == 1;
    return 4.0 * k * n > 10.0 * (4.0 * k + 8.0 * n);
}

namespace {

constexpr int kBS = 256;        // 4 waves
constexpr int kStep = 16;       // reals of the reduction index per wave step

__device__ __forceinline__ dvec4 mfma(double a, double b, dvec4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Eigenvector (V) storage may be double or float; products and sums are FP64.
typedef float fvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void load4(const double *p, double (&o)[4]) {
    const dvec2 x0 = *reinterpret_cast<const dvec2 *>(p);
    const dvec2 x1 = *reinterpret_cast<const dvec2 *>(p + 2);
    o[0] = x0.x; o[1] = x0.y; o[2] = x1.x; o[3] = x1.y;
}
__device__ __forceinline__ void load4(const float *p, double (&o)[4]) {
    const fvec4 x = *reinterpret_cast<const fvec4 *>(p);
    o[0] = x.x; o[1] = x.y; o[2] = x.z; o[3] = x.w;
}
__device__ __forceinline__ dvec2 load2(const double *p) { return *reinterpret_cast<const dvec2 *>(p); }
__device__ __forceinline__ dvec2 load2(const float *p) {
    const fvec2 x = *reinterpret_cast<const fvec2 *>(p);
    return dvec2{(double)x.x, (double)x.y};
}

// ------------------------------------------------------------------- tn
// Grid: x = reduction chunks, y = 64-column tiles of V (i), z = 32-column
// tiles of the real right-hand-side columns (2n).
// partials: [gridDim.x][kpad][ncpad] doubles.
template <typename TV>
struct TnArgs {
    const TV *V;       // k columns of 2N reals
    const double *B;   // n columns of 2N reals
    double *partials;
    int64_t twoN;      // reals per column
    int k, n;
    int kpad, ncpad;   // multiples of 16
    int64_t steps;     // twoN / kStep
};

template <typename TV, int MT, int NT>
__global__ __launch_bounds__(kBS) void k_gemm_tn(TnArgs<TV> a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, q = lane >> 4;
    const int i0 = blockIdx.y * (16 * MT);
    const int j0 = blockIdx.z * (16 * NT);
    dvec4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = dvec4{0, 0, 0, 0};

    // column pointers of this lane (null when past the end: contributes 0)
    const TV *vcol[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int i = i0 + 16 * m + lr;
        vcol[m] = i < a.k ? a.V + (int64_t)i * a.twoN : nullptr;
    }
    const double *bcol[NT];
    bool imag_part[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int j = j0 + 16 * t + lr;  // real column index in [0, 2n)
        imag_part[t] = j >= a.n;
        const int jj = imag_part[t] ? j - a.n : j;
        bcol[t] = j < 2 * a.n ? a.B + (int64_t)jj * a.twoN : nullptr;
    }

    // the block owns steps [s0, s1), its waves interleave
    const int64_t per = (a.steps + gridDim.x - 1) / gridDim.x;
    const int64_t s0 = blockIdx.x * per;
    const int64_t s1 = min(a.steps, s0 + per);
    for (int64_t s = s0 + wave; s < s1; s += 4) {
        const int64_t off = s * kStep + 4 * q;
        double av[MT][4], bv[NT][4];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            if (vcol[m]) {
                load4(vcol[m] + off, av[m]);
            } else {
                av[m][0] = av[m][1] = av[m][2] = av[m][3] = 0.0;
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (bcol[t]) {
                const dvec2 y0 = *reinterpret_cast<const dvec2 *>(bcol[t] + off);
                const dvec2 y1 = *reinterpret_cast<const dvec2 *>(bcol[t] + off + 2);
                if (imag_part[t]) {
                    // (re, im) -> (im, -re)
                    bv[t][0] = y0.y; bv[t][1] = -y0.x; bv[t][2] = y1.y; bv[t][3] = -y1.x;
                } else {
                    bv[t][0] = y0.x; bv[t][1] = y0.y; bv[t][2] = y1.x; bv[t][3] = y1.y;
                }
            } else {
                bv[t][0] = bv[t][1] = bv[t][2] = bv[t][3] = 0.0;
            }
        }
        // K slot q of sub-step u <-> real index off_q + u: the same map for A and B
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[m][t] = mfma(av[m][u], bv[t][u], acc[m][t]);
    }

    // sum the four waves in a fixed order through LDS, then store the partial tile
    __shared__ double lds[4][MT * NT * 4][64];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[wave][(m * NT + t) * 4 + r][lane] = acc[m][t][r];
    __syncthreads();
    double *P = a.partials + (int64_t)blockIdx.x * a.kpad * a.ncpad;
    for (int e = threadIdx.x; e < MT * NT * 4 * 64; e += kBS) {
        const int slot = e / 64, ln = e % 64;
        const double v = ((lds[0][slot][ln] + lds[1][slot][ln]) + lds[2][slot][ln]) + lds[3][slot][ln];
        const int mt = slot / (NT * 4), t = (slot / 4) % NT, r = slot % 4;
        const int i = i0 + 16 * mt + 4 * r + (ln >> 4);
        const int j = j0 + 16 * t + (ln & 15);
        if (i < a.kpad && j < a.ncpad) P[(int64_t)i * a.ncpad + j] = v;
    }
}

// The same contraction for FP32 V on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32, B rounded to FP32 on load): each wave accumulates
// its part of the reduction index in FP32, the four waves and the blocks are
// summed in FP64.  Lane layout of this instruction (checked on gfx950): lane l
// supplies A[l%16][l/16] and B[l/16][l%16] as the FP64 form does, and
// accumulator register r holds C[4 (l/16) + r][l%16].
template <int MT, int NT>
__global__ __launch_bounds__(kBS) void k_gemm_tn_f32(TnArgs<float> a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, q = lane >> 4;
    const int i0 = blockIdx.y * (16 * MT);
    const int j0 = blockIdx.z * (16 * NT);
    fvec4 acc[MT][NT];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = fvec4{0, 0, 0, 0};
    const float *vcol[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int i = i0 + 16 * m + lr;
        vcol[m] = i < a.k ? a.V + (int64_t)i * a.twoN : nullptr;
    }
    const double *bcol[NT];
    bool imag_part[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int j = j0 + 16 * t + lr;
        imag_part[t] = j >= a.n;
        const int jj = imag_part[t] ? j - a.n : j;
        bcol[t] = j < 2 * a.n ? a.B + (int64_t)jj * a.twoN : nullptr;
    }
    const int64_t per = (a.steps + gridDim.x - 1) / gridDim.x;
    const int64_t s0 = blockIdx.x * per;
    const int64_t s1 = min(a.steps, s0 + per);
    for (int64_t s = s0 + wave; s < s1; s += 4) {
        const int64_t off = s * kStep + 4 * q;
        float av[MT][4], bv[NT][4];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            if (vcol[m]) {
                const fvec4 x = *reinterpret_cast<const fvec4 *>(vcol[m] + off);
                av[m][0] = x.x; av[m][1] = x.y; av[m][2] = x.z; av[m][3] = x.w;
            } else {
                av[m][0] = av[m][1] = av[m][2] = av[m][3] = 0.0f;
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (bcol[t]) {
                const dvec2 y0 = *reinterpret_cast<const dvec2 *>(bcol[t] + off);
                const dvec2 y1 = *reinterpret_cast<const dvec2 *>(bcol[t] + off + 2);
                if (imag_part[t]) {
                    bv[t][0] = (float)y0.y; bv[t][1] = (float)-y0.x;
                    bv[t][2] = (float)y1.y; bv[t][3] = (float)-y1.x;
                } else {
                    bv[t][0] = (float)y0.x; bv[t][1] = (float)y0.y;
                    bv[t][2] = (float)y1.x; bv[t][3] = (float)y1.y;
                }
            } else {
                bv[t][0] = bv[t][1] = bv[t][2] = bv[t][3] = 0.0f;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int m = 0; m < MT; ++m)
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[m][u], bv[t][u], acc[m][t],
                                                                     0, 0, 0);
    }
    __shared__ double lds[4][MT * NT * 4][64];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) lds[wave][(m * NT + t) * 4 + r][lane] = (double)acc[m][t][r];
    __syncthreads();
    double *P = a.partials + (int64_t)blockIdx.x * a.kpad * a.ncpad;
    for (int e = threadIdx.x; e < MT * NT * 4 * 64; e += kBS) {
        const int slot = e / 64, ln = e % 64;
        const double v = ((lds[0][slot][ln] + lds[1][slot][ln]) + lds[2][slot][ln]) + lds[3][slot][ln];
        const int mt = slot / (NT * 4), t = (slot / 4) % NT, r = slot % 4;
        const int i = i0 + 16 * mt + 4 * (ln >> 4) + r;
        const int j = j0 + 16 * t + (ln & 15);
        if (i < a.kpad && j < a.ncpad) P[(int64_t)i * a.ncpad + j] = v;
    }
}

// C[j][i] (complex, [n][k] row-major) = out_scale * row_scale_i *
// sum_b partials[b][i][j or n+j]; one wave per output entry, lanes stride the
// partials and the wave sums them in a fixed butterfly order.
__global__ __launch_bounds__(kBS) void k_tn_reduce(const double *__restrict__ partials, int nb,
                                                   int k, int n, int kpad, int ncpad,
                                                   const double *__restrict__ row_scale,
                                                   double out_scale, dvec2 *__restrict__ C) {
    const int e = blockIdx.x * (kBS / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (e >= k * n) return;
    const int j = e / k, i = e % k;
    double re = 0.0, im = 0.0;
    for (int b = lane; b < nb; b += kWave) {
        const double *P = partials + (int64_t)b * kpad * ncpad + (int64_t)i * ncpad;
        re += P[j];
        im += P[n + j];
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) {
        double s = out_scale;
        if (row_scale) s *= row_scale[i];
        C[(int64_t)j * k + i] = dvec2{re * s, im * s};
    }
}

// Matrix-vector forms for one or two right-hand sides, on the vector units:
// with so few columns the matrix-core tiles would be mostly padding.
//   gemv_tn: partial[b][i][j] = sum over the block's sites of conj(V[i][s]) B[j][s]
template <typename TV, int NB>
__global__ __launch_bounds__(kBS) void k_gemv_tn(const TV *__restrict__ V, int k,
                                                 const dvec2 *__restrict__ B, int64_t N,
                                                 double *__restrict__ partials, int ldp) {
    // block: a contiguous chunk of sites; each wave takes CU columns at a time
    // (i0 = CU * wave, CU * (wave + 4), ...), so every site iteration has CU + NB
    // independent loads in flight and the B entries are loaded once per CU columns
    constexpr int CU = 4;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t per = (N + gridDim.x - 1) / gridDim.x;
    const int64_t s0 = blockIdx.x * per, s1 = min(N, s0 + per);
    for (int i0 = wave * CU; i0 < k; i0 += (kBS / kWave) * CU) {
        const int nc = min(CU, k - i0);
        double acc[CU][NB][2];
#pragma unroll
        for (int c = 0; c < CU; ++c)
#pragma unroll
            for (int j = 0; j < NB; ++j) acc[c][j][0] = acc[c][j][1] = 0.0;
#pragma unroll 2
        for (int64_t s = s0 + lane; s < s1; s += kWave) {
            dvec2 b[NB];
#pragma unroll
            for (int j = 0; j < NB; ++j) b[j] = B[(int64_t)j * N + s];
#pragma unroll
            for (int c = 0; c < CU; ++c) {
                if (c < nc) {
                    const dvec2 a = load2(V + 2 * ((int64_t)(i0 + c) * N + s));
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        acc[c][j][0] = fma(a.x, b[j].x, fma(a.y, b[j].y, acc[c][j][0]));
                        acc[c][j][1] = fma(a.x, b[j].y, fma(-a.y, b[j].x, acc[c][j][1]));
                    }
                }
            }
        }
#pragma unroll
        for (int c = 0; c < CU; ++c) {
            if (c >= nc) break;
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const double re = wave_sum(acc[c][j][0]), im = wave_sum(acc[c][j][1]);
                if (lane == 0) {
                    double *P = partials + (int64_t)blockIdx.x * ldp + (int64_t)(i0 + c) * 2 * NB;
                    P[2 * j] = re;
                    P[2 * j + 1] = im;
                }
            }
        }
    }
}

// C[j][i] = out_scale * row_scale_i * sum_b partials[b][i][j]  (gemv layout)
__global__ __launch_bounds__(kBS) void k_gemv_reduce(const double *__restrict__ partials, int nb,
                                                     int k, int NB, int ldp,
                                                     const double *__restrict__ row_scale,
                                                     double out_scale, dvec2 *__restrict__ C) {
    const int e = blockIdx.x * (kBS / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (e >= k * NB) return;
    const int j = e / k, i = e % k;
    double re = 0.0, im = 0.0;
    for (int b = lane; b < nb; b += kWave) {
        const double *P = partials + (int64_t)b * ldp + (int64_t)i * 2 * NB + 2 * j;
        re += P[0];
        im += P[1];
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) {
        double s = out_scale;
        if (row_scale) s *= row_scale[i];
        C[(int64_t)j * k + i] = dvec2{re * s, im * s};
    }
}

//   gemv_nn: X[j][s] = beta X[j][s] + sum_i V[i][s] C[j][i], one thread per site
template <typename TV, int NB>
__global__ __launch_bounds__(kBS) void k_gemv_nn(const TV *__restrict__ V, int64_t ldv, int k,
                                                 const dvec2 *__restrict__ C, int64_t N,
                                                 double beta, dvec2 *__restrict__ X, int64_t ldx) {
    extern __shared__ dvec2 cs[];  // [NB][k]
    for (int e = threadIdx.x; e < NB * k; e += kBS) cs[e] = C[e];
    __syncthreads();
    for (int64_t s = (int64_t)blockIdx.x * kBS + threadIdx.x; s < N; s += (int64_t)gridDim.x * kBS) {
        double acc[NB][2];
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[j][0] = acc[j][1] = 0.0;
        int i = 0;
        for (; i + 4 <= k; i += 4) {
            dvec2 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = load2(V + 2 * ((int64_t)(i + u) * ldv + s));
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const dvec2 c = cs[j * k + i + u];
                    acc[j][0] = fma(v[u].x, c.x, fma(-v[u].y, c.y, acc[j][0]));
                    acc[j][1] = fma(v[u].x, c.y, fma(v[u].y, c.x, acc[j][1]));
                }
        }
        for (; i < k; ++i) {
            const dvec2 v = load2(V + 2 * ((int64_t)i * ldv + s));
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const dvec2 c = cs[j * k + i];
                acc[j][0] = fma(v.x, c.x, fma(-v.y, c.y, acc[j][0]));
                acc[j][1] = fma(v.x, c.y, fma(v.y, c.x, acc[j][1]));
            }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            dvec2 o = dvec2{acc[j][0], acc[j][1]};
            if (beta != 0.0) {
                const dvec2 x = X[(int64_t)j * ldx + s];
                o.x = fma(beta, x.x, o.x);
                o.y = fma(beta, x.y, o.y);
            }
            X[(int64_t)j * ldx + s] = o;
        }
    }
}

// ------------------------------------------------------------------- nn
// X[j][s] = beta X[j][s] + sum_i V[i][s] C[j][i], as four real products on
// the matrix cores: with A = V (rows: 16 sites, K: 4 eigenvectors) and
// B = C^T (K: the same 4 eigenvectors, columns: 16 RHS),
//   Re X += Re V Re C - Im V Im C,   Im X += Re V Im C + Im V Re C.
// Lane l supplies A[l%16][l/16] and B[l/16][l%16]: one complex V entry (site
// l%16 of the tile, eigenvector l/16 of the step) and one complex
// coefficient per lane and step, each used by two instructions; no entry is
// loaded twice.  Grid: x = 16-site tiles (grid-stride, a wave per tile),
// y = groups of 16 MT right-hand sides.  Per output, the sum over the
// eigenvectors runs in the same order for any MT and batch size.
template <typename TV>
struct NnArgs {
    const TV *V;          // k columns, column i at V + i * ldv (reals)
    const dvec2 *C;       // [n][k] complex coefficients
    double *X;            // n columns, column j at X + j * ldx (reals)
    int64_t ldv, ldx;     // reals between consecutive columns
    int k, n;
    double beta;
    int64_t rows;         // complex entries per column
    int64_t tiles;        // ceil(rows / 16)
};

__device__ __forceinline__ fvec4 mfma_any(float a, float b, fvec4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ dvec4 mfma_any(double a, double b, dvec4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// accumulator row (site of the tile) of register r for lane quarter q
template <bool F32>
__device__ __forceinline__ int acc_row(int r, int q) { return F32 ? 4 * q + r : 4 * r + q; }

// E: arithmetic (double: FP64 matrix cores; float: FP32, the coefficients
// and, for FP64 V, the vectors rounded to float)
template <typename TV, typename E, int MT>
__global__ __launch_bounds__(kBS) void k_gemm_nn(NnArgs<TV> a) {
    using Acc = typename std::conditional<std::is_same<E, float>::value, fvec4, dvec4>::type;
    constexpr bool F32 = std::is_same<E, float>::value;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int lr = lane & 15, q = lane >> 4;
    const int jbase = blockIdx.y * (16 * MT);
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < a.tiles;
         tile += (int64_t)gridDim.x * 4) {
        const int64_t site = tile * 16 + lr;  // A row of this lane
        const bool site_ok = site < a.rows;
        Acc re[MT], im[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) re[m] = im[m] = Acc{0, 0, 0, 0};
        for (int i0 = 0; i0 < a.k; i0 += 4) {
            const int i = i0 + q;  // K slot of this lane
            E vr = 0, vi = 0;
            if (site_ok && i < a.k) {
                const dvec2 v = load2(a.V + (int64_t)i * a.ldv + 2 * site);
                vr = (E)v.x;
                vi = (E)v.y;
            }
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                const int j = jbase + 16 * m + lr;  // B column of this lane
                E cr = 0, ci = 0;
                if (j < a.n && i < a.k) {
                    const dvec2 c = a.C[(int64_t)j * a.k + i];
                    cr = (E)c.x;
                    ci = (E)c.y;
                }
                re[m] = mfma_any(vr, cr, re[m]);
                re[m] = mfma_any(-vi, ci, re[m]);
                im[m] = mfma_any(vr, ci, im[m]);
                im[m] = mfma_any(vi, cr, im[m]);
            }
        }
        // register r of lane (lr, q): site tile*16 + acc_row(r, q), RHS jbase + 16m + lr
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            const int j = jbase + 16 * m + lr;
            if (j >= a.n) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t st = tile * 16 + acc_row<F32>(r, q);
                if (st >= a.rows) continue;
                dvec2 *dst = reinterpret_cast<dvec2 *>(a.X + (int64_t)j * a.ldx + 2 * st);
                dvec2 o = dvec2{(double)re[m][r], (double)im[m][r]};
                if (a.beta != 0.0) {
                    const dvec2 x = *dst;
                    o.x = fma(a.beta, x.x, o.x);
                    o.y = fma(a.beta, x.y, o.y);
                }
                *dst = o;
            }
        }
    }
}

int round16(int v) { return (v + 15) / 16 * 16; }

}  // namespace

template <typename TV, int MT, int NT>
void launch_tn(const TnArgs<TV> &a, int nbx, int mtiles, int ntiles, hipStream_t s) {
    hipLaunchKernelGGL((k_gemm_tn<TV, MT, NT>), dim3((unsigned)nbx, mtiles, ntiles), dim3(kBS), 0,
                       s, a);
}

// C = out_scale * diag(row_scale) * V^H B   (C complex [n][k] on the device)
template <typename TV>
hisq_status gemm_tn_t(hisq_gauge_s *g, const TV *V, int k, const double2 *B, int n, int64_t N,
                      const double *row_scale_dev, double out_scale, double2 *C, hipStream_t s) {
    if (n <= 2) {
        // vector-unit form: ~4 sites per lane, partials [nb][k][2 n]
        int64_t nb = (N + 4 * kBS - 1) / (4 * kBS);
        nb = std::max<int64_t>(1, std::min<int64_t>(nb, 512));
        const int ldp = 2 * n * k;
        void *p = nullptr;
        HISQ_TRY(g->ws.get("gemm_partials", sizeof(double) * nb * ldp, &p));
        double *P = static_cast<double *>(p);
        const dvec2 *Bv = reinterpret_cast<const dvec2 *>(B);
        {
            ProfileScope prof("gemm", s);
            if (n == 1)
                hipLaunchKernelGGL((k_gemv_tn<TV, 1>), dim3((unsigned)nb), dim3(kBS), 0, s, V, k, Bv,
                                   N, P, ldp);
            else
                hipLaunchKernelGGL((k_gemv_tn<TV, 2>), dim3((unsigned)nb), dim3(kBS), 0, s, V, k, Bv,
                                   N, P, ldp);
            HISQ_HIP(hipGetLastError());
        }
        const int waves = k * n;
        hipLaunchKernelGGL(k_gemv_reduce, dim3((waves + 3) / 4), dim3(kBS), 0, s, P, (int)nb, k, n,
                           ldp, row_scale_dev, out_scale, reinterpret_cast<dvec2 *>(C));
        HISQ_HIP(hipGetLastError());
        return HISQ_OK;
    }
    TnArgs<TV> a{};
    a.V = V;
    a.B = reinterpret_cast<const double *>(B);
    a.twoN = 2 * N;
    a.k = k;
    a.n = n;
    a.kpad = round16(k);
    a.ncpad = round16(2 * n);
    if (a.twoN % kStep) return fail(HISQ_ERR_INVALID_ARG, "gemm_tn: 2N must be a multiple of 16");
    a.steps = a.twoN / kStep;
    const int MT = a.kpad >= 64 ? 4 : a.kpad / 16;     // 1, 2 or 4 (kpad 48 -> 2 tiles of 2)
    const int mt = MT == 3 ? 2 : MT;
    const int NT = a.ncpad >= 32 ? 2 : 1;
    const int mtiles = (a.kpad + 16 * mt - 1) / (16 * mt), ntiles = (a.ncpad + 16 * NT - 1) / (16 * NT);
    int64_t nbx = (a.steps + 63) / 64;  // about 16 steps per wave
    nbx = std::max<int64_t>(1, std::min<int64_t>(nbx, 1024));
    void *p = nullptr;
    HISQ_TRY(g->ws.get("gemm_partials", sizeof(double) * nbx * a.kpad * a.ncpad, &p));
    a.partials = static_cast<double *>(p);
    if constexpr (std::is_same<TV, float>::value) {
        if (use_f32_mfma(k, n)) {
            ProfileScope prof("gemm", s);
            const dim3 grid((unsigned)nbx, mtiles, ntiles);
            if (mt == 4 && NT == 2) hipLaunchKernelGGL((k_gemm_tn_f32<4, 2>), grid, dim3(kBS), 0, s, a);
            else if (mt == 4) hipLaunchKernelGGL((k_gemm_tn_f32<4, 1>), grid, dim3(kBS), 0, s, a);
            else if (mt == 2 && NT == 2) hipLaunchKernelGGL((k_gemm_tn_f32<2, 2>), grid, dim3(kBS), 0, s, a);
            else if (mt == 2) hipLaunchKernelGGL((k_gemm_tn_f32<2, 1>), grid, dim3(kBS), 0, s, a);
            else if (NT == 2) hipLaunchKernelGGL((k_gemm_tn_f32<1, 2>), grid, dim3(kBS), 0, s, a);
            else hipLaunchKernelGGL((k_gemm_tn_f32<1, 1>), grid, dim3(kBS), 0, s, a);
            HISQ_HIP(hipGetLastError());
            const int waves = k * n;
            hipLaunchKernelGGL(k_tn_reduce, dim3((waves + 3) / 4), dim3(kBS), 0, s, a.partials,
                               (int)nbx, k, n, a.kpad, a.ncpad, row_scale_dev, out_scale,
                               reinterpret_cast<dvec2 *>(C));
            HISQ_HIP(hipGetLastError());
            return HISQ_OK;
        }
    }
    {
        ProfileScope prof("gemm", s);
        if (mt == 4 && NT == 2) launch_tn<TV, 4, 2>(a, (int)nbx, mtiles, ntiles, s);
        else if (mt == 4) launch_tn<TV, 4, 1>(a, (int)nbx, mtiles, ntiles, s);
        else if (mt == 2 && NT == 2) launch_tn<TV, 2, 2>(a, (int)nbx, mtiles, ntiles, s);
        else if (mt == 2) launch_tn<TV, 2, 1>(a, (int)nbx, mtiles, ntiles, s);
        else if (NT == 2) launch_tn<TV, 1, 2>(a, (int)nbx, mtiles, ntiles, s);
        else launch_tn<TV, 1, 1>(a, (int)nbx, mtiles, ntiles, s);
        HISQ_HIP(hipGetLastError());
    }
    const int waves = k * n;
    hipLaunchKernelGGL(k_tn_reduce, dim3((waves + 3) / 4), dim3(kBS), 0, s, a.partials, (int)nbx, k,
                       n, a.kpad, a.ncpad, row_scale_dev, out_scale, reinterpret_cast<dvec2 *>(C));
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

// X = beta X + V C   (C complex [n][k] on the device) over `rows` rows of
// columns ldv (V) and ldx (X) complex numbers apart
template <typename TV>
hisq_status gemm_nn_t(const TV *V, int64_t ldv, int k, const double2 *C, int n, int64_t rows,
                      double beta, double2 *X, int64_t ldx, hipStream_t s) {
    NnArgs<TV> a{};
    a.V = V;
    a.C = reinterpret_cast<const dvec2 *>(C);
    a.X = reinterpret_cast<double *>(X);
    a.ldv = 2 * ldv;
    a.ldx = 2 * ldx;
    a.k = k;
    a.n = n;
    a.beta = beta;
    a.rows = rows;
    a.tiles = (rows + 15) / 16;
    ProfileScope prof("gemm", s);
    if (n <= 2) {
        int64_t nb = (rows + 4 * kBS - 1) / (4 * kBS);
        nb = std::max<int64_t>(1, std::min<int64_t>(nb, 4096));
        const size_t lds = sizeof(dvec2) * n * k;
        if (lds > 64 * 1024) return fail(HISQ_ERR_INVALID_ARG, "gemm_nn: too many columns");
        const dvec2 *Cv = reinterpret_cast<const dvec2 *>(C);
        dvec2 *Xv = reinterpret_cast<dvec2 *>(X);
        if (n == 1)
            hipLaunchKernelGGL((k_gemv_nn<TV, 1>), dim3((unsigned)nb), dim3(kBS), lds, s, V, ldv, k,
                               Cv, rows, beta, Xv, ldx);
        else
            hipLaunchKernelGGL((k_gemv_nn<TV, 2>), dim3((unsigned)nb), dim3(kBS), lds, s, V, ldv, k,
                               Cv, rows, beta, Xv, ldx);
        HISQ_HIP(hipGetLastError());
        return HISQ_OK;
    }
    int64_t nbx = (a.tiles + 3) / 4;
    nbx = std::max<int64_t>(1, std::min<int64_t>(nbx, 2048));
    const bool f32 = std::is_same<TV, float>::value && use_f32_mfma(k, n);
    const int groups = n <= 16 ? 1 : (n + 63) / 64;
    const dim3 grid((unsigned)nbx, groups);
    if (f32) {
        if (n <= 16) hipLaunchKernelGGL((k_gemm_nn<TV, float, 1>), grid, dim3(kBS), 0, s, a);
        else hipLaunchKernelGGL((k_gemm_nn<TV, float, 4>), grid, dim3(kBS), 0, s, a);
    } else {
        if (n <= 16) hipLaunchKernelGGL((k_gemm_nn<TV, double, 1>), grid, dim3(kBS), 0, s, a);
        else hipLaunchKernelGGL((k_gemm_nn<TV, double, 4>), grid, dim3(kBS), 0, s, a);
    }
    HISQ_HIP(hipGetLastError());
    return HISQ_OK;
}

hisq_status gemm_tn(hisq_gauge_s *g, const double2 *V, int k, const double2 *B, int n,
                    int64_t N, const double *row_scale_dev, double out_scale, double2 *C,
                    hipStream_t s) {
    return gemm_tn_t<double>(g, reinterpret_cast<const double *>(V), k, B, n, N, row_scale_dev,
                             out_scale, C, s);
}
hisq_status gemm_tn(hisq_gauge_s *g, const float2 *V, int k, const double2 *B, int n,
                    int64_t N, const double *row_scale_dev, double out_scale, double2 *C,
                    hipStream_t s) {
    return gemm_tn_t<float>(g, reinterpret_cast<const float *>(V), k, B, n, N, row_scale_dev,
                            out_scale, C, s);
}
hisq_status gemm_nn(const double2 *V, int k, const double2 *C, int n, int64_t N, double beta,
                    double2 *X, hipStream_t s) {
    return gemm_nn_t<double>(reinterpret_cast<const double *>(V), N, k, C, n, N, beta, X, N, s);
}
hisq_status gemm_nn(const float2 *V, int k, const double2 *C, int n, int64_t N, double beta,
                    double2 *X, hipStream_t s) {
    return gemm_nn_t<float>(reinterpret_cast<const float *>(V), N, k, C, n, N, beta, X, N, s);
}
hisq_status gemm_nn_ld(const double2 *V, int64_t ldv, int k, const double2 *C, int n,
                       int64_t rows, double beta, double2 *X, int64_t ldx, hipStream_t s) {
    return gemm_nn_t<double>(reinterpret_cast<const double *>(V), ldv, k, C, n, rows, beta, X, ldx,
                             s);
}

}  // namespace hisq

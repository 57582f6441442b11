// mc_poisson.hpp -- HIP kernels of the cylindrical Poisson solve (gfx950).
//
// The space-charge potential solves the finite-volume cylindrical Poisson
// equation with Dirichlet ends in z and at r = R (the space-charge section):
// a sine transform (DST-I) along z per radial row diagonalises the axial
// operator, leaving one tridiagonal system in r per sine mode.
//
//   k_dst_bluestein  forward / inverse DST-I of one radial row by Bluestein's
//                    chirp z-transform: power-of-two FFTs held in LDS
//   k_dst_rows, k_idst_rows  the same transforms as direct sums (used when
//                    the FFT length does not fit in a workgroup's LDS)
//   k_pcr            per-mode tridiagonal solve in r by parallel cyclic
//                    reduction, one wavefront per mode, FP64 always
//   k_thomas_coef, k_thomas  the same solve by Thomas sweeps (one thread per
//                    mode), for grids taller than k_pcr takes
//   k_mask_*         the metal-mask Dirichlet condition by a capacitance-
//                    matrix correction (induced charges on the mask nodes)
//
// A solve takes its right-hand side either from the int64 charge grid
// (b = -rho/eps0 with rho from the control volumes) or from an FP64 array of
// b values, and either writes Phi or adds to it.
#pragma once
#include "mc_capmat.hpp"
#include "mc_device.hpp"

#include <algorithm>
#include <string>
#include <vector>

namespace mc {

static __global__ __launch_bounds__(256) void k_sine_table(double *s, int32_t nz) {
    const int32_t n2 = 2 * (nz - 1);
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n2) s[q] = sin(kPi * (double)q / (double)(nz - 1));
}

// ---------------------------------------------------------------------------
// Poisson: unknowns Phi[i][j], 0 <= i <= nr-2, 1 <= j <= nz-2 (m = nz-2).
// Right-hand side b = -rho/eps0 with rho = Q e 2^-32 / V_i over the annular
// control volume of the finite-volume operator (control_volume).  Forward
// DST-I per radial row (scaled 2/(m+1)), one
// tridiagonal system per mode (coefficients precomputed), inverse DST-I.
// Row-major work arrays bh[i][k], k contiguous.
// ---------------------------------------------------------------------------
// Annular control volume of node i (the space-charge section): the cell of
// the finite-volume radial operator, a disk of radius dr/2 on the axis and an
// annulus of width dr about r_i elsewhere, so the solve holds exactly the
// deposited charge and its Gauss flux through every cell face equals the
// charge inside.
__device__ __forceinline__ double control_volume(int32_t i, double dr, double dz) {
    return i == 0 ? kPi * (0.5 * dr) * (0.5 * dr) * dz : 2.0 * kPi * ((double)i * dr) * dr * dz;
}

template <class D>
__global__ __launch_bounds__(256) void k_dst_rows(const unsigned long long *q, const double *rhs, const double *sine,
                                                  D *bh, int32_t nr, int32_t nz, double dr, double dz) {
    extern __shared__ unsigned char smem_raw[];
    D *row = reinterpret_cast<D *>(smem_raw);
    const int32_t i = blockIdx.x, m = nz - 2, n2 = 2 * (nz - 1);
    const double vol = control_volume(i, dr, dz);
    const double scale = -kQe * 0x1p-32 / (vol * kEps0);
    for (int32_t j = threadIdx.x; j < m; j += blockDim.x) {
        const int64_t o = (int64_t)(j + 1) * nr + i;
        row[j] = (D)(q ? (double)(int64_t)q[o] * scale : rhs[o]);
    }
    __syncthreads();
    const D norm = (D)(2.0 / (double)(nz - 1));
    for (int32_t k = 1 + threadIdx.x; k <= m; k += blockDim.x) {
        D acc = 0;
        int32_t idx = 0;
        for (int32_t j = 1; j <= m; ++j) {
            idx += k;
            if (idx >= n2) idx -= n2;
            acc += row[j - 1] * (D)sine[idx];
        }
        bh[(int64_t)i * m + (k - 1)] = acc * norm;
    }
}

// Tridiagonal coefficients per (row i, mode k): cp = up / den, inv = 1 / den,
// den_i = diag_i(k) - lo_i cp_{i-1}; diag = -(lo + up) + lambda_k,
// lambda_k = -(4/dz^2) sin^2(pi k / (2 (nz-1))).
static __global__ __launch_bounds__(256) void k_thomas_coef(double *cp, double *inv, int32_t nr, int32_t nz, double dr,
                                                     double dz) {
    const int32_t m = nz - 2, nu = nr - 1;
    const int32_t k = 1 + blockIdx.x * blockDim.x + threadIdx.x;
    if (k > m) return;
    const double sk = sin(kPi * (double)k / (2.0 * (double)(nz - 1)));
    const double lam = -(4.0 / (dz * dz)) * sk * sk;
    double cprev = 0.0;
    for (int32_t i = 0; i < nu; ++i) {
        double lo, up, di;
        if (i == 0) {
            lo = 0.0;
            di = -4.0 / (dr * dr) + lam;
            up = 4.0 / (dr * dr);
        } else {
            const double ri = (double)i * dr;
            lo = (ri - 0.5 * dr) / (ri * dr * dr);
            up = (ri + 0.5 * dr) / (ri * dr * dr);
            di = -(lo + up) + lam;
        }
        const double den = (i == 0) ? di : di - lo * cprev;
        cprev = up / den;
        cp[(int64_t)i * m + (k - 1)] = cprev;
        inv[(int64_t)i * m + (k - 1)] = 1.0 / den;
    }
}

// One tridiagonal system per mode k (one thread each, coalesced across k).
// The sweeps are a chain of dependent updates, so each group of kThomasGroup
// rows has all of its loads issued before its updates: one memory latency per
// group instead of one per row.
constexpr int kThomasGroup = 16;

// Lower diagonal of the radial operator in row i >= 1.
__device__ __forceinline__ double thomas_lower(int32_t i, double dr) {
    const double ri = (double)i * dr;
    return (ri - 0.5 * dr) / (ri * dr * dr);
}

template <class D>
__global__ __launch_bounds__(256) void k_thomas(D *bh, const double *cp, const double *inv, int32_t nr, int32_t nz,
                                                double dr) {
    constexpr int U = kThomasGroup;
    const int32_t m = nz - 2, nu = nr - 1;
    const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    // forward sweep in FP64: whole groups (loads first), then the remaining rows
    double dprev = 0.0;
    int32_t i = 0;
    for (; i + U <= nu; i += U) {
        double b[U], v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t o = (int64_t)(i + u) * m + k;
            b[u] = (double)bh[o];
            v[u] = inv[o];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double lo = (i + u > 0) ? thomas_lower(i + u, dr) : 0.0;
            dprev = (b[u] - lo * dprev) * v[u];
            bh[(int64_t)(i + u) * m + k] = (D)dprev;
        }
    }
    for (; i < nu; ++i) {
        const int64_t o = (int64_t)i * m + k;
        const double lo = (i > 0) ? thomas_lower(i, dr) : 0.0;
        dprev = ((double)bh[o] - lo * dprev) * inv[o];
        bh[o] = (D)dprev;
    }
    // back substitution: the last row, then whole groups downwards, then the rest
    double x = (double)bh[(int64_t)(nu - 1) * m + k];
    i = nu - 2;
    for (; i - U + 1 >= 0; i -= U) {
        double b[U], c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t o = (int64_t)(i - u) * m + k;
            b[u] = (double)bh[o];
            c[u] = cp[o];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            x = b[u] - c[u] * x;
            bh[(int64_t)(i - u) * m + k] = (D)x;
        }
    }
    for (; i >= 0; --i) {
        const int64_t o = (int64_t)i * m + k;
        x = (double)bh[o] - cp[o] * x;
        bh[o] = (D)x;
    }
}

// The same systems by parallel cyclic reduction: one wavefront per mode k,
// its nu = nr - 1 rows padded with identity rows to 64 R (R rows per lane,
// held in LDS), W wavefronts (modes) per block.  Step h = 1, 2, 4, ...
// eliminates every row's couplings to the rows h away:
//   alpha = -a_i / b_{i-h},  gamma = -c_i / b_{i+h},
//   a_i <- alpha a_{i-h},  c_i <- gamma c_{i+h},
//   b_i <- b_i + alpha c_{i-h} + gamma a_{i+h},  d_i <- d_i + alpha d_{i-h} + gamma d_{i+h},
// rows outside [0, 64 R) taken as identity rows; after log2(64 R) steps
// x_i = d_i / b_i.  FP64 throughout; each step reads one LDS copy of the
// rows and writes the other.  The rows are those of k_thomas_coef
// (lower lo_i, upper up_i, diagonal -(lo_i + up_i) + lambda_k; the axis row
// -4/dr^2 + lambda_k, 4/dr^2; x = 0 beyond the last row): strictly
// diagonally dominant since lambda_k < 0, where cyclic reduction is stable.
// 1022 modes of 255 rows are 1022 wavefronts across the chip instead of
// 1022 threads stepping through 255 dependent rows.
template <class D, int R, int W>
__global__ __launch_bounds__(64 * W) void k_pcr(D *bh, int32_t nr, int32_t nz, double dr, double dz) {
    constexpr int N = 64 * R;
    // two copies of (a, b, c, d): each step reads one and writes the other
    __shared__ double s_abcd[2][4][W][N];
    const int32_t m = nz - 2, nu = nr - 1;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t k = blockIdx.x * W + w + 1;  // mode 1..m (uniform per wavefront)
    const bool live = k <= m;
    double lam = 0.0;
    if (live) {
        const double sk = sin(kPi * (double)k / (2.0 * (double)(nz - 1)));
        lam = -(4.0 / (dz * dz)) * sk * sk;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int32_t i = lane + 64 * q;
        double a = 0.0, b = 1.0, c = 0.0, d = 0.0;
        if (live && i < nu) {
            if (i == 0) {
                b = -4.0 / (dr * dr) + lam;
                c = 4.0 / (dr * dr);
            } else {
                const double ri = (double)i * dr;
                a = (ri - 0.5 * dr) / (ri * dr * dr);
                c = (ri + 0.5 * dr) / (ri * dr * dr);
                b = -(a + c) + lam;
            }
            if (i == nu - 1) c = 0.0;  // Phi = 0 at r = R
            d = (double)bh[(int64_t)i * m + (k - 1)];
        }
        s_abcd[0][0][w][i] = a;
        s_abcd[0][1][w][i] = b;
        s_abcd[0][2][w][i] = c;
        s_abcd[0][3][w][i] = d;
    }
    __syncthreads();
    int src = 0;
    for (int h = 1; h < N; h <<= 1) {
        const double *A = s_abcd[src][0][w], *B = s_abcd[src][1][w], *C = s_abcd[src][2][w], *Dv = s_abcd[src][3][w];
        double *A2 = s_abcd[1 - src][0][w], *B2 = s_abcd[1 - src][1][w], *C2 = s_abcd[1 - src][2][w],
               *D2 = s_abcd[1 - src][3][w];
#pragma unroll 4
        for (int q = 0; q < R; ++q) {
            const int32_t i = lane + 64 * q, l = i - h, u = i + h;
            const double al = l >= 0 ? A[l] : 0.0, bl = l >= 0 ? B[l] : 1.0, cl = l >= 0 ? C[l] : 0.0,
                         dl = l >= 0 ? Dv[l] : 0.0;
            const double au = u < N ? A[u] : 0.0, bu = u < N ? B[u] : 1.0, cu = u < N ? C[u] : 0.0,
                         du = u < N ? Dv[u] : 0.0;
            const double alpha = -A[i] / bl, gamma = -C[i] / bu;
            A2[i] = alpha * al;
            C2[i] = gamma * cu;
            B2[i] = B[i] + alpha * cl + gamma * au;
            D2[i] = Dv[i] + alpha * dl + gamma * du;
        }
        __syncthreads();
        src = 1 - src;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int32_t i = lane + 64 * q;
        if (live && i < nu) bh[(int64_t)i * m + (k - 1)] = (D)(s_abcd[src][3][w][i] / s_abcd[src][1][w][i]);
    }
}

template <class D>
__global__ __launch_bounds__(256) void k_idst_rows(const D *ph, const double *sine, double *phi, int32_t nr,
                                                   int32_t nz, int32_t accumulate) {
    extern __shared__ unsigned char smem_raw[];
    D *row = reinterpret_cast<D *>(smem_raw);
    const int32_t i = blockIdx.x, m = nz - 2, n2 = 2 * (nz - 1);
    for (int32_t k = threadIdx.x; k < m; k += blockDim.x) row[k] = ph[(int64_t)i * m + k];
    __syncthreads();
    for (int32_t j = 1 + threadIdx.x; j <= m; j += blockDim.x) {
        D acc = 0;
        int32_t idx = 0;
        for (int32_t k = 1; k <= m; ++k) {
            idx += j;
            if (idx >= n2) idx -= n2;
            acc += row[k - 1] * (D)sine[idx];
        }
        const int64_t o = (int64_t)j * nr + i;
        phi[o] = accumulate ? phi[o] + (double)acc : (double)acc;
    }
}

// ---------------------------------------------------------------------------
// Sine transform by Bluestein's chirp z-transform (O(L log L) per row).
// With kj = (k^2 + j^2 - (k-j)^2)/2,
//   X_k = sum_j x_j sin(pi k j / N) = Im[ c_k sum_j (x_j c_j) b_{k-j} ],
//   c_j = exp(i pi j^2 / 2N),  b_d = exp(-i pi d^2 / 2N),
// a linear convolution of length m evaluated with power-of-two FFTs of
// length L >= 2m - 1 held in LDS.  The forward FFT is decimation in
// frequency (natural order in, bit-reversed out), the filter spectrum FFT(b)
// is stored bit-reversed, and the inverse is decimation in time
// (bit-reversed in, natural out), so no permutation pass is needed.
// Phases use j^2 mod 4N in integers, so large j lose no accuracy.
// ---------------------------------------------------------------------------
template <class D>
struct Cx {
    D re, im;
};

template <class D>
__device__ __forceinline__ Cx<D> cmul(Cx<D> a, Cx<D> b) {
    return Cx<D>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// LDS slot of complex value i: one spare slot after every 8 values, so that
// the passes which give a thread 8 consecutive values (stride 8 across the
// wavefront) spread their accesses over the banks.
__device__ __forceinline__ int32_t cslot(int32_t i) { return i + (i >> 3); }

// The FFTs are in-place radix-2 transforms (forward: decimation in frequency,
// twiddles exp(-2 pi i k / L), natural order in, bit-reversed out; inverse:
// decimation in time with conjugate twiddles, bit-reversed in, natural out,
// unscaled) whose consecutive stages are taken G at a time: a thread loads
// the 2^G values that those stages combine, applies the G stages in
// registers, and stores them back, so a transform of L = 2^S values takes
// about S/3 passes (and barriers) instead of S.  The arithmetic of each
// butterfly is that of the radix-2 stage it belongs to.
//
// Forward stages of lengths len, len/2, ..., len/2^(G-1): a group holds
// the values B + o + j sub (j < 2^G, sub = len / 2^G, o < sub) of one block
// of len values.
template <class D, int G>
__device__ __forceinline__ void dif_stages(Cx<D> (&v)[1 << G], int32_t o, int32_t sub, int32_t len, int32_t L,
                                           const Cx<D> *tw) {
#pragma unroll
    for (int t = 0; t < G; ++t) {
        const int h = 1 << (G - 1 - t);  // partner distance within the group
        const int32_t stride = L / (len >> t);
#pragma unroll
        for (int j = 0; j < (1 << G); ++j) {
            if (j & h) continue;
            const Cx<D> u = v[j], w = v[j + h];
            v[j] = Cx<D>{u.re + w.re, u.im + w.im};
            v[j + h] = cmul(Cx<D>{u.re - w.re, u.im - w.im}, tw[(o + (j & (h - 1)) * sub) * stride]);
        }
    }
}

// Inverse stages of lengths ls, 2 ls, ..., 2^(G-1) ls: a group holds the
// values B + o + j hs (j < 2^G, hs = ls / 2, o < hs) of one block of
// 2^(G-1) ls values.
template <class D, int G>
__device__ __forceinline__ void dit_stages(Cx<D> (&v)[1 << G], int32_t o, int32_t hs, int32_t ls, int32_t L,
                                           const Cx<D> *tw) {
#pragma unroll
    for (int t = 0; t < G; ++t) {
        const int h = 1 << t;
        const int32_t stride = L / (ls << t);
#pragma unroll
        for (int j = 0; j < (1 << G); ++j) {
            if (j & h) continue;
            const Cx<D> w = tw[(o + (j & (h - 1)) * hs) * stride];
            const Cx<D> tt = cmul(v[j + h], Cx<D>{w.re, -w.im});
            const Cx<D> u = v[j];
            v[j] = Cx<D>{u.re + tt.re, u.im + tt.im};
            v[j + h] = Cx<D>{u.re - tt.re, u.im - tt.im};
        }
    }
}

// One pass of G forward stages starting at block length len, every group
// of the transform, then a barrier.
template <class D, int G>
__device__ __forceinline__ void dif_pass(Cx<D> *a, int32_t len, int32_t L, const Cx<D> *tw) {
    const int32_t sub = len >> G;
    for (int32_t gi = threadIdx.x; gi < (L >> G); gi += blockDim.x) {
        const int32_t o = gi & (sub - 1), base = (gi - o) << G | o;  // (gi / sub) len + o
        Cx<D> v[1 << G];
#pragma unroll
        for (int j = 0; j < (1 << G); ++j) v[j] = a[cslot(base + j * sub)];
        dif_stages<D, G>(v, o, sub, len, L, tw);
#pragma unroll
        for (int j = 0; j < (1 << G); ++j) a[cslot(base + j * sub)] = v[j];
    }
    __syncthreads();
}

template <class D, int G>
__device__ __forceinline__ void dit_pass(Cx<D> *a, int32_t ls, int32_t L, const Cx<D> *tw) {
    const int32_t hs = ls >> 1;
    for (int32_t gi = threadIdx.x; gi < (L >> G); gi += blockDim.x) {
        const int32_t o = gi & (hs - 1), base = (gi - o) << G | o;  // (gi / hs) 2^(G-1) ls + o
        Cx<D> v[1 << G];
#pragma unroll
        for (int j = 0; j < (1 << G); ++j) v[j] = a[cslot(base + j * hs)];
        dit_stages<D, G>(v, o, hs, ls, L, tw);
#pragma unroll
        for (int j = 0; j < (1 << G); ++j) a[cslot(base + j * hs)] = v[j];
    }
    __syncthreads();
}

// Forward stages of lengths L down to 16 (all but the last three), values
// in LDS slots cslot(i); L = 2^S with S >= 6.  The first pass takes the
// S mod 3 stages that do not make a full group of three.
template <class D>
__device__ __forceinline__ void fft_forward_head(Cx<D> *a, int32_t L, int32_t S, const Cx<D> *tw) {
    int32_t len = L;
    const int32_t r = S % 3;
    if (r == 1) {
        dif_pass<D, 1>(a, len, L, tw);
        len >>= 1;
    } else if (r == 2) {
        dif_pass<D, 2>(a, len, L, tw);
        len >>= 2;
    }
    for (; len > 8; len >>= 3) dif_pass<D, 3>(a, len, L, tw);
}

// Inverse stages of lengths 16 up to L (all but the first three).
template <class D>
__device__ __forceinline__ void fft_inverse_tail(Cx<D> *a, int32_t L, int32_t S, const Cx<D> *tw) {
    int32_t ls = 16;
    for (int32_t p = 0; p < (S - 3) / 3; ++p, ls <<= 3) dit_pass<D, 3>(a, ls, L, tw);
    const int32_t r = S % 3;
    if (r == 1) dit_pass<D, 1>(a, ls, L, tw);
    else if (r == 2) dit_pass<D, 2>(a, ls, L, tw);
}

// Tables for one grid: chirp[n] = c_{n+1} (n < m), tw[k] = exp(-2 pi i k/L)
// (k < L/2), and fb = FFT(b) in bit-reversed order (built by k_bluestein_filter).
template <class D>
__global__ __launch_bounds__(256) void k_bluestein_tables(Cx<D> *chirp, Cx<D> *tw, int32_t m, int32_t L) {
    const int32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t fourN = 4 * (int64_t)(m + 1);
    if (n < m) {
        const int64_t j = n + 1, q = (j * j) % fourN;
        double sv, cv;
        sincospi((double)q / (double)(2 * (m + 1)), &sv, &cv);
        chirp[n] = Cx<D>{(D)cv, (D)sv};
    }
    if (n < (L >> 1)) {
        double sv, cv;
        sincospi(-2.0 * (double)n / (double)L, &sv, &cv);
        tw[n] = Cx<D>{(D)cv, (D)sv};
    }
}

template <class D>
__global__ __launch_bounds__(1024) void k_bluestein_filter(Cx<D> *fb, const Cx<D> *tw, int32_t m, int32_t L) {
    extern __shared__ unsigned char smem_raw[];
    Cx<D> *a = reinterpret_cast<Cx<D> *>(smem_raw);
    const int64_t fourN = 4 * (int64_t)(m + 1);
    for (int32_t n = threadIdx.x; n < L; n += blockDim.x) {
        int64_t d = -1;
        if (n < m) d = n;
        else if (n > L - m) d = L - n;  // b_{-d} = b_d
        Cx<D> v{(D)0, (D)0};
        if (d >= 0) {
            const int64_t q = (d * d) % fourN;
            double sv, cv;
            sincospi((double)q / (double)(2 * (m + 1)), &sv, &cv);
            v = Cx<D>{(D)cv, (D)(-sv)};
        }
        a[cslot(n)] = v;
    }
    __syncthreads();
    const int32_t S = __builtin_ctz((uint32_t)L);
    fft_forward_head<D>(a, L, S, tw);
    dif_pass<D, 3>(a, 8, L, tw);
    for (int32_t n = threadIdx.x; n < L; n += blockDim.x) fb[n] = a[cslot(n)];
}

// One radial row per block of dst_threads(L) threads (one group of 8 values
// per thread and pass, 64 to 1024 threads: long rows, whose LDS allows one
// block per CU, get the most).  kForward: input -rho/eps0 of column i from
// the int64 charge grid, output bh[i][:] scaled by 2/N.  Inverse: input
// bh[i][:], output Phi[1..m][i].
inline int dst_threads(int32_t L) { return std::min(1024, std::max(64, L / 8)); }

template <class D, bool kForward>
__global__ __launch_bounds__(1024) void k_dst_bluestein(const unsigned long long *q, const double *rhs, D *bh,
                                                               double *phi, int32_t accumulate, const Cx<D> *chirp,
                                                               const Cx<D> *fb, const Cx<D> *tw, int32_t nr,
                                                               int32_t nz, int32_t L, double dr, double dz) {
    extern __shared__ unsigned char smem_raw[];
    Cx<D> *a = reinterpret_cast<Cx<D> *>(smem_raw);
    const int32_t i = blockIdx.x, m = nz - 2, S = __builtin_ctz((uint32_t)L);
    const double vol = control_volume(i, dr, dz);
    const double scale = -kQe * 0x1p-32 / (vol * kEps0);
#pragma unroll 4
    for (int32_t n = threadIdx.x; n < L; n += blockDim.x) {
        Cx<D> v{(D)0, (D)0};
        if (n < m) {
            const int64_t o = (int64_t)(n + 1) * nr + i;
            const D x = kForward ? (D)(q ? (double)(int64_t)q[o] * scale : rhs[o]) : bh[(int64_t)i * m + n];
            const Cx<D> c = chirp[n];
            v = Cx<D>{x * c.re, x * c.im};
        }
        a[cslot(n)] = v;
    }
    __syncthreads();
    fft_forward_head<D>(a, L, S, tw);
    // the last three forward stages, the product with the filter spectrum
    // (both in bit-reversed order) and the first three inverse stages all act
    // on the same 8 consecutive values: one pass
    for (int32_t gi = threadIdx.x; gi < (L >> 3); gi += blockDim.x) {
        const int32_t base = gi << 3;
        Cx<D> v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = a[cslot(base + j)];
        dif_stages<D, 3>(v, 0, 1, 8, L, tw);
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = cmul(v[j], fb[base + j]);
        dit_stages<D, 3>(v, 0, 1, 2, L, tw);
#pragma unroll
        for (int j = 0; j < 8; ++j) a[cslot(base + j)] = v[j];
    }
    __syncthreads();
    fft_inverse_tail<D>(a, L, S, tw);
    // the inverse transform's 1/L folded into the output scale (a power of two)
    const D norm = (D)((kForward ? 2.0 / (double)(nz - 1) : 1.0) / (double)L);
#pragma unroll 4
    for (int32_t k = threadIdx.x; k < m; k += blockDim.x) {
        const Cx<D> c = chirp[k], y = a[cslot(k)];
        const D X = (c.re * y.im + c.im * y.re) * norm;  // Im(c y)
        if (kForward) bh[(int64_t)i * m + k] = X;
        else {
            const int64_t o = (int64_t)(k + 1) * nr + i;
            phi[o] = accumulate ? phi[o] + (double)X : (double)X;
        }
    }
}

// Host side of the chirp z sine transform: one set of tables per grid.
struct Bluestein {
    int32_t L = 0;      // 0: not used (FFT length would not fit in LDS)
    size_t lds = 0;     // bytes of LDS per row block
    void *chirp = nullptr, *tw = nullptr, *fb = nullptr;
};

constexpr size_t kLdsLimit = 160 * 1024;  // LDS per workgroup on gfx950

// Modes from which systems of more than 256 rows take Thomas sweeps: on the
// 1024 x 8192 grid (8190 modes of 1023 rows) the sweeps took 0.21 ms and
// cyclic reduction 0.80 ms; on the 256 x 1024 grid (1022 modes of 255 rows)
// the sweeps took 0.056 ms and cyclic reduction 0.015 ms.
constexpr int32_t kPcrMaxModes = 4096;

// LDS a workgroup may take on the current device (the smaller of the
// architectural limit and what the runtime reports).
inline size_t lds_per_block() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        return 65536;
    return std::min(kLdsLimit, (size_t)v);
}

// FFT length: the smallest power of two >= 2m - 1, at least 16 (the passes
// take the last three forward and first three inverse stages together).
inline int32_t bluestein_length(int32_t m) {
    int32_t L = 16;
    while (L < 2 * m - 1) L <<= 1;
    return L;
}

// LDS bytes of one row's transform: L complex values of cx bytes and one
// spare slot per 8 (cslot).
inline size_t bluestein_lds(int32_t L, size_t cx) { return ((size_t)L + (size_t)(L >> 3)) * cx; }

template <class D>
inline hipError_t bluestein_prepare(Bluestein &B, int32_t m, hipStream_t st) {
    const int32_t n = std::max(m, B.L >> 1);
    k_bluestein_tables<D><<<(n + 255) / 256, 256, 0, st>>>((Cx<D> *)B.chirp, (Cx<D> *)B.tw, m, B.L);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (B.lds > 65536) {
        e = hipFuncSetAttribute((const void *)&k_bluestein_filter<D>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)B.lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)&k_dst_bluestein<D, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)B.lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void *)&k_dst_bluestein<D, false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)B.lds);
        if (e != hipSuccess) return e;
    }
    k_bluestein_filter<D><<<1, 1024, B.lds, st>>>((Cx<D> *)B.fb, (const Cx<D> *)B.tw, m, B.L);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One Poisson solve (host side): forward transform of the right-hand side
// (int64 charge grid q, or FP64 b values rhs when q is null), one
// tridiagonal system per mode, inverse transform into phi (or added to phi).
// ---------------------------------------------------------------------------
struct PoissonGrid {
    int32_t nr = 0, nz = 0;
    double dr = 0, dz = 0;
    const double *sine = nullptr, *tcp = nullptr, *tinv = nullptr;
    const Bluestein *blu = nullptr;
};

template <class D>
inline hipError_t poisson_solve(const PoissonGrid &g, const unsigned long long *q, const double *rhs, D *bh,
                                double *phi, bool accumulate, hipStream_t st) {
    const int32_t m = g.nz - 2, nu = g.nr - 1;
    const Bluestein &B = *g.blu;
    const Cx<D> *chirp = (const Cx<D> *)B.chirp, *fb = (const Cx<D> *)B.fb, *tw = (const Cx<D> *)B.tw;
    if (B.L > 0)
        k_dst_bluestein<D, true><<<nu, dst_threads(B.L), B.lds, st>>>(q, rhs, bh, nullptr, 0, chirp, fb, tw, g.nr, g.nz, B.L,
                                                           g.dr, g.dz);
    else
        k_dst_rows<D><<<nu, 256, m * sizeof(D), st>>>(q, rhs, g.sine, bh, g.nr, g.nz, g.dr, g.dz);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // tridiagonal solves: cyclic reduction up to 256 rows, and up to 1024
    // rows while the modes are too few to fill the GPU with Thomas sweeps
    // (one thread per mode); Thomas sweeps otherwise
    if (nu <= 256)
        k_pcr<D, 4, 4><<<(m + 3) / 4, 256, 0, st>>>(bh, g.nr, g.nz, g.dr, g.dz);
    else if (nu <= 512 && m < kPcrMaxModes)
        k_pcr<D, 8, 2><<<(m + 1) / 2, 128, 0, st>>>(bh, g.nr, g.nz, g.dr, g.dz);
    else if (nu <= 1024 && m < kPcrMaxModes)
        k_pcr<D, 16, 1><<<m, 64, 0, st>>>(bh, g.nr, g.nz, g.dr, g.dz);
    else
        k_thomas<D><<<(m + 255) / 256, 256, 0, st>>>(bh, g.tcp, g.tinv, g.nr, g.nz, g.dr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (B.L > 0)
        k_dst_bluestein<D, false><<<nu, dst_threads(B.L), B.lds, st>>>(nullptr, nullptr, bh, phi, accumulate ? 1 : 0, chirp, fb,
                                                            tw, g.nr, g.nz, B.L, g.dr, g.dz);
    else
        k_idst_rows<D><<<nu, 256, m * sizeof(D), st>>>(bh, g.sine, phi, g.nr, g.nz, accumulate ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Metal-mask Dirichlet condition (Phi = 0 on the mask nodes among the
// unknowns) by a capacitance-matrix correction.  With G_m = A^-1 e_m the
// response to a unit right-hand side at mask node m, the potential
// Phi = Phi_0 + sum_m s_m G_m vanishes on every mask node a when
// C s = -Phi_0|mask with C[a][m] = G_m(node a).  C is built once per grid
// (one solve per mask node) and inverted on the host in FP64 (Gauss-Jordan,
// partial pivoting); each space-charge update then costs one matrix-vector
// product and a second solve whose right-hand side is s on the mask nodes.
// The correction solve is exact for the masked system: the equation holds at
// every other unknown, and the mask rows are replaced by Phi = 0.
// ---------------------------------------------------------------------------
constexpr int32_t kMaxMaskNodes = 2048;

static __global__ __launch_bounds__(64) void k_mask_unit(double *rhs, const int32_t *nodes, int32_t prev,
                                                         int32_t cur) {
    if (threadIdx.x == 0) {
        if (prev >= 0) rhs[nodes[prev]] = 0.0;
        rhs[nodes[cur]] = 1.0;
    }
}

static __global__ __launch_bounds__(256) void k_mask_column(const double *phi, const int32_t *nodes, int32_t M,
                                                            double *c, int32_t col) {
    const int32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < M) c[(int64_t)a * M + col] = phi[nodes[a]];
}

// rhs[node_a] = -sum_m cinv[a][m] phi[node_m]: one block per row a.
static __global__ __launch_bounds__(256) void k_mask_correct(const double *cinv, const int32_t *nodes,
                                                             const double *phi, double *rhs, int32_t M) {
    __shared__ double red[256];
    const int32_t a = blockIdx.x;
    double acc = 0.0;
    for (int32_t m = threadIdx.x; m < M; m += blockDim.x) acc += cinv[(int64_t)a * M + m] * phi[nodes[m]];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int32_t w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int32_t)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) rhs[nodes[a]] = -red[0];
}

static __global__ __launch_bounds__(256) void k_mask_zero(double *phi, const int32_t *nodes, int32_t M) {
    const int32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < M) phi[nodes[a]] = 0.0;
}

// Device tables of the correction; the caller owns the buffers.
struct MaskCap {
    int32_t M = 0;
    bool ready = false;
    int32_t *nodes = nullptr;  // [M] node index j * nr + i
    double *cinv = nullptr;    // [M * M] row-major inverse capacitance
};

// Build C column by column (unit right-hand sides in rhs_tmp, potentials in
// phi_tmp, both nz*nr, rhs_tmp all zero on entry and on return) and store
// its inverse in cap.cinv.  Returns an empty string on success.
template <class D>
inline std::string mask_prepare(const PoissonGrid &g, MaskCap &cap, const std::vector<int32_t> &nodes, D *bh,
                                double *rhs_tmp, double *phi_tmp, hipStream_t st) {
    const int32_t M = (int32_t)nodes.size();
    cap.M = M;
    if (M == 0) {
        cap.ready = true;
        return "";
    }
    hipError_t e = hipMemcpyAsync(cap.nodes, nodes.data(), M * sizeof(int32_t), hipMemcpyHostToDevice, st);
    for (int32_t m = 0; m < M && e == hipSuccess; ++m) {
        k_mask_unit<<<1, 64, 0, st>>>(rhs_tmp, cap.nodes, m - 1, m);
        if ((e = hipGetLastError()) != hipSuccess) break;
        if ((e = poisson_solve<D>(g, nullptr, rhs_tmp, bh, phi_tmp, false, st)) != hipSuccess) break;
        k_mask_column<<<(M + 255) / 256, 256, 0, st>>>(phi_tmp, cap.nodes, M, cap.cinv, m);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        k_mask_zero<<<(M + 255) / 256, 256, 0, st>>>(rhs_tmp, cap.nodes, M);
        e = hipGetLastError();
    }
    std::vector<double> c((size_t)M * M);
    if (e == hipSuccess) e = hipMemcpyAsync(c.data(), cap.cinv, c.size() * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return std::string("capacitance matrix: ") + hipGetErrorString(e);
    if (!invert_in_place(c, M)) return "capacitance matrix is singular";
    e = hipMemcpyAsync(cap.cinv, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return std::string("capacitance matrix upload: ") + hipGetErrorString(e);
    cap.ready = true;
    return "";
}

// After Phi_0 is in phi: induced right-hand side on the mask nodes, the
// correction solve added to phi, and Phi = 0 set on the mask nodes.
template <class D>
inline hipError_t mask_correct(const PoissonGrid &g, const MaskCap &cap, D *bh, double *rhs, double *phi,
                               hipStream_t st) {
    if (cap.M == 0) return hipSuccess;
    k_mask_correct<<<cap.M, 256, 0, st>>>(cap.cinv, cap.nodes, phi, rhs, cap.M);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = poisson_solve<D>(g, nullptr, rhs, bh, phi, true, st)) != hipSuccess) return e;
    k_mask_zero<<<(cap.M + 255) / 256, 256, 0, st>>>(phi, cap.nodes, cap.M);
    return hipGetLastError();
}

}  // namespace mc

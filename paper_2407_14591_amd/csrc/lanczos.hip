// Lanczos on one sector: FP64 scalars on the device, vectors in FP32 or FP64.
//
// Every step is enqueued without a host round trip: the scalars alpha_j,
// beta_j, the re-orthogonalisation coefficients and the stop flag live in
// device memory and are read by the kernels that need them.  Dot products are
// reduced deterministically (per-block partials, then one block that sums
// them in a fixed order), all in FP64.  The Ritz values come from Sturm
// bisection of the tridiagonal matrix in FP64 on the device.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "dcs_internal.h"

namespace dcs {
namespace {

constexpr int kVecThreads = 256;
constexpr int kMaxVecBlocks = 2048;
constexpr int kReduceThreads = 256;
constexpr double kBreakdownTol = 1e-12;

// Device-resident scalar state of one run.
struct LzState {
    int done;          // set once the recurrence stopped
    int steps_done;    // number of alpha values recorded
    double scale;      // running max of |alpha_i|, beta_i
    double inv_beta;   // 1 / beta_j for the next normalisation
    double sc, scp;    // two-vector form: 1/|u_j| and 1/|u_{j-1}| of the stored vectors
    int j;             // two-vector form: the current step (kernels of a captured step read it)
};

template <typename T>
__device__ __forceinline__ double ld(const T *p, uint64_t i) {
    return (double)p[i];
}

// 16-byte vector of T and a test that a pointer allows it.
template <typename T>
struct V16 {
    static constexpr int N = 16 / sizeof(T);
    typedef T type __attribute__((ext_vector_type(16 / sizeof(T))));
};

__device__ __forceinline__ bool aligned16(const void *p) {
    return ((uintptr_t)p & 15u) == 0;
}

// Block-level sum of `v` into slot `slot` of this block's partial row.
__device__ __forceinline__ void block_partial(double v, double *partials, int nslots, int slot) {
    __shared__ double red[kVecThreads / 64];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
        partials[(size_t)blockIdx.x * nslots + slot] = s;
    }
    __syncthreads();
}

// v0 norm^2 partials
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_norm2(const T *__restrict__ v, uint64_t n,
                                                       double *partials) {
    double s = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double a = ld(v, i);
        s += a * a;
    }
    block_partial(s, partials, 1, 0);
}

// out = in * scal[0] (scal on device); skipped once stopped.
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_scale(const T *__restrict__ in, T *__restrict__ out,
                                                       uint64_t n, const double *scal,
                                                       const LzState *st) {
    if (st && st->done) return;
    const double a = *scal;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = (T)(ld(in, i) * a);
}

// w -= beta_{j-1} v_{j-1} (when vprev != NULL), then partial of v_j . w
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_sub_dot(T *__restrict__ w, const T *__restrict__ vj,
                                                         const T *__restrict__ vprev,
                                                         const double *beta_prev, uint64_t n,
                                                         double *partials, const LzState *st) {
    if (st->done) return;
    const double b = vprev ? *beta_prev : 0.0;
    double s = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        double wi = ld(w, i);
        if (vprev) {
            wi -= b * ld(vprev, i);
            w[i] = (T)wi;
            wi = ld(w, i);
        }
        s += ld(vj, i) * wi;
    }
    block_partial(s, partials, 1, 0);
}

// Address of basis vector i: full storage, or a ring of two slots.
template <typename T>
__device__ __forceinline__ const T *basis(const T *V, uint64_t n, int i, int ring) {
    return V + (uint64_t)(ring ? (i & 1) : i) * n;
}

// Optionally w -= a * v_sub (a = *coef_sub), then partials of V_i . w for
// i in [i0, i0 + cnt).  A block owns a contiguous row range; w's slice is
// kept in registers across the cnt dots.
template <typename T, int R>
__global__ __launch_bounds__(kVecThreads) void k_multidot(T *__restrict__ w, const T *__restrict__ V,
                                                          uint64_t n, int ring, int i0, int cnt,
                                                          const T *__restrict__ vsub,
                                                          const double *coef_sub, double *partials,
                                                          const LzState *st) {
    if (st->done) return;
    const uint64_t per_block = ((n + gridDim.x - 1) / gridDim.x + blockDim.x * R - 1) /
                               (blockDim.x * R) * (blockDim.x * R);
    const uint64_t r0 = (uint64_t)blockIdx.x * per_block;
    const uint64_t r1 = min(r0 + per_block, n);
    const double a = vsub ? *coef_sub : 0.0;
    if (vsub)
        for (uint64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
            w[i] = (T)(ld(w, i) - a * ld(vsub, i));
        }
    __syncthreads();
    for (int c = 0; c < cnt; ++c) {
        const T *vi = basis(V, n, i0 + c, ring);
        double s = 0.0;
        for (uint64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) s += ld(vi, i) * ld(w, i);
        block_partial(s, partials, cnt, c);
    }
}

// w -= sum_c coef[c] V_{i0+c}; then partial of |w|^2 (slot 0).
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_sub_multi(T *__restrict__ w, const T *__restrict__ V,
                                                           uint64_t n, int ring, int i0, int cnt,
                                                           const double *coef, double *partials,
                                                           const LzState *st) {
    if (st->done) return;
    __shared__ double cf[512];
    for (int c = threadIdx.x; c < cnt && c < 512; c += blockDim.x) cf[c] = coef[c];
    __syncthreads();
    double s = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        double wi = ld(w, i);
        for (int c = 0; c < cnt; ++c) wi -= (c < 512 ? cf[c] : coef[c]) * ld(basis(V, n, i0 + c, ring), i);
        const T wt = (T)wi;
        w[i] = wt;
        s += (double)wt * (double)wt;
    }
    block_partial(s, partials, 1, 0);
}

// Fixed-order reduction of nblocks x nslots partials into out[0..nslots).
// mode 0: plain sums.  mode 1: alpha_j (records it, updates the scale).
// mode 2: beta_j = sqrt(sum): records it, tests for breakdown, sets 1/beta.
// mode 3: out[0] = 1/sqrt(sum) (vector normalisation).
__global__ __launch_bounds__(kReduceThreads) void k_reduce(const double *partials, int nblocks,
                                                           int nslots, double *out, int mode,
                                                           LzState *st, double *alpha, double *beta,
                                                           int j, int m) {
    if (st && st->done) return;
    __shared__ double red[kReduceThreads];
    for (int slot = 0; slot < nslots; ++slot) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partials[(size_t)b * nslots + slot];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double v = red[0];
            if (mode == 0) {
                out[slot] = v;
            } else if (mode == 1) {
                alpha[j] = v;
                st->steps_done = j + 1;
                st->scale = fmax(st->scale, fabs(v));
            } else if (mode == 2) {
                const double b = sqrt(v);
                st->scale = fmax(st->scale, b);
                if (j + 1 >= m || b <= kBreakdownTol * st->scale) {
                    st->done = 1;
                } else {
                    beta[j] = b;
                    st->inv_beta = 1.0 / b;
                }
            } else {
                out[0] = 1.0 / sqrt(v);
            }
        }
        __syncthreads();
    }
}

// ---- two-vector form (no stored basis) --------------------------------------
//
// The stored vectors are the unnormalised u_j (v_j = u_j / |u_j|, u_0 = v0), so
// no pass rescales a vector.  One step after w = H u_j is two passes:
//  * k_gram: u_j.w, u_{j-1}.w, u_j.u_{j-1};
//  * k_lz_update: u_{j+1} = s w - A u_{j-1} - B u_j and |u_{j+1}|^2,
// with the coefficients from k_lz_coef.  With re-orthogonalisation (LOCAL)
// (A, B) project H v_j onto span(v_{j-1}, v_j) exactly (the 2x2 Gram system of
// the stored operands); without it they are the three-term recurrence's
// (beta_{j-1}, alpha_j).  The coefficients are recorded so the Ritz vector
// pass repeats the same vectors bit for bit.

// partials: slot 0 u_j.w, slot 1 u_{j-1}.w, slot 2 u_j.u_{j-1}
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_gram(const T *__restrict__ w, const T *__restrict__ uj,
                                                      const T *__restrict__ ujm1, uint64_t n,
                                                      double *partials, const LzState *st) {
    if (st->done) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    const uint64_t g0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t head = 0;  // elements done by the 16-byte loop
    if (aligned16(w) && aligned16(uj) && (!ujm1 || aligned16(ujm1))) {
        constexpr int N = V16<T>::N;
        typedef typename V16<T>::type vt;
        const uint64_t nv = n / N;
        for (uint64_t i = g0; i < nv; i += stride) {
            const vt wv = reinterpret_cast<const vt *>(w)[i], av = reinterpret_cast<const vt *>(uj)[i];
            if (ujm1) {
                const vt bv = reinterpret_cast<const vt *>(ujm1)[i];
#pragma unroll
                for (int e = 0; e < N; ++e) {
                    s0 += (double)av[e] * (double)wv[e];
                    s1 += (double)bv[e] * (double)wv[e];
                    s2 += (double)av[e] * (double)bv[e];
                }
            } else {
#pragma unroll
                for (int e = 0; e < N; ++e) s0 += (double)av[e] * (double)wv[e];
            }
        }
        head = nv * N;
    }
    for (uint64_t i = head + g0; i < n; i += stride) {
        const double wi = ld(w, i), a = ld(uj, i);
        s0 += a * wi;
        if (ujm1) {
            const double b = ld(ujm1, i);
            s1 += b * wi;
            s2 += a * b;
        }
    }
    block_partial(s0, partials, 3, 0);
    block_partial(s1, partials, 3, 1);
    block_partial(s2, partials, 3, 2);
}

// Step coefficients from the reduced sums g[0..2]; rec[3j..3j+2] = (s, A, B).
__global__ void k_lz_coef(const double *g, LzState *st, double *alpha, const double *beta,
                          double *rec, int local) {
    if (st->done || threadIdx.x != 0) return;
    const int j = st->j;
    const double s = st->sc, p = st->scp;
    const double r1 = s * s * g[0];  // v_j . H v_j
    const double r0 = p * s * g[1];  // v_{j-1} . H v_j
    const double gm = p * s * g[2];  // v_{j-1} . v_j
    double a = 0.0, b = r1;
    if (j > 0) {
        if (local) {
            const double det = 1.0 - gm * gm;
            a = (r0 - gm * r1) / det;
            b = (r1 - gm * r0) / det;
        } else {
            a = beta[j - 1];
            b = r1 - a * gm;
        }
    }
    alpha[j] = b;
    st->steps_done = j + 1;
    st->scale = fmax(st->scale, fabs(b));
    rec[3 * j] = s;
    rec[3 * j + 1] = a * p;
    rec[3 * j + 2] = b * s;
}

// out = s w - A ujm1 - B uj with (s, A, B) = rec[3j..3j+2] (j = st->j when st is
// given); partial of |out|^2 when
// partials is not NULL.  out may alias ujm1: each element is read before it is
// written, by the same thread.
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_lz_update(const T *__restrict__ w, const T *__restrict__ uj,
                                                           const T *ujm1, T *out, uint64_t n,
                                                           const double *rec, int j, double *partials,
                                                           const LzState *st) {
    if (st && st->done) return;
    const double *c = rec + 3 * (st ? st->j : j);
    const double sw = c[0], A = c[1], B = c[2];
    double s = 0.0;
    const uint64_t g0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t head = 0;
    if (aligned16(w) && aligned16(uj) && (!ujm1 || aligned16(ujm1)) && aligned16(out)) {
        constexpr int N = V16<T>::N;
        typedef typename V16<T>::type vt;
        const uint64_t nv = n / N;
        for (uint64_t i = g0; i < nv; i += stride) {
            const vt wv = reinterpret_cast<const vt *>(w)[i], av = reinterpret_cast<const vt *>(uj)[i];
            vt bv = (vt)(T)0;
            if (ujm1) bv = reinterpret_cast<const vt *>(ujm1)[i];
            vt ov;
#pragma unroll
            for (int e = 0; e < N; ++e) {
                const T vte = (T)(sw * (double)wv[e] - B * (double)av[e] - A * (double)bv[e]);
                ov[e] = vte;
                s += (double)vte * (double)vte;
            }
            reinterpret_cast<vt *>(out)[i] = ov;  // may overwrite ujm1[i], read above by this thread
        }
        head = nv * N;
    }
    for (uint64_t i = head + g0; i < n; i += stride) {
        double v = sw * ld(w, i) - B * ld(uj, i);
        if (ujm1) v -= A * ld(ujm1, i);
        const T vt = (T)v;
        out[i] = vt;
        s += (double)vt * (double)vt;
    }
    if (partials) block_partial(s, partials, 1, 0);
}

// beta_j = sqrt(sum of partials); breakdown test; the new vector's 1/|u|.
__global__ __launch_bounds__(kReduceThreads) void k_lz_norm(const double *partials, int nblocks, LzState *st,
                                                            double *beta, int m) {
    if (st->done) return;
    const int j = st->j;
    __shared__ double red[kReduceThreads];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partials[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double b = sqrt(red[0]);
        st->scale = fmax(st->scale, b);
        if (j + 1 >= m || b <= kBreakdownTol * st->scale) {
            st->done = 1;
        } else {
            beta[j] = b;
            st->scp = st->sc;
            st->sc = 1.0 / b;
            st->j = j + 1;
        }
    }
}

// psi (+)= y_j * s_j * u (y = Ritz coefficients, s_j = rec[3j])
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_axpy_rec(T *__restrict__ psi, const T *__restrict__ u,
                                                          uint64_t n, const double *y, const double *rec,
                                                          int j, int first) {
    const double c = y[j] * rec[3 * j];
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        psi[i] = (T)((first ? 0.0 : ld(psi, i)) + c * ld(u, i));
}

// ---- tridiagonal eigenvalues: Sturm bisection ------------------------------

// Number of eigenvalues of T below x (LDL^T pivots of T - x I).
__device__ int sturm_count(const double *a, const double *b, int m, double x) {
    int c = 0;
    double q = a[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < m; ++i) {
        const double bb = b[i - 1] * b[i - 1];
        if (q == 0.0) q = 1e-300;
        q = a[i] - x - bb / q;
        if (q < 0) ++c;
    }
    return c;
}

__global__ void k_tridiag_bisect(const double *a, const double *b, int m, int num, double *eig) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= num) return;
    double lo = 0, hi = 0;
    for (int i = 0; i < m; ++i) {  // Gershgorin interval
        double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < m ? fabs(b[i]) : 0.0);
        lo = i == 0 ? a[i] - r : fmin(lo, a[i] - r);
        hi = i == 0 ? a[i] + r : fmax(hi, a[i] + r);
    }
    const double span = fmax(hi - lo, 1e-300);
    lo -= 1e-12 * span;
    hi += 1e-12 * span;
    // smallest x with count(x) > e
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count(a, b, m, mid) > e)
            hi = mid;
        else
            lo = mid;
    }
    eig[e] = 0.5 * (lo + hi);
}

// Eigenvector of T for eigenvalue lam by inverse iteration (tridiagonal LU with
// partial pivoting, three sweeps), normalised; one thread.
__global__ void k_tridiag_vec(const double *a, const double *b, int m, const double *lam_p,
                              double *vec, double *work) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double lam = *lam_p;
    double *d = work, *u = work + m, *u2 = work + 2 * m, *l = work + 3 * m;
    int *piv = (int *)(work + 4 * m);
    double scale = 0.0;
    for (int i = 0; i < m; ++i) scale = fmax(scale, fabs(a[i]) + (i < m - 1 ? fabs(b[i]) : 0.0));
    const double tiny = 1e-14 * fmax(scale, 1e-300);
    // LU of T - lam I with partial pivoting: rows i, i+1
    for (int i = 0; i < m; ++i) {
        d[i] = a[i] - lam;
        u[i] = i < m - 1 ? b[i] : 0.0;
        u2[i] = 0.0;
    }
    for (int i = 0; i < m - 1; ++i) {
        const double sub = b[i];
        if (fabs(sub) > fabs(d[i])) {  // swap rows i and i+1
            piv[i] = 1;
            const double nd = sub, nu = d[i + 1], nu2 = i + 1 < m - 1 ? u[i + 1] : 0.0;
            const double od = d[i], ou = u[i];
            d[i] = nd;
            u[i] = nu;
            u2[i] = nu2;
            const double f = od / nd;
            l[i] = f;
            d[i + 1] = ou - f * nu;
            u[i + 1] = (i + 1 < m - 1) ? 0.0 - f * nu2 : 0.0;
        } else {
            piv[i] = 0;
            const double dd = fabs(d[i]) < tiny ? tiny : d[i];
            d[i] = dd;
            const double f = sub / dd;
            l[i] = f;
            d[i + 1] -= f * u[i];
        }
    }
    if (fabs(d[m - 1]) < tiny) d[m - 1] = tiny;
    for (int i = 0; i < m; ++i) vec[i] = 1.0;
    for (int sweep = 0; sweep < 3; ++sweep) {
        // forward: apply L^{-1} P
        for (int i = 0; i < m - 1; ++i) {
            if (piv[i]) {
                const double t = vec[i];
                vec[i] = vec[i + 1];
                vec[i + 1] = t;
            }
            vec[i + 1] -= l[i] * vec[i];
        }
        // backward: U x = y
        for (int i = m - 1; i >= 0; --i) {
            double s = vec[i];
            if (i + 1 < m) s -= u[i] * vec[i + 1];
            if (i + 2 < m) s -= u2[i] * vec[i + 2];
            vec[i] = s / d[i];
        }
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += vec[i] * vec[i];
        nrm = sqrt(nrm);
        for (int i = 0; i < m; ++i) vec[i] /= nrm;
    }
}

// psi += s[j] * v  (s on device)
template <typename T>
__global__ __launch_bounds__(kVecThreads) void k_axpy_s(T *__restrict__ psi, const T *__restrict__ v,
                                                        uint64_t n, const double *s, int j, int first) {
    const double c = s[j];
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        psi[i] = (T)((first ? 0.0 : ld(psi, i)) + c * ld(v, i));
}

int vec_blocks(uint64_t n) {
    uint64_t b = (n + kVecThreads * 4 - 1) / (kVecThreads * 4);
    if (b > kMaxVecBlocks) b = kMaxVecBlocks;
    return (int)std::max<uint64_t>(b, 1);
}

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Slot stride of the two-vector ring: a multiple of 64 elements, so both slots
// allow 16-byte vector access.
inline uint64_t ring_stride(uint64_t n) { return (n + 63) / 64 * 64; }

struct Layout {
    size_t V, w, psi_tmp, partials, alpha, beta, coef, rec, state, trid, total;
    int m, nvec;
};

Layout layout(const dcs_sector *s, int dtype, int steps, int reorth, int num_vec) {
    const int want_vec = num_vec > 0;
    Layout L;
    const uint64_t n = s->desc.dim;
    const size_t es = dtype == DCS_F32 ? 4 : 8;
    L.m = (int)std::min<uint64_t>((uint64_t)std::max(steps, 1), n);
    L.nvec = reorth == DCS_REORTH_FULL ? L.m : 2;
    size_t p = 0;
    L.V = p;
    p = align256(p + (size_t)L.nvec * (reorth == DCS_REORTH_FULL ? n : ring_stride(n)) * es);
    L.w = p;
    p = align256(p + n * es);
    L.psi_tmp = p;  // second-pass vectors (ring of 2) when the basis is not stored
    if (want_vec && reorth != DCS_REORTH_FULL) p = align256(p + 2 * ring_stride(n) * es);
    L.partials = p;
    p = align256(p + (size_t)kMaxVecBlocks * (size_t)std::max(L.m, 2) * sizeof(double));
    L.alpha = p;
    p = align256(p + (size_t)L.m * sizeof(double));
    L.beta = p;
    p = align256(p + (size_t)L.m * sizeof(double));
    L.coef = p;
    p = align256(p + (size_t)(L.m + 4) * sizeof(double));
    L.rec = p;  // two-vector form: (s, A, B) per step
    p = align256(p + (size_t)(3 * L.m + 3) * sizeof(double));
    L.state = p;
    p = align256(p + sizeof(LzState));
    L.trid = p;  // eigenvalues, inverse-iteration work, eigenvectors of T (one per Ritz vector)
    p = align256(p + (size_t)(7 * L.m + 16 + (size_t)std::max(num_vec, 1) * L.m) * sizeof(double));
    L.total = p;
    return L;
}

// DCS_LANCZOS_GRAPH=0 in the environment (read at every call) launches every step
// eagerly instead of replaying captured steps.
bool lanczos_graph_enabled() {
    const char *e = getenv("DCS_LANCZOS_GRAPH");
    return !(e && e[0] == '0');
}

// Steps 2..m-1 of the two-vector form as two captured HIP graphs (one per parity
// of j), replayed on a private stream ordered after and before `stream`.  The
// step's launches read the step index from device memory, so a replay needs no
// host work.
template <typename StepFn, typename T>
int replay_steps(StepFn &step, T *ring0, T *ring1, int m, hipStream_t stream) {
    hipStream_t gs = nullptr;
    hipEvent_t ev = nullptr;
    hipGraphExec_t ex[2] = {nullptr, nullptr};
    int r = check_hip(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking), "Lanczos graph stream");
    if (!r) r = check_hip(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "Lanczos graph event");
    if (!r) r = check_hip(hipEventRecord(ev, stream), "Lanczos graph event record");
    if (!r) r = check_hip(hipStreamWaitEvent(gs, ev, 0), "Lanczos graph stream wait");
    for (int p = 0; p < 2 && !r; ++p) {
        T *cur = p ? ring1 : ring0, *prev = p ? ring0 : ring1;
        hipGraph_t g = nullptr;
        r = check_hip(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal), "Lanczos capture");
        if (r) break;
        const int rs = step(cur, prev, prev, gs);
        const int re = check_hip(hipStreamEndCapture(gs, &g), "Lanczos end capture");
        r = rs ? rs : re;
        if (!r) r = check_hip(hipGraphInstantiate(&ex[p], g, nullptr, nullptr, 0), "Lanczos graph instantiate");
        if (g) hipGraphDestroy(g);
    }
    for (int j = 2; j < m && !r; ++j) r = check_hip(hipGraphLaunch(ex[j & 1], gs), "Lanczos graph launch");
    if (!r) r = check_hip(hipEventRecord(ev, gs), "Lanczos graph event record");
    if (!r) r = check_hip(hipStreamWaitEvent(stream, ev, 0), "Lanczos graph join");
    if (gs) hipStreamSynchronize(gs);
    for (auto &e : ex)
        if (e) hipGraphExecDestroy(e);
    if (ev) hipEventDestroy(ev);
    if (gs) hipStreamDestroy(gs);
    return r;
}

// apply(in, out, stream) launches w = A v for the operator of the run (the XXZ
// Hamiltonian of a terms object, or a generic operator); it must be capturable.
template <typename T, typename Apply>
int run_lanczos(const dcs_sector *s, const Apply &apply, int dtype, int steps, int reorth,
                const void *v0, double *h_alpha, double *h_beta, int *h_steps, int num_eig,
                double *h_eig, void *vecs, int num_vec, char *ws, hipStream_t stream) {
    const uint64_t n = s->desc.dim;
    const Layout L = layout(s, dtype, steps, reorth, vecs ? num_vec : 0);
    T *V = (T *)(ws + L.V);
    T *w = (T *)(ws + L.w);
    double *part = (double *)(ws + L.partials);
    double *alpha = (double *)(ws + L.alpha);
    double *beta = (double *)(ws + L.beta);
    double *coef = (double *)(ws + L.coef);
    LzState *st = (LzState *)(ws + L.state);
    double *trid = (double *)(ws + L.trid);
    const int nb = vec_blocks(n);
    const int ring = reorth == DCS_REORTH_FULL ? 0 : 1;
    auto vec = [&](int i) -> T * { return V + (uint64_t)(ring ? (i & 1) : i) * n; };
    auto chk = [&](const char *what) { return check_hip(hipGetLastError(), what); };

    if (int r = check_hip(hipMemsetAsync(st, 0, sizeof(LzState), stream), "hipMemsetAsync"))
        return r;
    double *rec = (double *)(ws + L.rec);
    const T *u0 = (const T *)v0;
    // two-vector form: u_0 = v0 as given, u_{j>0} in the ring (slot j & 1)
    if (ring) {
        k_norm2<T><<<nb, kVecThreads, 0, stream>>>(u0, n, part);
        k_reduce<<<1, kReduceThreads, 0, stream>>>(part, nb, 1, &st->sc, 3, nullptr, alpha, beta, 0,
                                                   L.m);
        if (int r = chk("Lanczos start")) return r;
        const int local = reorth == DCS_REORTH_LOCAL ? 1 : 0;
        T *ring0 = V, *ring1 = V + ring_stride(n);
        // one step; the kernels take the step index from the device state, so the
        // same launches serve every step of one parity (u_j, u_{j-1}, u_{j+1} slots)
        auto step = [&](const T *uj, const T *ujm1, T *out, hipStream_t q) -> int {
            if (int r = apply(uj, w, q)) return r;
            k_gram<T><<<nb, kVecThreads, 0, q>>>(w, uj, ujm1, n, part, st);
            k_reduce<<<1, kReduceThreads, 0, q>>>(part, nb, 3, coef, 0, st, alpha, beta, 0, L.m);
            k_lz_coef<<<1, 64, 0, q>>>(coef, st, alpha, beta, rec, local);
            k_lz_update<T><<<nb, kVecThreads, 0, q>>>(w, uj, ujm1, out, n, rec, 0, part, st);
            k_lz_norm<<<1, kReduceThreads, 0, q>>>(part, nb, st, beta, L.m);
            return chk("Lanczos step");
        };
        if (int r = step(u0, nullptr, ring1, stream)) return r;               // j = 0
        if (L.m > 1)
            if (int r = step(ring1, u0, ring0, stream)) return r;             // j = 1
        if (L.m > 2) {
            if (lanczos_graph_enabled()) {
                if (int r = replay_steps(step, ring0, ring1, L.m, stream)) return r;
            } else {
                for (int j = 2; j < L.m; ++j) {
                    T *cur = (j & 1) ? ring1 : ring0, *prev = (j & 1) ? ring0 : ring1;
                    if (int r = step(cur, prev, prev, stream)) return r;
                }
            }
        }
    } else {
        // v_0 = v0 / |v0|
        k_norm2<T><<<nb, kVecThreads, 0, stream>>>((const T *)v0, n, part);
        k_reduce<<<1, kReduceThreads, 0, stream>>>(part, nb, 1, &st->inv_beta, 3, nullptr, alpha,
                                                   beta, 0, L.m);
        k_scale<T><<<nb, kVecThreads, 0, stream>>>((const T *)v0, vec(0), n, &st->inv_beta, nullptr);
        if (int r = chk("Lanczos start")) return r;
        for (int j = 0; j < L.m; ++j) {
            if (int r = apply(vec(j), w, stream)) return r;
            k_sub_dot<T><<<nb, kVecThreads, 0, stream>>>(w, vec(j), j > 0 ? vec(j - 1) : nullptr,
                                                         j > 0 ? beta + j - 1 : nullptr, n, part, st);
            k_reduce<<<1, kReduceThreads, 0, stream>>>(part, nb, 1, nullptr, 1, st, alpha, beta, j,
                                                       L.m);
            // full re-orthogonalisation: classical Gram-Schmidt twice against v_0..v_j
            for (int p = 0; p < 2; ++p) {
                k_multidot<T, 4><<<nb, kVecThreads, 0, stream>>>(
                    w, V, n, 0, 0, j + 1, p == 0 ? vec(j) : nullptr, alpha + j, part, st);
                k_reduce<<<1, kReduceThreads, 0, stream>>>(part, nb, j + 1, coef, 0, st, alpha, beta,
                                                           j, L.m);
                k_sub_multi<T><<<nb, kVecThreads, 0, stream>>>(w, V, n, 0, 0, j + 1, coef, part, st);
            }
            k_reduce<<<1, kReduceThreads, 0, stream>>>(part, nb, 1, nullptr, 2, st, alpha, beta, j,
                                                       L.m);
            if (j + 1 < L.m)
                k_scale<T><<<nb, kVecThreads, 0, stream>>>(w, vec(j + 1), n, &st->inv_beta, st);
            if (int r = chk("Lanczos step")) return r;
        }
    }
    LzState hs;
    if (int r = check_hip(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, stream),
                          "copy Lanczos state"))
        return r;
    if (int r = check_hip(hipStreamSynchronize(stream), "Lanczos synchronise")) return r;
    const int md = hs.steps_done;
    *h_steps = md;
    if (md < 1) return set_error(DCS_EHIP, "Lanczos recorded no step");
    std::vector<double> ha(md), hb(std::max(md - 1, 0));
    if (int r = check_hip(hipMemcpy(ha.data(), alpha, md * sizeof(double), hipMemcpyDeviceToHost),
                          "copy alpha"))
        return r;
    if (md > 1 &&
        check_hip(hipMemcpy(hb.data(), beta, (md - 1) * sizeof(double), hipMemcpyDeviceToHost),
                  "copy beta"))
        return DCS_EHIP;
    if (h_alpha) memcpy(h_alpha, ha.data(), md * sizeof(double));
    if (h_beta && md > 1) memcpy(h_beta, hb.data(), (md - 1) * sizeof(double));
    const int nv = vecs ? std::min(num_vec, md) : 0;  // Ritz vectors asked for (at most md)
    const int ne = std::max(std::min(num_eig, md), nv);
    double *eig = trid, *work = trid + 16 + md, *svecs = trid + 16 + 7 * md;
    if (ne > 0) {
        k_tridiag_bisect<<<(ne + 63) / 64, 64, 0, stream>>>(alpha, beta, md, ne, eig);
        if (int r = chk("tridiagonal bisection")) return r;
        std::vector<double> he(ne);
        if (int r = check_hip(hipMemcpyAsync(he.data(), eig, ne * sizeof(double),
                                             hipMemcpyDeviceToHost, stream),
                              "copy Ritz values"))
            return r;
        if (int r = check_hip(hipStreamSynchronize(stream), "Ritz synchronise")) return r;
        if (h_eig)
            for (int e = 0; e < std::min(num_eig, md); ++e) h_eig[e] = he[e];
    }
    if (!nv) return DCS_OK;
    // Ritz vectors of the nv lowest Ritz values: psi_e = sum_j s_e[j] v_j, normalised
    // (s_e: eigenvector of T for eig[e] by inverse iteration)
    for (int e = 0; e < nv; ++e)
        k_tridiag_vec<<<1, 1, 0, stream>>>(alpha, beta, md, eig + e, svecs + (size_t)e * md, work);
    auto psi_of = [&](int e) { return (T *)vecs + (uint64_t)e * n; };
    double *inv = coef + L.m;  // two spare scalars
    if (reorth == DCS_REORTH_FULL) {
        for (int e = 0; e < nv; ++e)
            for (int j = 0; j < md; ++j)
                k_axpy_s<T><<<nb, kVecThreads, 0, stream>>>(psi_of(e), vec(j), n, svecs + (size_t)e * md, j, j == 0);
    } else {
        // repeat the recorded two-vector recurrence once (same kernels, same vectors),
        // adding every step's vector to all nv Ritz vectors
        T *R = (T *)(ws + L.psi_tmp);
        auto rv = [&](int i) -> const T * { return i == 0 ? u0 : R + (uint64_t)(i & 1) * ring_stride(n); };
        for (int e = 0; e < nv; ++e)
            k_axpy_rec<T><<<nb, kVecThreads, 0, stream>>>(psi_of(e), rv(0), n, svecs + (size_t)e * md, rec, 0, 1);
        for (int j = 0; j + 1 < md; ++j) {
            if (int r = apply(rv(j), w, stream)) return r;
            k_lz_update<T><<<nb, kVecThreads, 0, stream>>>(w, rv(j), j > 0 ? rv(j - 1) : nullptr,
                                                           R + (uint64_t)((j + 1) & 1) * ring_stride(n), n,
                                                           rec, j, nullptr, nullptr);
            for (int e = 0; e < nv; ++e)
                k_axpy_rec<T><<<nb, kVecThreads, 0, stream>>>(psi_of(e), rv(j + 1), n, svecs + (size_t)e * md,
                                                              rec, j + 1, 0);
            if (int r = chk("Ritz vector replay")) return r;
        }
    }
    if (int r = chk("Ritz vector")) return r;
    for (int e = 0; e < nv; ++e) {
        k_norm2<T><<<nb, kVecThreads, 0, stream>>>(psi_of(e), n, part);
        k_reduce<<<1, kReduceThreads, 0, stream>>>(part, nb, 1, inv + 1, 3, nullptr, alpha, beta, 0,
                                                   L.m);
        k_scale<T><<<nb, kVecThreads, 0, stream>>>(psi_of(e), psi_of(e), n, inv + 1, nullptr);
    }
    return chk("Ritz vector norm");
}

}  // namespace
}  // namespace dcs

using namespace dcs;

extern "C" int dcs_lanczos_workspace_size(const dcs_sector *s, int dtype, int steps, int reorth,
                                          int num_vec, size_t *bytes) {
    clear_error();
    if (!s || !bytes) return set_error(DCS_EINVAL, "NULL argument");
    if (dtype != DCS_F32 && dtype != DCS_F64) return set_error(DCS_EINVAL, "dtype %d", dtype);
    if (reorth < DCS_REORTH_NONE || reorth > DCS_REORTH_FULL)
        return set_error(DCS_EINVAL, "reorth %d", reorth);
    if (steps < 1) return set_error(DCS_EINVAL, "steps %d < 1", steps);
    if (num_vec < 0) return set_error(DCS_EINVAL, "num_vec %d", num_vec);
    *bytes = layout(s, dtype, steps, reorth, num_vec).total;
    return DCS_OK;
}

extern "C" int dcs_lanczos(const dcs_sector *s, const dcs_terms *t, const double *jxy,
                           const double *jz, const double *h, int dtype, int steps, int reorth,
                           const void *v0, double *h_alpha, double *h_beta, int *h_steps,
                           int num_eig, double *h_eig, void *vecs, int num_vec, void *ws,
                           size_t ws_bytes, void *stream) {
    clear_error();
    if (!s || !t || !v0 || !h_steps) return set_error(DCS_EINVAL, "NULL argument");
    if (int r = refuse_mixed(s)) return r;
    if (dtype != DCS_F32 && dtype != DCS_F64) return set_error(DCS_EINVAL, "dtype %d", dtype);
    if (reorth < DCS_REORTH_NONE || reorth > DCS_REORTH_FULL)
        return set_error(DCS_EINVAL, "reorth %d", reorth);
    if (steps < 1) return set_error(DCS_EINVAL, "steps %d < 1", steps);
    if (num_eig < 0 || (num_eig > 0 && !h_eig)) return set_error(DCS_EINVAL, "num_eig / h_eig");
    if (t->num_bonds > 0 && (!jxy || !jz)) return set_error(DCS_EINVAL, "NULL couplings");
    if (vecs && num_vec < 1) return set_error(DCS_EINVAL, "num_vec %d with a vector output", num_vec);
    if (!vecs) num_vec = 0;
    const Layout L = layout(s, dtype, steps, reorth, num_vec);
    if (!ws || ws_bytes < L.total)
        return set_error(DCS_EINVAL, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
    DeviceGuard dg(s->device);
    auto apply = [&](const void *in, void *out, hipStream_t q) {
        return launch_hx(s, t, jxy, jz, h, dtype, 1, in, out, q);
    };
    if (dtype == DCS_F32)
        return run_lanczos<float>(s, apply, dtype, steps, reorth, v0, h_alpha, h_beta, h_steps, num_eig, h_eig,
                                  vecs, num_vec, (char *)ws, (hipStream_t)stream);
    return run_lanczos<double>(s, apply, dtype, steps, reorth, v0, h_alpha, h_beta, h_steps, num_eig, h_eig,
                               vecs, num_vec, (char *)ws, (hipStream_t)stream);
}

extern "C" int dcs_lanczos_operator(const dcs_sector *s, const dcs_operator *op, int dtype, int steps,
                                    int reorth, const void *v0, double *h_alpha, double *h_beta,
                                    int *h_steps, int num_eig, double *h_eig, void *vecs, int num_vec,
                                    void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    if (!s || !op || !v0 || !h_steps) return set_error(DCS_EINVAL, "NULL argument");
    if (dtype != DCS_F32 && dtype != DCS_F64) return set_error(DCS_EINVAL, "dtype %d", dtype);
    if (reorth < DCS_REORTH_NONE || reorth > DCS_REORTH_FULL)
        return set_error(DCS_EINVAL, "reorth %d", reorth);
    if (steps < 1) return set_error(DCS_EINVAL, "steps %d < 1", steps);
    if (num_eig < 0 || (num_eig > 0 && !h_eig)) return set_error(DCS_EINVAL, "num_eig / h_eig");
    if (vecs && num_vec < 1) return set_error(DCS_EINVAL, "num_vec %d with a vector output", num_vec);
    if (!vecs) num_vec = 0;
    if (int r = operator_check(s, op, dtype, 1)) return r;
    const Layout L = layout(s, dtype, steps, reorth, num_vec);
    if (!ws || ws_bytes < L.total)
        return set_error(DCS_EINVAL, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
    DeviceGuard dg(s->device);
    auto apply = [&](const void *in, void *out, hipStream_t q) {
        return launch_operator(s, op, dtype, 1, in, out, q);
    };
    if (dtype == DCS_F32)
        return run_lanczos<float>(s, apply, dtype, steps, reorth, v0, h_alpha, h_beta, h_steps, num_eig, h_eig,
                                  vecs, num_vec, (char *)ws, (hipStream_t)stream);
    return run_lanczos<double>(s, apply, dtype, steps, reorth, v0, h_alpha, h_beta, h_steps, num_eig, h_eig,
                               vecs, num_vec, (char *)ws, (hipStream_t)stream);
}

extern "C" int dcs_tridiag_eigvals(const double *h_alpha, const double *h_beta, int m, int num,
                                   double *h_eig, int device) {
    clear_error();
    if (!h_alpha || (m > 1 && !h_beta) || !h_eig || m < 1 || num < 1 || num > m)
        return set_error(DCS_EINVAL, "bad arguments");
    DeviceGuard dg(device);
    double *d = nullptr;
    if (int r = check_hip(hipMalloc(&d, (size_t)(3 * m + 1) * sizeof(double)), "hipMalloc"))
        return r;
    int r = check_hip(hipMemcpy(d, h_alpha, m * sizeof(double), hipMemcpyHostToDevice), "copy");
    if (!r && m > 1)
        r = check_hip(hipMemcpy(d + m, h_beta, (m - 1) * sizeof(double), hipMemcpyHostToDevice),
                      "copy");
    if (!r) {
        k_tridiag_bisect<<<(num + 63) / 64, 64>>>(d, d + m, m, num, d + 2 * m);
        r = check_hip(hipGetLastError(), "bisection launch");
    }
    if (!r)
        r = check_hip(hipMemcpy(h_eig, d + 2 * m, num * sizeof(double), hipMemcpyDeviceToHost),
                      "copy eigenvalues");
    hipFree(d);
    return r;
}

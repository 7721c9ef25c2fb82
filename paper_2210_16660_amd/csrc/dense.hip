// Coarsest level: dense Cholesky factorization A_L = L L^T and the explicit
// inverse A_L^{-1} = L^{-T} L^{-1}, computed once at setup on the device
// (Sec. 3.1 solves the coarsest system directly).  The V-cycle then applies
// the inverse as one matrix-vector (or, for 16 right-hand sides, one
// matrix-matrix) product.
//
// Blocked algorithms on 64 x 64 tiles of the zero-padded N x N matrix
// (N = n rounded up to 64; the padding carries an identity diagonal, so the
// factor and the inverse of the padded matrix are block-diagonal with the
// wanted ones in the top-left corner):
//   factor:  for each block column k: unblocked Cholesky of the diagonal tile
//            and its triangular inverse in LDS; panel L_ik = A_ik L_kk^{-T};
//            trailing update A_ij -= L_ik L_jk^T  (j <= i);
//   inverse: X = L^{-1} by block forward substitution on the identity
//            (X_ic = L_ii^{-1} X_ic, then X_mc -= L_mi X_ic for m > i);
//            A^{-1} = X^T X on the lower block triangle, mirrored.
// Every tile product runs on the matrix cores (v_mfma_f64_16x16x4_f64): one
// wave per 16-row strip of the 64 x 64 output tile, four 16-column tiles.
// All sums have a fixed order, so the result is deterministic.
#include <hip/hip_runtime.h>

#include <cmath>

#include "hier.hpp"

namespace pamg {
namespace {

constexpr int kT = 64;             // tile edge
constexpr int kTP = kT + 1;        // padded LDS row (bank spread)
constexpr int kDenseThreads = 256; // four waves

using d4 = __attribute__((__vector_size__(4 * sizeof(double)))) double;

// acc[ct] += A(strip rows, 0..63) * B(0..63, tile ct columns) for this wave's
// 16-row strip.  MFMA operand layout (16x16x4, FP64): the A fragment lane l
// holds A[l % 16][l / 16], the B fragment lane l holds B[l / 16][l % 16]; the
// result register i of lane l is row 4 i + l / 16, column l % 16.
template <class FA, class FB>
__device__ __forceinline__ void strip_product(d4 (&acc)[4], int wave, int lane, FA a_at, FB b_at) {
    const int ar = 16 * wave + (lane % 16);
    const int kq = lane / 16;
    const int bc = lane % 16;
#pragma unroll 4
    for (int k0 = 0; k0 < kT; k0 += 4) {
        const double a = a_at(ar, k0 + kq);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b_at(k0 + kq, 16 * ct + bc), acc[ct], 0, 0, 0);
    }
}

__device__ __forceinline__ void zero(d4 (&acc)[4]) {
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[ct] = d4{0.0, 0.0, 0.0, 0.0};
}

// (row, col) inside the 64 x 64 tile of result register i, column tile ct
__device__ __forceinline__ int res_row(int wave, int lane, int i) { return 16 * wave + 4 * i + lane / 16; }
__device__ __forceinline__ int res_col(int lane, int ct) { return 16 * ct + lane % 16; }

__device__ __forceinline__ void load_tile(double (*S)[kTP], const double* __restrict__ g, int ld) {
    for (int e = threadIdx.x; e < kT * kT; e += kDenseThreads) S[e / kT][e % kT] = g[(size_t)(e / kT) * ld + e % kT];
}

// M = 0 beforehand; scatter the CSR of the coarsest level, identity padding
__global__ __launch_bounds__(kDenseThreads) void k_dense_scatter(int n, int N, const int* __restrict__ rp,
                                                                 const int* __restrict__ ci,
                                                                 const double* __restrict__ v, double* __restrict__ M) {
    const int i = blockIdx.x * kDenseThreads + threadIdx.x;
    if (i >= N) return;
    if (i >= n) {
        M[(size_t)i * N + i] = 1.0;
        return;
    }
    for (int k = rp[i]; k < rp[i + 1]; ++k) M[(size_t)i * N + ci[k]] = v[k];
}

__global__ __launch_bounds__(kDenseThreads) void k_dense_eye(int N, double* __restrict__ X) {
    const int i = blockIdx.x * kDenseThreads + threadIdx.x;
    if (i < N) X[(size_t)i * N + i] = 1.0;
}

// Diagonal tile kb: unblocked Cholesky in LDS (lower), written back with
// zeros above the diagonal, and its triangular inverse into Dinv[kb].  A
// pivot that is not positive sets *bad and is replaced by 1 so that the rest
// stays finite; the host then reports the matrix as not positive definite.
__global__ __launch_bounds__(kDenseThreads) void k_dense_potrf_tile(double* __restrict__ M, int N, int kb,
                                                                    double* __restrict__ Dinv, int* __restrict__ bad) {
    __shared__ double S[kT][kTP];
    __shared__ double T[kT][kTP];
    const int tid = threadIdx.x;
    double* G = M + (size_t)kb * kT * N + (size_t)kb * kT;
    load_tile(S, G, N);
    __syncthreads();
    for (int j = 0; j < kT; ++j) {
        if (tid == 0) {
            double d = S[j][j];
            if (!(d > 0.0)) {
                *bad = 1;
                d = 1.0;
            }
            S[j][j] = sqrt(d);
        }
        __syncthreads();
        const double djj = S[j][j];
        for (int i = j + 1 + tid; i < kT; i += kDenseThreads) S[i][j] /= djj;
        __syncthreads();
        for (int e = tid; e < kT * kT; e += kDenseThreads) {
            const int r = e / kT, c = e % kT;
            if (c > j && r >= c) S[r][c] -= S[r][j] * S[c][j];
        }
        __syncthreads();
    }
    // column c of the inverse by forward substitution (one thread per column)
    if (tid < kT) {
        const int c = tid;
        for (int i = 0; i < c; ++i) T[i][c] = 0.0;
        T[c][c] = 1.0 / S[c][c];
        for (int i = c + 1; i < kT; ++i) {
            double s = 0.0;
            for (int m = c; m < i; ++m) s += S[i][m] * T[m][c];
            T[i][c] = -s / S[i][i];
        }
    }
    __syncthreads();
    double* D = Dinv + (size_t)kb * kT * kT;
    for (int e = tid; e < kT * kT; e += kDenseThreads) {
        const int r = e / kT, c = e % kT;
        G[(size_t)r * N + c] = c <= r ? S[r][c] : 0.0;
        D[e] = T[r][c];
    }
}

// Panel: L_ik = A_ik L_kk^{-T} for the row tiles i = kb+1+blockIdx.x.
__global__ __launch_bounds__(kDenseThreads) void k_dense_panel(double* __restrict__ M, int N, int kb,
                                                               const double* __restrict__ Dinv) {
    __shared__ double Dk[kT][kTP];
    __shared__ double A[kT][kTP];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int ib = kb + 1 + blockIdx.x;
    double* G = M + (size_t)ib * kT * N + (size_t)kb * kT;
    load_tile(Dk, Dinv + (size_t)kb * kT * kT, kT);
    load_tile(A, G, N);
    __syncthreads();
    d4 acc[4];
    zero(acc);
    strip_product(acc, wave, lane, [&](int r, int k) { return A[r][k]; }, [&](int k, int c) { return Dk[c][k]; });
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) G[(size_t)res_row(wave, lane, i) * N + res_col(lane, ct)] = acc[ct][i];
}

// Decode p -> (i, j), 0 <= j <= i, p = i (i + 1) / 2 + j.
__device__ __forceinline__ void tri_index(long long p, int& i, int& j) {
    int r = (int)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while ((long long)(r + 1) * (r + 2) / 2 <= p) ++r;
    while ((long long)r * (r + 1) / 2 > p) --r;
    i = r;
    j = (int)(p - (long long)r * (r + 1) / 2);
}

// Trailing update: A_ij -= L_ik L_jk^T for kb < j <= i (one tile per block).
__global__ __launch_bounds__(kDenseThreads) void k_dense_syrk(double* __restrict__ M, int N, int kb) {
    __shared__ double Pi[kT][kTP];
    __shared__ double Pj[kT][kTP];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    int i, j;
    tri_index(blockIdx.x, i, j);
    const int ib = kb + 1 + i, jb = kb + 1 + j;
    load_tile(Pi, M + (size_t)ib * kT * N + (size_t)kb * kT, N);
    load_tile(Pj, M + (size_t)jb * kT * N + (size_t)kb * kT, N);
    __syncthreads();
    d4 acc[4];
    zero(acc);
    strip_product(acc, wave, lane, [&](int r, int k) { return Pi[r][k]; }, [&](int k, int c) { return Pj[c][k]; });
    double* G = M + (size_t)ib * kT * N + (size_t)jb * kT;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int q = 0; q < 4; ++q) G[(size_t)res_row(wave, lane, q) * N + res_col(lane, ct)] -= acc[ct][q];
}

// X_ic = L_ii^{-1} X_ic for the block columns c = blockIdx.x <= i.
__global__ __launch_bounds__(kDenseThreads) void k_dense_trmm(double* __restrict__ X, int N, int ib,
                                                              const double* __restrict__ Dinv) {
    __shared__ double Di[kT][kTP];
    __shared__ double B[kT][kTP];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    double* G = X + (size_t)ib * kT * N + (size_t)blockIdx.x * kT;
    load_tile(Di, Dinv + (size_t)ib * kT * kT, kT);
    load_tile(B, G, N);
    __syncthreads();
    d4 acc[4];
    zero(acc);
    strip_product(acc, wave, lane, [&](int r, int k) { return Di[r][k]; }, [&](int k, int c) { return B[k][c]; });
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int q = 0; q < 4; ++q) G[(size_t)res_row(wave, lane, q) * N + res_col(lane, ct)] = acc[ct][q];
}

// X_mc -= L_mi X_ic for m = ib+1 .. nb-1 and c = 0 .. ib
// (blockIdx.x = (m - ib - 1) * (ib + 1) + c).
__global__ __launch_bounds__(kDenseThreads) void k_dense_fwd_update(double* __restrict__ X, const double* __restrict__ M,
                                                                    int N, int ib) {
    __shared__ double Lm[kT][kTP];
    __shared__ double B[kT][kTP];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int m = ib + 1 + (int)(blockIdx.x / (ib + 1));
    const int c = (int)(blockIdx.x % (ib + 1));
    load_tile(Lm, M + (size_t)m * kT * N + (size_t)ib * kT, N);
    load_tile(B, X + (size_t)ib * kT * N + (size_t)c * kT, N);
    __syncthreads();
    d4 acc[4];
    zero(acc);
    strip_product(acc, wave, lane, [&](int r, int k) { return Lm[r][k]; }, [&](int k, int cc) { return B[k][cc]; });
    double* G = X + (size_t)m * kT * N + (size_t)c * kT;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int q = 0; q < 4; ++q) G[(size_t)res_row(wave, lane, q) * N + res_col(lane, ct)] -= acc[ct][q];
}

// A^{-1}_ab = sum_{k >= a} X_ka^T X_kb for a >= b (one tile per block),
// written to the n x n output and mirrored; on diagonal tiles only the lower
// triangle is computed-and-mirrored so that the output is exactly symmetric.
__global__ __launch_bounds__(kDenseThreads) void k_dense_xtx(const double* __restrict__ X, int N, int nb, int n,
                                                             double* __restrict__ out) {
    __shared__ double Xa[kT][kTP];
    __shared__ double Xb[kT][kTP];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    int a, b;
    tri_index(blockIdx.x, a, b);
    d4 acc[4];
    zero(acc);
    for (int k = a; k < nb; ++k) {
        load_tile(Xa, X + (size_t)k * kT * N + (size_t)a * kT, N);
        load_tile(Xb, X + (size_t)k * kT * N + (size_t)b * kT, N);
        __syncthreads();
        strip_product(acc, wave, lane, [&](int r, int kk) { return Xa[kk][r]; }, [&](int kk, int c) { return Xb[kk][c]; });
        __syncthreads();
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = a * kT + res_row(wave, lane, q), c = b * kT + res_col(lane, ct);
            if (r >= n || c >= n || (a == b && c > r)) continue;
            out[(size_t)r * n + c] = acc[ct][q];
            if (r != c) out[(size_t)c * n + r] = acc[ct][q];
        }
}

}  // namespace

std::unique_ptr<DenseWork> dense_work(pamg_context* ctx, int n, hipStream_t s) {
    const int N = (n + kT - 1) / kT * kT;
    const int nb = N / kT;
    const size_t NN = (size_t)N * N;
    std::unique_ptr<DenseWork> w(new DenseWork());
    w->ctx = ctx;
    auto get = [&](size_t bytes) {
        void* p = ctx_alloc(ctx, bytes, s);
        w->bufs.push_back({p, bytes});
        return p;
    };
    w->M = static_cast<double*>(get(NN * sizeof(double)));
    w->X = static_cast<double*>(get(NN * sizeof(double)));
    w->D = static_cast<double*>(get((size_t)nb * kT * kT * sizeof(double)));
    w->flag = static_cast<int*>(get(sizeof(int)));
    return w;
}

// A_L^{-1} (FP64, n x n row-major) of the coarsest level from its device CSR,
// in the workspace w (from dense_work for this n).
void coarse_inverse_device(DenseWork& w, int n, const int* rp, const int* ci, const double* v, double* ainv,
                           hipStream_t s) {
    const int N = (n + kT - 1) / kT * kT;
    const int nb = N / kT;
    const size_t NN = (size_t)N * N;
    double* dM = w.M;
    double* dX = w.X;
    double* dD = w.D;
    int* dflag = w.flag;
    HIP_CHECK(hipMemsetAsync(dM, 0, NN * sizeof(double), s));
    HIP_CHECK(hipMemsetAsync(dX, 0, NN * sizeof(double), s));
    HIP_CHECK(hipMemsetAsync(dflag, 0, sizeof(int), s));
    const int rows_grid = (N + kDenseThreads - 1) / kDenseThreads;
    hipLaunchKernelGGL(k_dense_scatter, dim3(rows_grid), dim3(kDenseThreads), 0, s, n, N, rp, ci, v, dM);
    hipLaunchKernelGGL(k_dense_eye, dim3(rows_grid), dim3(kDenseThreads), 0, s, N, dX);
    for (int kb = 0; kb < nb; ++kb) {
        hipLaunchKernelGGL(k_dense_potrf_tile, dim3(1), dim3(kDenseThreads), 0, s, dM, N, kb, dD, dflag);
        const int t = nb - kb - 1;
        if (t > 0) {
            hipLaunchKernelGGL(k_dense_panel, dim3(t), dim3(kDenseThreads), 0, s, dM, N, kb, (const double*)dD);
            hipLaunchKernelGGL(k_dense_syrk, dim3((unsigned)((long long)t * (t + 1) / 2)), dim3(kDenseThreads), 0,
                               s, dM, N, kb);
        }
    }
    HIP_CHECK(hipGetLastError());
    int bad = 0;
    HIP_CHECK(hipMemcpyAsync(&bad, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_CHECK(hipStreamSynchronize(s));
    if (bad) throw Error(PAMG_E_NOT_SPD, "coarsest matrix is not positive definite");
    for (int ib = 0; ib < nb; ++ib) {
        hipLaunchKernelGGL(k_dense_trmm, dim3(ib + 1), dim3(kDenseThreads), 0, s, dX, N, ib, (const double*)dD);
        if (ib + 1 < nb)
            hipLaunchKernelGGL(k_dense_fwd_update, dim3((unsigned)((long long)(nb - 1 - ib) * (ib + 1))),
                               dim3(kDenseThreads), 0, s, dX, (const double*)dM, N, ib);
    }
    hipLaunchKernelGGL(k_dense_xtx, dim3((unsigned)((long long)nb * (nb + 1) / 2)), dim3(kDenseThreads), 0, s,
                       (const double*)dX, N, nb, n, ainv);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipStreamSynchronize(s));
}

}  // namespace pamg

// Low-rank factors K ~= U V of a coagulation kernel that has no exact
// low-rank form, such as the free-molecular kernel of Sec. 3.1, so that the
// O(M R log M) right-hand side applies to it.  Method: adaptive cross
// approximation with partial pivoting (Bebendorf, Numer. Math. 86 (2000);
// Bebendorf and Rjasanow, Computing 70 (2003)): rank-one terms built from one
// residual row and one residual column of K per step, entries evaluated on
// demand (the M x M matrix is never formed), stopped at the first term whose
// Frobenius norm is at most tol times that of the approximation (the norm
// kept up to date from the terms' inner products); that term is not kept.
#include "host.h"

#define ACA_NT 256                 // one workgroup, one wave per SIMD
#define ACA_WAVES (ACA_NT / 64)
#define ACA_NQ (SMOL_MAX_R + 1)  // inner products gathered per pass

// K_ij for 1-based sizes i, j (as doubles).
__device__ inline double kernel_value(int kind, double p0, double p1, double i, double j)
{
    switch (kind) {
    case SMOL_KERNEL_CONSTANT: return p0;
    case SMOL_KERNEL_BROWNIAN: return pow(i / j, p0) + pow(j / i, p0) + p1;
    default: {  // SMOL_KERNEL_FREE_MOLECULAR
        const double c = cbrt(i) + cbrt(j);
        return c * c * sqrt(1.0 / i + 1.0 / j);
    }
    }
}

// Block-wide sums of q[0..nq) (wave butterflies, then waves in order): every
// thread receives the totals in tot.
__device__ inline void aca_sums(double *q, int nq, double (*shw)[ACA_NQ], double *tot)
{
    const int lane = lane_id(), w = wave_id();
#pragma unroll
    for (int k = 0; k < ACA_NQ; ++k)
        if (k < nq) q[k] = wave_sum(q[k]);
    if (lane == 0)
        for (int k = 0; k < nq; ++k) shw[w][k] = q[k];
    __syncthreads();
    if (threadIdx.x < nq) {
        double a = 0.0;
        for (int v = 0; v < ACA_WAVES; ++v) a += shw[v][threadIdx.x];
        tot[threadIdx.x] = a;
    }
    __syncthreads();
}

// Block-wide argmax of (val, idx), ties to the smaller index.
__device__ inline int64_t aca_argmax(double val, int64_t idx, double *shv, int64_t *shi)
{
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(val, off, 64);
        const int64_t oi = __shfl_xor(idx, off, 64);
        if (ov > val || (ov == val && oi < idx)) {
            val = ov;
            idx = oi;
        }
    }
    const int lane = lane_id(), w = wave_id();
    if (lane == 0) {
        shv[w] = val;
        shi[w] = idx;
    }
    __syncthreads();
    double bv = shv[0];
    int64_t bi = shi[0];
    for (int v = 1; v < ACA_WAVES; ++v)
        if (shv[v] > bv || (shv[v] == bv && shi[v] < bi)) {
            bv = shv[v];
            bi = shi[v];
        }
    __syncthreads();
    return bi;
}

// The whole approximation in one workgroup.  Term k: residual row ip,
// r_j = K(ip, j) - sum_{l<k} U[l][ip] V[l][j], column pivot jp = argmax |r_j|
// over unused columns, v_k = r / r_jp; residual column
// u_k(i) = K(i, jp) - sum_{l<k} U[l][i] V[l][jp]; next row pivot argmax |u_k|
// over unused rows.  The inner products V[l].v_k and U[l].u_k that update
// ||U V||_F^2 are accumulated in the same passes.  out: rank, estimate.
__global__ __launch_bounds__(ACA_NT) void k_aca(int64_t M, int kind, double p0, double p1,
                                                double tol, int rmax, double *U, double *V,
                                                double *out)
{
    __shared__ double shw[ACA_WAVES][ACA_NQ];
    __shared__ double tot[ACA_NQ];
    __shared__ double coef[SMOL_MAX_R];
    __shared__ int64_t rows[SMOL_MAX_R], cols[SMOL_MAX_R];
    __shared__ double shv[ACA_WAVES];
    __shared__ int64_t shi[ACA_WAVES];
    const int tid = threadIdx.x;
    int64_t ip = 0;
    double nrm2 = 0.0, est = INFINITY;
    int rank = 0;
    for (int k = 0; k < rmax; ++k) {
        if (tid < k) coef[tid] = U[(int64_t)tid * M + ip];
        if (tid == 0) rows[k] = ip;
        __syncthreads();
        // residual row ip into V[k]; V[l].r and r.r on the way
        double q[ACA_NQ];
#pragma unroll
        for (int l = 0; l < ACA_NQ; ++l) q[l] = 0.0;
        double bv = -1.0;
        int64_t bi = M;
        const double x = (double)(ip + 1);
        for (int64_t j = tid; j < M; j += ACA_NT) {
            double r = kernel_value(kind, p0, p1, x, (double)(j + 1));
            double vl[SMOL_MAX_R];
#pragma unroll
            for (int l = 0; l < SMOL_MAX_R; ++l)
                if (l < k) {
                    vl[l] = V[(int64_t)l * M + j];
                    r = fma(-coef[l], vl[l], r);
                }
#pragma unroll
            for (int l = 0; l < SMOL_MAX_R; ++l)
                if (l < k) q[l] = fma(vl[l], r, q[l]);
            q[SMOL_MAX_R] = fma(r, r, q[SMOL_MAX_R]);
            V[(int64_t)k * M + j] = r;
            bool used = false;
            for (int l = 0; l < k; ++l) used = used || cols[l] == j;
            const double a = used ? -1.0 : fabs(r);
            if (a > bv) {
                bv = a;
                bi = j;
            }
        }
        const int64_t jp = aca_argmax(bv, bi, shv, shi);  // barriers make V[k] visible
        const double delta = jp < M ? V[(int64_t)k * M + jp] : 0.0;
        if (!(fabs(delta) > 0.0) || !isfinite(delta)) break;  // residual row vanished
        // sums over the row: V[l].v = (V[l].r) / delta, v.v = (r.r) / delta^2
        aca_sums(q, ACA_NQ, shw, tot);
        double vdot[SMOL_MAX_R + 1];
#pragma unroll
        for (int l = 0; l <= SMOL_MAX_R; ++l) vdot[l] = tot[l];
        const double inv = 1.0 / delta;
        for (int64_t j = tid; j < M; j += ACA_NT) V[(int64_t)k * M + j] *= inv;
        if (tid < k) coef[tid] = V[(int64_t)tid * M + jp];
        if (tid == 0) cols[k] = jp;
        __syncthreads();
        // residual column jp into U[k]; U[l].u and u.u on the way
#pragma unroll
        for (int l = 0; l < ACA_NQ; ++l) q[l] = 0.0;
        bv = -1.0;
        bi = M;
        const double y = (double)(jp + 1);
        for (int64_t i = tid; i < M; i += ACA_NT) {
            double c = kernel_value(kind, p0, p1, (double)(i + 1), y);
            double ul[SMOL_MAX_R];
#pragma unroll
            for (int l = 0; l < SMOL_MAX_R; ++l)
                if (l < k) {
                    ul[l] = U[(int64_t)l * M + i];
                    c = fma(-ul[l], coef[l], c);
                }
#pragma unroll
            for (int l = 0; l < SMOL_MAX_R; ++l)
                if (l < k) q[l] = fma(ul[l], c, q[l]);
            q[SMOL_MAX_R] = fma(c, c, q[SMOL_MAX_R]);
            U[(int64_t)k * M + i] = c;
            bool used = false;
            for (int l = 0; l <= k; ++l) used = used || rows[l] == i;
            const double a = used ? -1.0 : fabs(c);
            if (a > bv) {
                bv = a;
                bi = i;
            }
        }
        aca_sums(q, ACA_NQ, shw, tot);
        const int64_t inext = aca_argmax(bv, bi, shv, shi);
        // ||U V||_F^2 after adding u_k v_k
        const double vv = vdot[SMOL_MAX_R] * inv * inv, uu = tot[SMOL_MAX_R];
        double cross = 0.0;
        for (int l = 0; l < k; ++l) cross = fma(tot[l], vdot[l] * inv, cross);
        nrm2 += 2.0 * cross + uu * vv;
        est = sqrt(uu * vv) / sqrt(nrm2);
        if (!(est > tol) && k > 0) break;  // the newest term is below tol: not kept
        rank = k + 1;
        if (inext >= M) break;
        ip = inext;
    }
    if (tid == 0) {
        out[0] = (double)rank;
        out[1] = est;
    }
}

extern "C" int smol_lowrank(int64_t M, int32_t kernel, double p0, double p1, double tol,
                            int32_t max_rank, double *U, double *V, int32_t *rank, double *est,
                            void *stream)
{
    if (M < 1 || !U || !V || !rank || U == V) return SMOL_EINVAL;
    if (kernel < SMOL_KERNEL_CONSTANT || kernel > SMOL_KERNEL_FREE_MOLECULAR) return SMOL_EINVAL;
    if (max_rank < 1 || max_rank > SMOL_MAX_R || !(tol >= 0.0) || !std::isfinite(p0) ||
        !std::isfinite(p1))
        return SMOL_EINVAL;
    if (2 * M - 2 > (1LL << SMOL_LOG_LMAX)) return SMOL_EUNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    double *dout = nullptr;
    if (hipMalloc(&dout, 2 * sizeof(double)) != hipSuccess) return SMOL_ENOMEM;
    double hout[2] = {0.0, 0.0};
    hipLaunchKernelGGL(k_aca, dim3(1), dim3(ACA_NT), 0, s, M, (int)kernel, p0, p1, tol,
                       (int)max_rank, U, V, dout);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(hout, dout, sizeof(hout), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dout);
    if (e != hipSuccess) return hip_fail(e, "smol_lowrank");
    *rank = (int32_t)hout[0];
    if (est) *est = hout[1];
    return SMOL_OK;
}

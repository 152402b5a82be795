// fd_naive.hip -- untiled reference kernels and small helper kernels.
//
// The untiled step is the plain one-thread-per-point form of the paper's
// "normal" stencil (Sec. 6.3.1 / Sec. 6.5 transformation types): every
// neighbour is read from memory.  It fixes the per-point FP32 operation order
// that every other kernel variant reproduces bit for bit:
//   lap = 0
//   for k = 1..M: lap = fma(wx_k, fma(-2, u_c, u(x-k)+u(x+k)), lap)
//                 lap = fma(wy_k, fma(-2, u_c, u(y-k)+u(y+k)), lap)
//                 lap = fma(wz_k, fma(-2, u_c, u(z-k)+u(z+k)), lap)
// (the centre weight c_0 = -2 sum_k c_k is folded into the pairs, so a constant
// field gives exactly zero and no rounded centre weight biases the sweep);
// on isotropic grids (all present axes share their FP32 weights) the form is
//   for k = 1..M: lap = fma(w_k, fma(cc, u_c, ((sx + sy) + sz)), lap),  cc = -2 d,
// with s_a = u(-k e_a) + u(+k e_a) (an absent axis contributes +0).
//   eta = q * (px[x] + (py[y] + pz[z]))
//   num = fma(q, lap, fma(eta - 1, u_prev, 2 u_c))
//   u_new = (eta != 0) ? num * rcp(1 + eta) : num       (damped(): hardware reciprocal)
// then, per source entry at the point in table order: u_new = fma(scale, w, u_new).
#include "fd_internal.h"

namespace fdw {

template <int M, bool ISO>
__global__ __launch_bounds__(256) void k_naive_step(SweepArgs a)
{
    const int z = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const int x = blockIdx.z;
    if (z >= a.nz || y >= a.ny) return;
    const float *u = a.u0;
    const int64_t c = (int64_t)x * a.sxy + (int64_t)y * a.nzp + z;
    const float uc = u[c];
    float lap = 0.0f;
#pragma unroll
    for (int k = 1; k <= M; ++k) {
        const float xm = (x - k >= 0) ? u[c - k * a.sxy] : 0.0f;
        const float xp = (x + k < a.nx) ? u[c + k * a.sxy] : 0.0f;
        const float ym = (y - k >= 0) ? u[c - (int64_t)k * a.nzp] : 0.0f;
        const float yp = (y + k < a.ny) ? u[c + (int64_t)k * a.nzp] : 0.0f;
        const float zm = (z - k >= 0) ? u[c - k] : 0.0f;
        const float zp = (z + k < a.nz) ? u[c + k] : 0.0f;
        if constexpr (ISO) {
            const float s = ((xm + xp) + (ym + yp)) + (zm + zp);
            lap = fmaf(a.w.wx[k - 1], fmaf(a.w.cc, uc, s), lap);
        } else {
            lap = fmaf(a.w.wx[k - 1], fmaf(-2.0f, uc, xm + xp), lap);
            lap = fmaf(a.w.wy[k - 1], fmaf(-2.0f, uc, ym + yp), lap);
            lap = fmaf(a.w.wz[k - 1], fmaf(-2.0f, uc, zm + zp), lap);
        }
    }
    const float qv = a.q[c];
    const float eta = qv * (a.px[x] + (a.py[y] + a.pz[z]));
    float num = fmaf(qv, lap, fmaf(eta - 1.0f, a.um[c], 2.0f * uc));
    if (a.bs) num = fmaf(a.bs[c], a.d2[a.dslot0 * (int64_t)a.nx * a.sxy + c], num);  // Born source
    a.o1[c] = damped(num, eta);
}

hipError_t launch_naive_step(int M, const SweepArgs &a, hipStream_t s)
{
    dim3 block(64, 4, 1);
    dim3 grid((a.nz + 63) / 64, (a.ny + 3) / 4, a.nx);
#define FDW_NAIVE(MM)                                                                      \
    case MM:                                                                               \
        if (a.w.iso) hipLaunchKernelGGL((k_naive_step<MM, true>), grid, block, 0, s, a);     \
        else hipLaunchKernelGGL((k_naive_step<MM, false>), grid, block, 0, s, a);            \
        break;
    switch (M) {
        FDW_NAIVE(1)
        FDW_NAIVE(2)
        FDW_NAIVE(3)
        FDW_NAIVE(4)
        FDW_NAIVE(5)
        FDW_NAIVE(6)
        FDW_NAIVE(7)
        FDW_NAIVE(8)
    default: return hipErrorInvalidValue;
    }
#undef FDW_NAIVE
    return hipGetLastError();
}

// One thread per table entry; the first entry of each run of equal grid nodes
// applies the whole run in table order, so repeated points are deterministic.
__global__ void k_inject(PointTable t, int64_t sxy, const float *amp, int64_t row, float *field)
{
    const int32_t *xe = t.xe;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= t.cnt) return;
    if (j > 0 && xe[j - 1] == xe[j] && t.yz[j - 1] == t.yz[j]) return;
    const int64_t p = (int64_t)xe[j] * sxy + t.yz[j];
    float val = field[p];
    for (int k = j; k < t.cnt && xe[k] == xe[j] && t.yz[k] == t.yz[j]; ++k)
        val = fmaf(t.scale[k], amp[row * t.stride + t.id[k]], val);
    field[p] = val;
}

__global__ void k_record(PointTable t, int64_t sxy, const float *field, float *out, int64_t row,
                         float rscale)
{
    const int32_t *xe = t.xe;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= t.cnt) return;
    const int64_t p = (int64_t)xe[j] * sxy + t.yz[j];
    if (t.etr) t.etr[row * t.cnt + j] = field[p];  // summed per point after the sweep
    else out[row * t.stride + t.id[j]] = field[p] * rscale;
}

__global__ void k_gather(const float *etr, int64_t rows, int cnt, const int32_t *pptr,
                         const int32_t *pent, const float *wt, int npts, float *out, float rscale)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= rows * npts) return;
    const int64_t row = i / npts;
    const int p = (int)(i - row * npts);
    // FP64 accumulation, one rounding at the end: a windowed-sinc point sums
    // up to 4096 products of alternating sign, several times larger than the
    // result, which an FP32 sum would round at every term
    double acc = 0.0;
    for (int k = pptr[p]; k < pptr[p + 1]; ++k)
        acc = fma((double)wt[pent[k]], (double)etr[row * cnt + pent[k]], acc);
    out[i] = (float)(acc * (double)rscale);
}

hipError_t launch_gather(const float *etr, int64_t rows, int cnt, const int32_t *pptr,
                         const int32_t *pent, const float *wt, int npts, float *out, float rscale,
                         hipStream_t s)
{
    const int64_t n = rows * npts;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, etr, rows, cnt,
                       pptr, pent, wt, npts, out, rscale);
    return hipGetLastError();
}

// The x coordinate of every entry is recovered from the CSR row pointers.
__global__ void k_entry_x(const int32_t *xptr, int nx, int32_t *xe)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    for (int j = xptr[x]; j < xptr[x + 1]; ++j) xe[j] = x;
}

hipError_t launch_entry_x(const PointTable &t, int nx, int32_t *xe, hipStream_t s)
{
    if (t.cnt == 0) return hipSuccess;
    hipLaunchKernelGGL(k_entry_x, dim3((nx + 255) / 256), dim3(256), 0, s, t.xptr, nx, xe);
    return hipGetLastError();
}

hipError_t launch_inject(const SweepArgs &a, float *field, int step, hipStream_t s)
{
    if (a.inj.cnt == 0) return hipSuccess;
    const int64_t row = a.abase + (int64_t)a.adir * step;
    hipLaunchKernelGGL(k_inject, dim3((a.inj.cnt + 63) / 64), dim3(64), 0, s, a.inj, a.sxy, a.amp,
                       row, field);
    return hipGetLastError();
}

hipError_t launch_record(const SweepArgs &a, const float *field, int step, hipStream_t s)
{
    if (a.rec.cnt == 0) return hipSuccess;
    const int64_t row = a.rbase + (int64_t)a.rdir * step;
    hipLaunchKernelGGL(k_record, dim3((a.rec.cnt + 63) / 64), dim3(64), 0, s, a.rec, a.sxy, field,
                       a.rec_out, row, a.rscale);
    return hipGetLastError();
}

__global__ void k_save_d2(const float *unew, const float *ucur, const float *uprev, float *d2,
                          int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        d2[i] = fmaf(-2.0f, ucur[i], unew[i]) + uprev[i];
}

hipError_t launch_save_d2(const SweepArgs &a, const float *unew, const float *ucur,
                          const float *uprev, float *d2, hipStream_t s)
{
    const int64_t n = (int64_t)a.nx * a.sxy;
    hipLaunchKernelGGL(k_save_d2, dim3(4096), dim3(256), 0, s, unew, ucur, uprev, d2, n);
    return hipGetLastError();
}

__global__ void k_imaging(const float *lam, const float *d2, float *g, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        g[i] = fmaf(lam[i], d2[i], g[i]);
}

hipError_t launch_imaging(const SweepArgs &a, const float *lam, const float *d2, float *g,
                          hipStream_t s)
{
    const int64_t n = (int64_t)a.nx * a.sxy;
    hipLaunchKernelGGL(k_imaging, dim3(4096), dim3(256), 0, s, lam, d2, g, n);
    return hipGetLastError();
}

__global__ void k_flush_image(float *part, double *g, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        g[i] += (double)part[i];
        part[i] = 0.0f;
    }
}

hipError_t launch_flush_image(float *part, double *g, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_flush_image, dim3(4096), dim3(256), 0, s, part, g, n);
    return hipGetLastError();
}

__global__ void k_make_q(const float *v, float *q, int64_t rows, int nz, int nzp, double dt2)
{
    const int64_t n = rows * nzp;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / nzp;
        const int z = (int)(i - r * nzp);
        float qv = 0.0f;
        if (z < nz) {
            const double vv = (double)v[r * nz + z];
            qv = (float)(vv * vv * dt2);
        }
        q[i] = qv;
    }
}

hipError_t launch_make_q(const float *v, float *q, int64_t rows, int nz, int nzp, double dt2,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_make_q, dim3(4096), dim3(256), 0, s, v, q, rows, nz, nzp, dt2);
    return hipGetLastError();
}

// Born scattering coefficient s = 2 dv / v (FP64, rounded once), padded rows.
__global__ void k_born_coef(const float *v, const float *dv, float *s, int64_t rows, int nz,
                            int nzp)
{
    const int64_t n = rows * nzp;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / nzp;
        const int z = (int)(i - r * nzp);
        const int64_t j = r * nz + z;
        s[i] = (z < nz) ? (float)(2.0 * (double)dv[j] / (double)v[j]) : 0.0f;
    }
}

hipError_t launch_born_coef(const float *v, const float *dv, float *s, int64_t rows, int nz, int nzp,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_born_coef, dim3(4096), dim3(256), 0, st, v, dv, s, rows, nz, nzp);
    return hipGetLastError();
}

__global__ void k_repitch(float *dst, int dpitch, const float *src, int spitch, int64_t rows,
                          int nz)
{
    const int64_t n = rows * dpitch;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / dpitch;
        const int z = (int)(i - r * dpitch);
        dst[i] = (z < nz) ? src[r * spitch + z] : 0.0f;
    }
}

hipError_t launch_repitch(float *dst, int dpitch, const float *src, int spitch, int64_t rows,
                          int nz, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_repitch, dim3(4096), dim3(256), 0, s, dst, dpitch, src, spitch, rows, nz);
    return hipGetLastError();
}

// Per-block (max v, min v, count of non-finite or non-positive v).
__global__ __launch_bounds__(256) void k_vstats(const float *v, int64_t n, float *partial)
{
    __shared__ float smax[256], smin[256], sbad[256];
    float mx = 0.0f, mn = 3.0e38f, bad = 0.0f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float x = v[i];
        if (!(x > 0.0f) || !(x < 3.0e38f)) bad += 1.0f;
        else {
            mx = fmaxf(mx, x);
            mn = fminf(mn, x);
        }
    }
    smax[threadIdx.x] = mx;
    smin[threadIdx.x] = mn;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + o]);
            smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + o]);
            sbad[threadIdx.x] += sbad[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x + 0] = smax[0];
        partial[3 * blockIdx.x + 1] = smin[0];
        partial[3 * blockIdx.x + 2] = sbad[0];
    }
}

hipError_t launch_vstats(const float *v, int64_t n, float *partial, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_vstats, dim3(nb), dim3(256), 0, s, v, n, partial);
    return hipGetLastError();
}

// Injection scale alpha * w * q / (1 + eta) at each entry's node (w its interpolation
// weight, 1 on grid nodes; same eta as the update).
__global__ void k_scales(SweepArgs a, PointTable t, float *scale, float alpha)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= t.cnt) return;
    const int x = t.xe[j];
    const int y = t.yz[j] / a.nzp;
    const int z = t.yz[j] - y * a.nzp;
    const float qv = a.q[(int64_t)x * a.sxy + t.yz[j]];
    const float eta = qv * (a.px[x] + (a.py[y] + a.pz[z]));
    scale[j] = (alpha * t.wt[j]) * damped(qv, eta);
}

hipError_t launch_scales(const SweepArgs &a, const PointTable &t, float *scale, float alpha,
                         hipStream_t s)
{
    if (t.cnt == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scales, dim3((t.cnt + 63) / 64), dim3(64), 0, s, a, t, scale, alpha);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_residual(const float *d, const float *dobs, float *res,
                                                  int64_t n, double *partial)
{
    __shared__ double sj[256];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double r = (double)d[i] - (double)dobs[i];
        res[i] = (float)r;
        acc += 0.5 * r * r;
    }
    sj[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sj[threadIdx.x] += sj[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sj[0];
}

hipError_t launch_residual(const float *d, const float *dobs, float *res, int64_t n,
                           double *partial, int nb, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual, dim3(nb), dim3(256), 0, s, d, dobs, res, n, partial);
    return hipGetLastError();
}

// grad_v = dJ/dm * (-2 / v^3) with dJ/dm = -2 g  ->  4 g / v^3, evaluated in FP64
// (g in the padded internal layout, v and grad_v dense).
__global__ void k_grad_v(const double *g, const float *v, float *gv, int64_t rows, int nz, int nzp)
{
    const int64_t n = rows * nz;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / nz;
        const int z = (int)(i - r * nz);
        const double vv = (double)v[i];
        gv[i] = (float)(4.0 * g[r * nzp + z] / (vv * vv * vv));
    }
}

hipError_t launch_grad_v(const double *g, const float *v, float *grad_v, int64_t rows, int nz,
                         int nzp, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad_v, dim3(4096), dim3(256), 0, s, g, v, grad_v, rows, nz, nzp);
    return hipGetLastError();
}

// Plain fill kernel (also safe inside captured graphs, unlike memset nodes).
__global__ void k_zero(uint32_t *p, int64_t nwords)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nwords;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_zero(void *p, int64_t bytes, hipStream_t s)
{
    if (bytes <= 0) return hipSuccess;
    if (bytes % 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero, dim3(2048), dim3(256), 0, s, (uint32_t *)p, bytes / 4);
    return hipGetLastError();
}

__global__ void k_copy(float *dst, const float *src, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_copy(float *dst, const float *src, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(4096), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

}  // namespace fdw

// Reverse-mode kernels of libdtvdd.so: the adjoint of the unrolled solve of
// Algorithm 1 (Lee & Park, arXiv 1901.00682, Sec. 4) with FISTA local steps,
// with respect to the image f and the weight alpha.
//
// The backward step has the work decomposition of the streaming forward step
// (one wave per 63 columns x R rows, lane 0 a halo column, rows swept top to
// bottom): the linear part of a FISTA step, a_keep y - kL div_s^* div_s y, is
// self-adjoint, so the reverse step is the same stencil applied to
// zbar = xbar * 1{|z| < 1}.  Gradients accumulate in FP32 edge and pixel
// arrays; the alpha derivative accumulates in FP64 per work item and is
// reduced in a fixed order.
#include "bwd.h"
#include "dtvdd_internal.h"
#include "fista_ops.h"

namespace dtv {

__device__ __forceinline__ double wave_sum_d(double x)
{
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

template <int R, bool MOM>
__global__ __launch_bounds__(64) void k_fista_bwd_step(FistaBwdArgs a)
{
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const StreamTile tile = a.tiles[t];
    const ImgDev im = a.imgs[tile.img];
    const int lane = threadIdx.x;
    const int H = im.H, W = im.W;
    const int j = tile.j0 - 1 + lane;
    const bool colok = (j >= 0) && (j < W);
    const int cw = colok ? a.info[im.cinfo + j] : 0;
    const int cs = info_sub(cw);
    const bool cfirst = info_first(cw), clast = info_last(cw);
    const int left = j + cs;
    const bool outlane = colok && lane >= 1;
    const long long P1 = im.pitch1, P2 = im.pitch2;

    const float *z1 = a.z1 + im.p1, *z2 = a.z2 + im.p2;
    const float *xa1 = a.xa1 + im.p1, *xa2 = a.xa2 + im.p2;
    const float *xb1 = MOM ? a.xb1 + im.p1 : nullptr, *xb2 = MOM ? a.xb2 + im.p2 : nullptr;
    const float *b1 = a.base1 + im.p1, *b2 = a.base2 + im.p2;
    const float *lam = a.lam + im.lam;
    const float *f = a.f + im.px;
    const float *gx1 = a.gx1 + im.p1, *gx2 = a.gx2 + im.p2;
    float *ga1 = a.ga1 + im.p1, *ga2 = a.ga2 + im.p2;
    float *gb1 = MOM ? a.gb1 + im.p1 : nullptr, *gb2 = MOM ? a.gb2 + im.p2 : nullptr;
    float *gh1 = a.gh1 + im.p1, *gh2 = a.gh2 + im.p2;
    float *gf = a.gf + im.px;
    const float beta = a.beta, tau = a.tau, itau = a.inv_tau;
    const float ak = im.a_keep, kL = im.kL, invL = im.invL;
    const float hL = invL * itau;  // 1/(L tau)
    const double dA = im.dA, dB = im.dB;
    const double ditau = (double)itau;

    auto zb1 = [&](long long idx) -> float { return fabsf(z1[idx]) < 1.0f ? gx1[idx] : 0.0f; };
    auto zb2 = [&](long long idx) -> float { return fabsf(z2[idx]) < 1.0f ? gx2[idx] : 0.0f; };
    auto y1 = [&](long long idx) -> float {
        if constexpr (MOM) return fista_y(xa1[idx], xb1[idx], beta);
        return xa1[idx];
    };
    auto y2 = [&](long long idx) -> float {
        if constexpr (MOM) return fista_y(xa2[idx], xb2[idx], beta);
        return xa2[idx];
    };
    // distribute ybar on one edge to the adjoints of x_{k-1}, x_{k-2}
    auto push1 = [&](long long idx, float yb) {
        if constexpr (MOM) {
            ga1[idx] = fmaf(1.0f + beta, yb, ga1[idx]);
            gb1[idx] = fmaf(-beta, yb, gb1[idx]);
        } else {
            ga1[idx] += yb;
        }
    };
    auto push2 = [&](long long idx, float yb) {
        if constexpr (MOM) {
            ga2[idx] = fmaf(1.0f + beta, yb, ga2[idx]);
            gb2[idx] = fmaf(-beta, yb, gb2[idx]);
        } else {
            ga2[idx] += yb;
        }
    };

    double acc = 0.0;
    const int i0 = tile.i0;
    const int iend = min(i0 + R, H);
    float dz_up = 0.0f, z_carry = 0.0f, y_carry = 0.0f;
    bool have = false;
    if (i0 > 0 && !info_first(a.info[im.rinfo + i0])) {
        const int i = i0 - 1;
        const int top = i + info_sub(a.info[im.rinfo + i]);
        if (colok) {
            const float zt = zb1(top * P1 + j), zb = zb1((top + 1) * P1 + j);
            dz_up = div4(zt, zb, zb2(i * P2 + left), zb2(i * P2 + left + 1));
            z_carry = zb;
            y_carry = y1((top + 1) * P1 + j);
        }
        have = true;
    }
    for (int i = i0; i < iend; ++i) {
        const int rw = a.info[im.rinfo + i];
        const int rs = info_sub(rw);
        const bool rfirst = info_first(rw), rlast = info_last(rw);
        const long long top = i + rs;
        if (rfirst) {
            have = false;
            dz_up = 0.0f;
        }
        float dz = 0.0f, zt = 0.0f, zbm = 0.0f, zl = 0.0f, zr = 0.0f;
        float yt = 0.0f, yb = 0.0f, yl = 0.0f, yr = 0.0f;
        if (colok) {
            zt = have ? z_carry : zb1(top * P1 + j);
            zbm = zb1((top + 1) * P1 + j);
            zl = zb2(i * P2 + left);
            zr = zb2(i * P2 + left + 1);
            dz = div4(zt, zbm, zl, zr);
            yt = have ? y_carry : y1(top * P1 + j);
            yb = y1((top + 1) * P1 + j);
            yl = y2(i * P2 + left);
            yr = y2(i * P2 + left + 1);
        }
        float dz_left = __shfl_up(dz, 1, 64);
        if (cfirst) dz_left = 0.0f;
        if (outlane) {
            const long long px = (long long)i * W + j;
            const float fv = f[px];
            const float dy = div4(yt, yb, yl, yr);
            gf[px] = fmaf(-invL, dz, gf[px]);
            acc += -dA * ((double)fv * dz) - dB * ((double)dz * dy);
            if (i > 0) {
                float anchor = b1[top * P1 + j];
                if (rfirst) anchor = fmaf(tau, lam[(long long)(rs - 1) * W + j], anchor);
                push1(top * P1 + j, fmaf(-kL, dz_up - dz, ak * zt));
                gh1[top * P1 + j] = fmaf(hL, zt, gh1[top * P1 + j]);
                acc += -dA * ditau * ((double)zt * ((double)yt - anchor));
            }
            if (j > 0) {
                float anchor = b2[i * P2 + left];
                if (cfirst) anchor = fmaf(tau, lam[im.nlh + (long long)(cs - 1) * H + i], anchor);
                push2(i * P2 + left, fmaf(-kL, dz_left - dz, ak * zl));
                gh2[i * P2 + left] = fmaf(hL, zl, gh2[i * P2 + left]);
                acc += -dA * ditau * ((double)zl * ((double)yl - anchor));
            }
            if (rlast && i < H - 1) {
                const float anchor = fmaf(-tau, lam[(long long)rs * W + j], b1[(top + 1) * P1 + j]);
                push1((top + 1) * P1 + j, fmaf(-kL, dz, ak * zbm));
                gh1[(top + 1) * P1 + j] = fmaf(hL, zbm, gh1[(top + 1) * P1 + j]);
                acc += -dA * ditau * ((double)zbm * ((double)yb - anchor));
            }
            if (clast && j < W - 1) {
                const float anchor = fmaf(-tau, lam[im.nlh + (long long)cs * H + i], b2[i * P2 + left + 1]);
                push2(i * P2 + left + 1, fmaf(-kL, dz, ak * zr));
                gh2[i * P2 + left + 1] = fmaf(hL, zr, gh2[i * P2 + left + 1]);
                acc += -dA * ditau * ((double)zr * ((double)yr - anchor));
            }
        }
        dz_up = dz;
        z_carry = zbm;
        y_carry = yb;
        have = true;
    }
    acc = wave_sum_d(acc);
    if (lane == 0) a.galpha[t] += acc;
}

template <int R>
static hipError_t bwd_rows(const FistaBwdArgs &a, bool mom, hipStream_t s)
{
    if (mom)
        hipLaunchKernelGGL((k_fista_bwd_step<R, true>), dim3(a.ntiles), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((k_fista_bwd_step<R, false>), dim3(a.ntiles), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fista_bwd_step(const FistaBwdArgs &a, bool momentum, int rows, hipStream_t s)
{
    if (a.ntiles <= 0) return hipSuccess;
    switch (rows) {
    case 4: return bwd_rows<4>(a, momentum, s);
    case 8: return bwd_rows<8>(a, momentum, s);
    case 16: return bwd_rows<16>(a, momentum, s);
    case 32: return bwd_rows<32>(a, momentum, s);
    default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------
// u = f + div_s p / alpha, reversed.  Work item t is the streaming tile
// (a 63-column x R-row strip); galpha[t] is indexed like the step kernels.
__global__ __launch_bounds__(64) void k_bwd_final_u(const ImgDev *imgs, const StreamTile *tiles, int rows,
                                                    const int *info, const float *p1, const float *p2,
                                                    const float *ubar, float *fbar, float *pb1, float *pb2,
                                                    double *galpha)
{
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const StreamTile tile = tiles[t];
    const ImgDev im = imgs[tile.img];
    const int lane = threadIdx.x;
    const int H = im.H, W = im.W;
    const int j = tile.j0 - 1 + lane;
    const bool colok = (j >= 0) && (j < W);
    const int cw = colok ? info[im.cinfo + j] : 0;
    const int cs = info_sub(cw);
    const bool cfirst = info_first(cw), clast = info_last(cw);
    const int left = j + cs;
    const bool outlane = colok && lane >= 1;
    const long long P1 = im.pitch1, P2 = im.pitch2;
    const float *q1 = p1 + im.p1, *q2 = p2 + im.p2;
    const float *ub = ubar + im.px;
    float *fb = fbar + im.px;
    float *o1 = pb1 + im.p1, *o2 = pb2 + im.p2;
    const float ia = im.inv_alpha;
    const double ia2 = 1.0 / ((double)im.alpha * (double)im.alpha);
    double acc = 0.0;
    const int i0 = tile.i0;
    const int iend = min(i0 + rows, H);
    float v_up = 0.0f;
    if (i0 > 0 && colok && !info_first(info[im.rinfo + i0])) v_up = ub[(long long)(i0 - 1) * W + j] * ia;
    for (int i = i0; i < iend; ++i) {
        const int rw = info[im.rinfo + i];
        const int rs = info_sub(rw);
        const bool rfirst = info_first(rw), rlast = info_last(rw);
        const long long top = i + rs;
        if (rfirst) v_up = 0.0f;
        float v = 0.0f;
        if (colok) v = ub[(long long)i * W + j] * ia;
        float v_left = __shfl_up(v, 1, 64);
        if (cfirst) v_left = 0.0f;
        if (outlane) {
            const long long px = (long long)i * W + j;
            const float u_b = ub[px];
            fb[px] = u_b;
            const float d = div4(q1[top * P1 + j], q1[(top + 1) * P1 + j], q2[i * P2 + left], q2[i * P2 + left + 1]);
            acc += -(double)u_b * d * ia2;
            if (i > 0) o1[top * P1 + j] = v_up - v;
            if (j > 0) o2[i * P2 + left] = v_left - v;
            if (rlast && i < H - 1) o1[(top + 1) * P1 + j] = v;
            if (clast && j < W - 1) o2[i * P2 + left + 1] = v;
        }
        v_up = v;
    }
    acc = wave_sum_d(acc);
    if (lane == 0) galpha[t] += acc;
}

hipError_t launch_bwd_final_u(const ImgDev *imgs, const StreamTile *tiles, int ntiles, int rows, const int *info,
                              const float *p1, const float *p2, const float *ubar, float *fbar, float *pb1,
                              float *pb2, double *galpha, hipStream_t s)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bwd_final_u, dim3(ntiles), dim3(64), 0, s, imgs, tiles, rows, info, p1, p2, ubar, fbar, pb1,
                       pb2, galpha);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_axpy_edges(const float *x, const float *y, float *out, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = x[i] + y[i];
}

hipError_t launch_axpy_edges(const float *x, const float *y, float *out, long long n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpy_edges, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, out, n);
    return hipGetLastError();
}

// per interface dof: adjoints of phat = p - tau B^* lambda^{n+1},
// prev^{n+1} = p^n on the copies and lambda^{n+1} = lambda^n + sigma B(2 p^n - prev^n)
__global__ __launch_bounds__(256) void k_bwd_interface(const ImgDev *imgs, const int *info, const float *hb1,
                                                       const float *hb2, float *pb1, float *pb2, float *lamb,
                                                       float tau, float sigma)
{
    const ImgDev im = imgs[blockIdx.y];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= im.nlam) return;
    long long is, it;
    const float *hb;
    float *pb;
    if (e < im.nlh) {
        const int r = e / im.W + 1, j = e - (r - 1) * im.W;
        const int cut = info[im.rcut + r];
        is = im.p1 + (long long)(cut + r - 1) * im.pitch1 + j;
        it = im.p1 + (long long)(cut + r) * im.pitch1 + j;
        hb = hb1;
        pb = pb1;
    } else {
        const int q = e - im.nlh;
        const int c = q / im.H + 1, i = q - (c - 1) * im.H;
        const int cut = info[im.ccut + c];
        is = im.p2 + (long long)i * im.pitch2 + cut + c - 1;
        it = im.p2 + (long long)i * im.pitch2 + cut + c;
        hb = hb2;
        pb = pb2;
    }
    float *L = lamb + im.lam;
    float lt = L[e], ds, dt;
    iface_bwd(hb[is], hb[it], tau, sigma, lt, L[im.nlam + e], L[2 * im.nlam + e], ds, dt);
    pb[is] += ds;
    pb[it] += dt;
    L[im.nlam + e] = -sigma * lt;
    L[2 * im.nlam + e] = sigma * lt;
    L[e] = lt;
}

hipError_t launch_bwd_interface(const ImgDev *imgs, int nimg, int max_nlam, const int *info, const float *hb1,
                                const float *hb2, float *pb1, float *pb2, float *lamb, float tau, float sigma,
                                hipStream_t s)
{
    if (max_nlam <= 0) return hipSuccess;
    dim3 grid((max_nlam + 255) / 256, nimg);
    hipLaunchKernelGGL(k_bwd_interface, grid, dim3(256), 0, s, imgs, info, hb1, hb2, pb1, pb2, lamb, tau, sigma);
    return hipGetLastError();
}

// alphabar per image from the per-tile (and per-subdomain) partial sums: one workgroup per
// image, each thread adds every 256th partial in order, then a fixed tree over the threads -- the
// same order in every run
constexpr int kReduceThreads = 256;

__device__ __forceinline__ float tree_sum(double *part, double acc)
{
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kReduceThreads / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    return (float)part[0];
}

__global__ __launch_bounds__(kReduceThreads) void k_alpha_reduce(const StreamTile *tiles, int ntiles,
                                                                 const double *galpha, float *out)
{
    __shared__ double part[kReduceThreads];
    const int img = blockIdx.x;
    double acc = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += kReduceThreads)
        if (tiles[t].img == img) acc += galpha[t];
    const float v = tree_sum(part, acc);
    if (threadIdx.x == 0) out[img] = v;
}

hipError_t launch_alpha_reduce(const StreamTile *tiles, int ntiles, int nimg, const double *galpha, float *out,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_alpha_reduce, dim3(nimg), dim3(kReduceThreads), 0, s, tiles, ntiles, galpha, out);
    return hipGetLastError();
}

// the same with the per-subdomain partial sums of the fused reverse steps added
__global__ __launch_bounds__(kReduceThreads) void k_alpha_reduce2(const StreamTile *tiles, int ntiles,
                                                                  const double *galpha, const SubTile *subs,
                                                                  int nsub, const double *gsub, float *out)
{
    __shared__ double part[kReduceThreads];
    const int img = blockIdx.x;
    double acc = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += kReduceThreads)
        if (tiles[t].img == img) acc += galpha[t];
    for (int t = threadIdx.x; t < nsub; t += kReduceThreads)
        if (subs[t].img == img) acc += gsub[t];
    const float v = tree_sum(part, acc);
    if (threadIdx.x == 0) out[img] = v;
}

hipError_t launch_alpha_reduce2(const StreamTile *tiles, int ntiles, const double *galpha, const SubTile *subs,
                                int nsub, const double *gsub, int nimg, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_alpha_reduce2, dim3(nimg), dim3(kReduceThreads), 0, s, tiles, ntiles, galpha, subs, nsub,
                       gsub, out);
    return hipGetLastError();
}

}  // namespace dtv

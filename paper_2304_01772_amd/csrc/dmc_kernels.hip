// Differentiable Monte Carlo (Methods, Algorithm 2) for the Ising model on
// gfx950: the relaxed checkerboard chain on continuous spins with one coupling
// per bond, and its reverse-mode gradient by replaying the chain backwards.
//
// One colour pass (colour c = (x + y) & 1, pass p = 2t + c) updates every
// site of colour c from the current spins:
//     hloc = Jx[y][x] s(y,x+1) + Jx[y][x-1] s(y,x-1) + Jy[y][x] s(y+1,x)
//            + Jy[y-1][x] s(y-1,x) + h
//     P = exp(-2 beta s hloc),  q = 1 / (1 + exp(-alpha (P - r))),
//     s <- s (1 - 2 q)          (the flip s' = -s mixed in with weight q)
// with r = (word >> 8) 2^-24 from Philox4x32-10 counter (k >> 2, p, rid, 3),
// word k & 3, k = y Lx/2 + (x >> 1).  A lane handles the four sites of one
// Philox block.  Spins and couplings are FP32, row-major [R][Ly][Lx].
//
// Backward of a pass, with a = dL/ds_new at a colour-c site and
// w = 4 alpha beta q (1 - q) P:
//     dL/ds_old = a ((1 - 2q) + w s_old hloc)
//     t = a w s_old^2  = dL/dhloc
//     dL/dJ(bond to n) += t s_n,   dL/ds_n += t J(bond to n)   (n of colour 1-c)
// Every bond has exactly one colour-c end, so the coupling gradients of a
// pass are written by one lane each; the neighbour terms are gathered by a
// second kernel from the per-site t.  The pre-pass spins of colour c are
// saved by the forward pass (one colour plane per pass), which is what the
// backward replay restores.
#include "dmc_internal.hpp"

namespace spinmc {

namespace {

constexpr uint32_t kTagDmc = 3u;

__device__ __forceinline__ int wrapd(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

struct DmcSite {
    int y, x;
    size_t i;  // natural index within the replica
};

__device__ __forceinline__ DmcSite dmc_site(int k, int W, int c) {
    DmcSite d;
    d.y = k / W;
    d.x = 2 * (k - d.y * W) + ((d.y + c) & 1);
    d.i = (size_t)d.y * (2 * W) + d.x;
    return d;
}

struct DmcLocal {
    float hloc, P, q;
    float sr, sl, sd, su;  // neighbour spins
};

__device__ __forceinline__ DmcLocal dmc_local(const float* s, const float* Jx, const float* Jy,
                                              int Lx, int Ly, int y, int x, float sv, float beta,
                                              float alpha, float h, uint32_t word) {
    DmcLocal L;
    const int xr = wrapd(x + 1, Lx), xl = wrapd(x - 1, Lx);
    const int yd = wrapd(y + 1, Ly), yu = wrapd(y - 1, Ly);
    const size_t row = (size_t)y * Lx;
    L.sr = s[row + xr];
    L.sl = s[row + xl];
    L.sd = s[(size_t)yd * Lx + x];
    L.su = s[(size_t)yu * Lx + x];
    L.hloc = Jx[row + x] * L.sr + Jx[row + xl] * L.sl + Jy[row + x] * L.sd +
             Jy[(size_t)yu * Lx + x] * L.su + h;
    L.P = expf(-beta * (2.0f * sv * L.hloc));
    const float r = (float)(word >> 8) * 0x1p-24f;
    L.q = 1.0f / (1.0f + expf(-alpha * (L.P - r)));
    return L;
}

}  // namespace

__global__ void __launch_bounds__(256) k_dmc_pass(DmcArgs a, int c, uint32_t p, float* save) {
    const int W = a.Lx >> 1;
    const int n_sites = a.Ly * W;
    const int n_blocks = (n_sites + 3) >> 2;
    const int r = blockIdx.y;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_blocks) return;
    const size_t off = (size_t)r * a.Lx * a.Ly;
    float* s = a.s + off;
    const float* Jx = a.Jx + off;
    const float* Jy = a.Jy + off;
    float* sv_save = save + (size_t)r * n_sites;
    uint32_t w[4];
    philox4x32_10((uint32_t)b, p, a.rid0 + (uint32_t)r, kTagDmc, a.key0, a.key1, w);
    // every load of the four sites first, then the stores (the buffers may
    // alias as far as the compiler knows); no two of a lane's sites share a
    // bond, since every bond has one end of each colour
    float snew[4], sold[4];
    size_t idx[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = 4 * b + u;
        idx[u] = 0;
        snew[u] = sold[u] = 0.f;
        if (k >= n_sites) continue;
        const DmcSite d = dmc_site(k, W, c);
        idx[u] = d.i;
        const float sv = s[d.i];
        const DmcLocal L = dmc_local(s, Jx, Jy, a.Lx, a.Ly, d.y, d.x, sv, a.beta, a.alpha, a.h,
                                     w[u]);
        sold[u] = sv;
        snew[u] = sv * (1.0f - 2.0f * L.q);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (4 * b + u < n_sites) {
            sv_save[4 * b + u] = sold[u];
            s[idx[u]] = snew[u];
        }
}

__global__ void __launch_bounds__(256) k_dmc_back(DmcArgs a, int c, uint32_t p,
                                                  const float* save, float* gs, float* gJx,
                                                  float* gJy, float* work) {
    const int W = a.Lx >> 1;
    const int n_sites = a.Ly * W;
    const int n_blocks = (n_sites + 3) >> 2;
    const int r = blockIdx.y;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_blocks) return;
    const size_t off = (size_t)r * a.Lx * a.Ly;
    float* s = a.s + off;
    const float* Jx = a.Jx + off;
    const float* Jy = a.Jy + off;
    float* g = gs + off;
    float* gx = gJx + off;
    float* gy = gJy + off;
    const float* sv_save = save + (size_t)r * n_sites;
    float* tw = work + (size_t)r * n_sites;
    uint32_t w[4];
    philox4x32_10((uint32_t)b, p, a.rid0 + (uint32_t)r, kTagDmc, a.key0, a.key1, w);
    // phase 1: every load of the four sites (including the coupling
    // gradients they add to); phase 2: every store
    float gout[4], tv[4], sold[4], gr[4], gl[4], gd[4], gu[4];
    float cr[4], cl[4], cd[4], cu[4];
    size_t ii[4], ir[4], il[4], idn[4], iu[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = 4 * b + u;
        gout[u] = tv[u] = sold[u] = gr[u] = gl[u] = gd[u] = gu[u] = 0.f;
        cr[u] = cl[u] = cd[u] = cu[u] = 0.f;
        ii[u] = ir[u] = il[u] = idn[u] = iu[u] = 0;
        if (k >= n_sites) continue;
        const DmcSite d = dmc_site(k, W, c);
        const float sv = sv_save[k];
        const DmcLocal L = dmc_local(s, Jx, Jy, a.Lx, a.Ly, d.y, d.x, sv, a.beta, a.alpha, a.h,
                                     w[u]);
        const float av = g[d.i];
        const float wq = 4.0f * a.alpha * a.beta * L.q * (1.0f - L.q) * L.P;
        gout[u] = av * ((1.0f - 2.0f * L.q) + wq * sv * L.hloc);
        const float t = av * wq * sv * sv;
        tv[u] = t;
        sold[u] = sv;
        const int xl = wrapd(d.x - 1, a.Lx), yu = wrapd(d.y - 1, a.Ly);
        const size_t row = (size_t)d.y * a.Lx;
        ii[u] = d.i;
        ir[u] = row + d.x;
        il[u] = row + xl;
        idn[u] = row + d.x;
        iu[u] = (size_t)yu * a.Lx + d.x;
        gr[u] = gx[ir[u]];
        gl[u] = gx[il[u]];
        gd[u] = gy[idn[u]];
        gu[u] = gy[iu[u]];
        cr[u] = t * L.sr;
        cl[u] = t * L.sl;
        cd[u] = t * L.sd;
        cu[u] = t * L.su;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = 4 * b + u;
        if (k >= n_sites) continue;
        g[ii[u]] = gout[u];
        tw[k] = tv[u];
        gx[ir[u]] = gr[u] + cr[u];
        gx[il[u]] = gl[u] + cl[u];
        gy[idn[u]] = gd[u] + cd[u];
        gy[iu[u]] = gu[u] + cu[u];
        s[ii[u]] = sold[u];  // the state before this pass
    }
}

// dL/ds_n += sum over the four colour-c neighbours i of t_i J(i, n), for the
// sites n of colour 1 - c.
__global__ void __launch_bounds__(256) k_dmc_gather(DmcArgs a, int c, float* gs,
                                                    const float* work) {
    const int W = a.Lx >> 1;
    const int n_sites = a.Ly * W;
    const int r = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_sites) return;
    const size_t off = (size_t)r * a.Lx * a.Ly;
    const float* Jx = a.Jx + off;
    const float* Jy = a.Jy + off;
    const float* tw = work + (size_t)r * n_sites;
    const DmcSite d = dmc_site(k, W, 1 - c);
    const int Lx = a.Lx, Ly = a.Ly;
    const int xr = wrapd(d.x + 1, Lx), xl = wrapd(d.x - 1, Lx);
    const int yd = wrapd(d.y + 1, Ly), yu = wrapd(d.y - 1, Ly);
    // within-colour index of a colour-c site (y', x'): y' W + (x' >> 1)
    const float tr = tw[d.y * W + (xr >> 1)], tl = tw[d.y * W + (xl >> 1)];
    const float td = tw[yd * W + (d.x >> 1)], tu = tw[yu * W + (d.x >> 1)];
    const size_t row = (size_t)d.y * Lx;
    const float acc = tr * Jx[row + d.x] + tl * Jx[row + xl] + td * Jy[row + d.x] +
                      tu * Jy[(size_t)yu * Lx + d.x];
    gs[off + d.i] += acc;
}

hipError_t launch_dmc_forward(const DmcArgs& a, uint64_t t0, int n_sweeps, float* save,
                              hipStream_t s) {
    const int n_sites = a.Ly * (a.Lx >> 1);
    const int n_blocks = (n_sites + 3) >> 2;
    const dim3 grid((n_blocks + 255) / 256, a.R), block(256);
    for (int i = 0; i < n_sweeps; ++i)
        for (int c = 0; c < 2; ++c) {
            const uint32_t p = (uint32_t)(2 * (t0 + (uint64_t)i) + (uint64_t)c);
            float* sv = save + (size_t)(2 * i + c) * a.R * n_sites;
            hipLaunchKernelGGL(k_dmc_pass, grid, block, 0, s, a, c, p, sv);
        }
    return hipGetLastError();
}

hipError_t launch_dmc_backward(const DmcArgs& a, uint64_t t0, int n_sweeps, const float* save,
                               float* gs, float* gJx, float* gJy, float* work, hipStream_t s) {
    const int n_sites = a.Ly * (a.Lx >> 1);
    const int n_blocks = (n_sites + 3) >> 2;
    const dim3 grid((n_blocks + 255) / 256, a.R), gridg((n_sites + 255) / 256, a.R), block(256);
    for (int i = n_sweeps - 1; i >= 0; --i)
        for (int c = 1; c >= 0; --c) {
            const uint32_t p = (uint32_t)(2 * (t0 + (uint64_t)i) + (uint64_t)c);
            const float* sv = save + (size_t)(2 * i + c) * a.R * n_sites;
            hipLaunchKernelGGL(k_dmc_back, grid, block, 0, s, a, c, p, sv, gs, gJx, gJy, work);
            hipLaunchKernelGGL(k_dmc_gather, gridg, block, 0, s, a, c, gs, work);
        }
    return hipGetLastError();
}

}  // namespace spinmc

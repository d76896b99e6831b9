// Differentiable Monte Carlo (Methods, Algorithm 2) for the Ising model on
// gfx950: the relaxed checkerboard chain on continuous spins with one coupling
// per bond, and its reverse-mode gradient by replaying the chain backwards.
//
// One colour pass (colour c = (x + y) & 1, pass p = 2t + c) updates every
// site of colour c from the current spins:
//     hloc = Jx[y][x] s(y,x+1) + Jx[y][x-1] s(y,x-1) + Jy[y][x] s(y+1,x)
//            + Jy[y-1][x] s(y-1,x) + h
//     P = exp(min(-2 beta s hloc, 80)),  q = 1 / (1 + exp(-alpha (P - r))),
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
// pass are written by one lane each.  The neighbour terms t J go to sites of
// the other colour, whose adjoints are only read again by the next pass of
// the replay: that pass adds them while it loads its own adjoint (the t of
// the previous pass is kept in a second plane of the work buffer), and one
// gather kernel adds those of the last pass.  The pre-pass spins of colour c
// are saved by the forward pass (one colour plane per pass), which is what
// the backward replay restores.
//
// Two layouts of the lane work: when Lx is a multiple of 8 (and every buffer
// is 16-byte aligned) the four sites of a Philox block are one 8-float span
// of a row, and a lane loads the spans of rows y-1, y, y+1 and of the
// couplings with 16-byte loads; otherwise every site is addressed on its own.
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

// the update of one site from its neighbourhood: local field, P and q
struct DmcUpd {
    float hloc, P, q;
};

__device__ __forceinline__ DmcUpd dmc_update(float sv, float jr, float sr, float jl, float sl,
                                             float jd, float sd, float ju, float su, float beta,
                                             float alpha, float h, uint32_t word) {
    DmcUpd U;
    U.hloc = jr * sr + jl * sl + jd * sd + ju * su + h;
    // exponent capped at 80: beyond it q is exactly 1 anyway, and an infinite
    // P would turn the backward's q (1 - q) P into 0 * inf
    U.P = expf(fminf(-beta * (2.0f * sv * U.hloc), 80.0f));
    const float r = (float)(word >> 8) * 0x1p-24f;
    U.q = 1.0f / (1.0f + expf(-alpha * (U.P - r)));
    return U;
}

// neighbourhood of a site addressed on its own
struct DmcNb {
    float sr, sl, sd, su;  // neighbour spins
    float jr, jl, jd, ju;  // couplings of the four bonds
    int xr, xl, yd, yu;
};

__device__ __forceinline__ DmcNb dmc_nb(const float* s, const float* Jx, const float* Jy, int Lx,
                                        int Ly, int y, int x) {
    DmcNb N;
    N.xr = wrapd(x + 1, Lx);
    N.xl = wrapd(x - 1, Lx);
    N.yd = wrapd(y + 1, Ly);
    N.yu = wrapd(y - 1, Ly);
    const size_t row = (size_t)y * Lx;
    N.sr = s[row + N.xr];
    N.sl = s[row + N.xl];
    N.sd = s[(size_t)N.yd * Lx + x];
    N.su = s[(size_t)N.yu * Lx + x];
    N.jr = Jx[row + x];
    N.jl = Jx[row + N.xl];
    N.jd = Jy[row + x];
    N.ju = Jy[(size_t)N.yu * Lx + x];
    return N;
}

// An 8-float span of a row held as two float4 values (registers only: the
// sites are picked by value selects, never by an index into a local array).
struct Row8 {
    float4 a, b;
};

__device__ __forceinline__ Row8 ld8(const float* p) {
    return Row8{*reinterpret_cast<const float4*>(p), *reinterpret_cast<const float4*>(p + 4)};
}

__device__ __forceinline__ float el4(const float4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// element i (0..7, a compile-time constant after unrolling) of a span
__device__ __forceinline__ float el8(const Row8& r, int i) { return i < 4 ? el4(r.a, i) : el4(r.b, i - 4); }

// element i of the span extended by one column on each side: index 0 is the
// column left of the span, 9 the one right of it (both are e: a lane needs
// only the side its parity reaches)
__device__ __forceinline__ float el10(const Row8& r, float e, int i) {
    return (i == 0 || i == 9) ? e : el8(r, i - 1);
}

// the same for a span extended on the left only (index 0)
__device__ __forceinline__ float el9(const Row8& r, float e, int i) {
    return i == 0 ? e : el8(r, i - 1);
}

__device__ __forceinline__ float pick(bool o, float odd, float even) { return o ? odd : even; }

// the span r with the four own sites (odd offsets if o, even otherwise)
// replaced by v, written as two 16-byte stores
__device__ __forceinline__ void store_span(float* p, const Row8& r, bool o, const float* v) {
    float4 A = r.a, B = r.b;
    if (o) {
        A.y = v[0]; A.w = v[1]; B.y = v[2]; B.w = v[3];
    } else {
        A.x = v[0]; A.z = v[1]; B.x = v[2]; B.z = v[3];
    }
    *reinterpret_cast<float4*>(p) = A;
    *reinterpret_cast<float4*>(p + 4) = B;
}

// Span of one Philox block when Lx % 8 == 0: block b covers row y, columns
// x0 .. x0 + 7 with x0 = 8 (b mod Lx/8); its sites are x0 + 2u + par,
// par = (y + c) & 1.  xe is the column beyond the span that the sites'
// horizontal neighbours reach (x0 - 1 for par 0, x0 + 8 for par 1), xj the
// bond left of the span (x0 - 1).
struct Span8 {
    int y, x0, par, yd, yu, xe, xj;
};

__device__ __forceinline__ Span8 span8(int b, int Lx, int Ly, int c) {
    Span8 S;
    const int G = Lx >> 3;
    S.y = b / G;
    S.x0 = 8 * (b - S.y * G);
    S.par = (S.y + c) & 1;
    S.yd = S.y + 1 == Ly ? 0 : S.y + 1;
    S.yu = S.y == 0 ? Ly - 1 : S.y - 1;
    S.xj = S.x0 == 0 ? Lx - 1 : S.x0 - 1;
    S.xe = S.par ? (S.x0 + 8 == Lx ? 0 : S.x0 + 8) : S.xj;
    return S;
}

}  // namespace

// ---- forward ---------------------------------------------------------------

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
        const DmcNb N = dmc_nb(s, Jx, Jy, a.Lx, a.Ly, d.y, d.x);
        const DmcUpd U = dmc_update(sv, N.jr, N.sr, N.jl, N.sl, N.jd, N.sd, N.ju, N.su, a.beta,
                                    a.alpha, a.h, w[u]);
        sold[u] = sv;
        snew[u] = sv * (1.0f - 2.0f * U.q);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (4 * b + u < n_sites) {
            sv_save[4 * b + u] = sold[u];
            s[idx[u]] = snew[u];
        }
}

// Lx % 8 == 0: rows y-1, y, y+1 of the spins and the coupling rows as 8-float
// spans; the own sites and their neighbours are picked by par.
// Offsets within a replica are 32-bit (Lx Ly <= 2^28), on a replica base that
// is uniform over the workgroup.
__device__ __forceinline__ void pass8_block(const DmcArgs& a, int c, uint32_t p, float* save,
                                            int r, int b, int n_blocks) {
    const int Lx = a.Lx;
    const Span8 P8 = span8(b, Lx, a.Ly, c);
    const size_t off = (size_t)r * Lx * a.Ly;
    float* s = a.s + off;
    const float* Jx = a.Jx + off;
    const float* Jy = a.Jy + off;
    const uint32_t rw = (uint32_t)P8.y * Lx, ro = rw + P8.x0, rd = (uint32_t)P8.yd * Lx + P8.x0,
                   ru = (uint32_t)P8.yu * Lx + P8.x0;
    // S: spins of row y over the span (plus the column beyond it that par
    // reaches), X: Jx of row y (plus the bond left of the span)
    const Row8 S = ld8(s + ro), D = ld8(s + rd), U = ld8(s + ru);
    const float se = s[rw + P8.xe];
    const Row8 X = ld8(Jx + ro), Y0 = ld8(Jy + ro), Y1 = ld8(Jy + ru);
    const float xe = Jx[rw + P8.xj];
    uint32_t w[4];
    philox4x32_10((uint32_t)b, p, a.rid0 + (uint32_t)r, kTagDmc, a.key0, a.key1, w);
    const bool o = P8.par != 0;
    float sold[4], snew[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const float sv = pick(o, el10(S, se, 2 * u + 2), el10(S, se, 2 * u + 1));
        const float sl = pick(o, el10(S, se, 2 * u + 1), el10(S, se, 2 * u));
        const float sr = pick(o, el10(S, se, 2 * u + 3), el10(S, se, 2 * u + 2));
        const float jr = pick(o, el9(X, xe, 2 * u + 2), el9(X, xe, 2 * u + 1));
        const float jl = pick(o, el9(X, xe, 2 * u + 1), el9(X, xe, 2 * u));
        const float sd = pick(o, el8(D, 2 * u + 1), el8(D, 2 * u));
        const float su = pick(o, el8(U, 2 * u + 1), el8(U, 2 * u));
        const float jd = pick(o, el8(Y0, 2 * u + 1), el8(Y0, 2 * u));
        const float ju = pick(o, el8(Y1, 2 * u + 1), el8(Y1, 2 * u));
        const DmcUpd Q = dmc_update(sv, jr, sr, jl, sl, jd, sd, ju, su, a.beta, a.alpha, a.h, w[u]);
        sold[u] = sv;
        snew[u] = sv * (1.0f - 2.0f * Q.q);
    }
    *reinterpret_cast<float4*>(save + (size_t)r * (4 * n_blocks) + 4 * (uint32_t)b) =
        make_float4(sold[0], sold[1], sold[2], sold[3]);
    // the whole span is written back, the other colour's values unchanged:
    // full cache lines instead of every other word (partial lines cost HBM
    // time), and no other lane writes the span during the pass
    store_span(s + ro, S, o, snew);
}

__global__ void __launch_bounds__(256) k_dmc_pass8(DmcArgs a, int c, uint32_t p, float* save) {
    const int n_blocks = a.Ly * (a.Lx >> 3);
    const int b = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (b >= n_blocks) return;
    pass8_block(a, c, p, save, blockIdx.y, b, n_blocks);
}

// ---- backward --------------------------------------------------------------

// tin: t of the pass replayed before this one (sites of colour 1 - c, the
// neighbours), or null for the first replayed pass; tout: t of this pass.
__global__ void __launch_bounds__(256) k_dmc_back(DmcArgs a, int c, uint32_t p,
                                                  const float* save, float* gs, float* gJx,
                                                  float* gJy, const float* tin, float* tout) {
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
    const float* ti = tin ? tin + (size_t)r * n_sites : nullptr;
    float* to = tout + (size_t)r * n_sites;
    uint32_t w[4];
    philox4x32_10((uint32_t)b, p, a.rid0 + (uint32_t)r, kTagDmc, a.key0, a.key1, w);
    // phase 1: every load of the four sites (including the coupling
    // gradients they add to); phase 2: every store
    float gout[4], tv[4], sold[4], gr[4], gl[4], gd[4], gu[4];
    size_t ii[4], ir[4], il[4], iu[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = 4 * b + u;
        gout[u] = tv[u] = sold[u] = gr[u] = gl[u] = gd[u] = gu[u] = 0.f;
        ii[u] = ir[u] = il[u] = iu[u] = 0;
        if (k >= n_sites) continue;
        const DmcSite d = dmc_site(k, W, c);
        const float sv = sv_save[k];
        const DmcNb N = dmc_nb(s, Jx, Jy, a.Lx, a.Ly, d.y, d.x);
        const DmcUpd U = dmc_update(sv, N.jr, N.sr, N.jl, N.sl, N.jd, N.sd, N.ju, N.su, a.beta,
                                    a.alpha, a.h, w[u]);
        float av = g[d.i];
        if (ti)  // within-colour index of (y', x'): y' W + (x' >> 1)
            av += N.jr * ti[d.y * W + (N.xr >> 1)] + N.jl * ti[d.y * W + (N.xl >> 1)] +
                  N.jd * ti[N.yd * W + (d.x >> 1)] + N.ju * ti[N.yu * W + (d.x >> 1)];
        const float wq = 4.0f * a.alpha * a.beta * U.q * (1.0f - U.q) * U.P;
        gout[u] = av * ((1.0f - 2.0f * U.q) + wq * sv * U.hloc);
        const float t = av * wq * sv * sv;
        tv[u] = t;
        sold[u] = sv;
        const size_t row = (size_t)d.y * a.Lx;
        ii[u] = d.i;
        ir[u] = row + d.x;
        il[u] = row + N.xl;
        iu[u] = (size_t)N.yu * a.Lx + d.x;
        gr[u] = gx[ir[u]] + t * N.sr;
        gl[u] = gx[il[u]] + t * N.sl;
        gd[u] = gy[ir[u]] + t * N.sd;
        gu[u] = gy[iu[u]] + t * N.su;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = 4 * b + u;
        if (k >= n_sites) continue;
        g[ii[u]] = gout[u];
        to[k] = tv[u];
        gx[ir[u]] = gr[u];
        gx[il[u]] = gl[u];
        gy[ir[u]] = gd[u];
        gy[iu[u]] = gu[u];
        s[ii[u]] = sold[u];  // the state before this pass
    }
}

// Lx % 8 == 0: the spans of the spins, couplings, adjoints and coupling
// gradients of rows y-1, y, y+1 as 16-byte loads.
__device__ __forceinline__ void back8_block(const DmcArgs& a, int c, uint32_t p,
                                            const float* save, float* gs, float* gJx, float* gJy,
                                            const float* tin, float* tout, int r, int b,
                                            int n_blocks) {
    const int Lx = a.Lx;
    const int W = Lx >> 1;
    const int n_sites = 4 * n_blocks;
    const Span8 P8 = span8(b, Lx, a.Ly, c);
    const size_t off = (size_t)r * Lx * a.Ly;
    float* s = a.s + off;
    const float* Jx = a.Jx + off;
    const float* Jy = a.Jy + off;
    float* g = gs + off;
    float* gx = gJx + off;
    float* gy = gJy + off;
    const uint32_t rw = (uint32_t)P8.y * Lx, ro = rw + P8.x0, rd = (uint32_t)P8.yd * Lx + P8.x0,
                   ru = (uint32_t)P8.yu * Lx + P8.x0;
    // as in the forward; G: adjoints of row y, GX: Jx gradients of row y
    // (plus the bond left of the span), GY0 / GY1: Jy gradients of rows y and
    // y - 1; T: t of the colour 1 - c sites of row y over the span (plus the
    // one beyond it that par reaches), TD / TU: the same in rows y + 1, y - 1
    const float4 sold4 = *reinterpret_cast<const float4*>(save + (size_t)r * n_sites +
                                                          4 * (uint32_t)b);
    const float sold[4] = {sold4.x, sold4.y, sold4.z, sold4.w};
    const Row8 S = ld8(s + ro), D = ld8(s + rd), U = ld8(s + ru);
    const float se = s[rw + P8.xe];
    const Row8 X = ld8(Jx + ro), Y0 = ld8(Jy + ro), Y1 = ld8(Jy + ru);
    const float xe = Jx[rw + P8.xj];
    const Row8 G = ld8(g + ro), GX = ld8(gx + ro), GY0 = ld8(gy + ro), GY1 = ld8(gy + ru);
    const float gxe = gx[rw + P8.xj];
    float4 T = make_float4(0.f, 0.f, 0.f, 0.f), TD = T, TU = T;
    float te = 0.f;
    if (tin) {
        // within-colour indices y' W + x0 / 2 + u (16-byte aligned)
        const float* ti = tin + (size_t)r * n_sites;
        T = *reinterpret_cast<const float4*>(ti + 4 * (uint32_t)b);
        te = ti[(uint32_t)P8.y * W + (P8.xe >> 1)];
        TD = *reinterpret_cast<const float4*>(ti + (uint32_t)P8.yd * W + (P8.x0 >> 1));
        TU = *reinterpret_cast<const float4*>(ti + (uint32_t)P8.yu * W + (P8.x0 >> 1));
    }
    uint32_t w[4];
    philox4x32_10((uint32_t)b, p, a.rid0 + (uint32_t)r, kTagDmc, a.key0, a.key1, w);
    const bool o = P8.par != 0;
    float gout[4], tv[4], gxl[4], gxr[4], gyd[4], gyu[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const float sv = sold[u];
        const float sl = pick(o, el10(S, se, 2 * u + 1), el10(S, se, 2 * u));
        const float sr = pick(o, el10(S, se, 2 * u + 3), el10(S, se, 2 * u + 2));
        const float jr = pick(o, el9(X, xe, 2 * u + 2), el9(X, xe, 2 * u + 1));
        const float jl = pick(o, el9(X, xe, 2 * u + 1), el9(X, xe, 2 * u));
        const float sd = pick(o, el8(D, 2 * u + 1), el8(D, 2 * u));
        const float su = pick(o, el8(U, 2 * u + 1), el8(U, 2 * u));
        const float jd = pick(o, el8(Y0, 2 * u + 1), el8(Y0, 2 * u));
        const float ju = pick(o, el8(Y1, 2 * u + 1), el8(Y1, 2 * u));
        const DmcUpd Q = dmc_update(sv, jr, sr, jl, sl, jd, sd, ju, su, a.beta, a.alpha, a.h, w[u]);
        float av = pick(o, el8(G, 2 * u + 1), el8(G, 2 * u));
        if (tin) {
            // T extended: index 0 = te (left, par 0), 1..4 = T, 5 = te (right, par 1)
            const float tl = pick(o, el4(T, u), u == 0 ? te : el4(T, u - 1));
            const float tr = pick(o, u == 3 ? te : el4(T, u + 1), el4(T, u));
            av += jr * tr + jl * tl + jd * el4(TD, u) + ju * el4(TU, u);
        }
        const float wq = 4.0f * a.alpha * a.beta * Q.q * (1.0f - Q.q) * Q.P;
        gout[u] = av * ((1.0f - 2.0f * Q.q) + wq * sv * Q.hloc);
        const float t = av * wq * sv * sv;
        tv[u] = t;
        gxr[u] = pick(o, el9(GX, gxe, 2 * u + 2), el9(GX, gxe, 2 * u + 1)) + t * sr;
        gxl[u] = pick(o, el9(GX, gxe, 2 * u + 1), el9(GX, gxe, 2 * u)) + t * sl;
        gyd[u] = pick(o, el8(GY0, 2 * u + 1), el8(GY0, 2 * u)) + t * sd;
        gyu[u] = pick(o, el8(GY1, 2 * u + 1), el8(GY1, 2 * u)) + t * su;
    }
    *reinterpret_cast<float4*>(tout + (size_t)r * n_sites + 4 * (uint32_t)b) =
        make_float4(tv[0], tv[1], tv[2], tv[3]);
    // the horizontal bonds of the span's sites: columns x0 .. x0 + 7 for
    // par 1; x0 - 1 .. x0 + 6 for par 0 (x0 + 7 belongs to the next span)
    if (o) {
        *reinterpret_cast<float4*>(gx + ro) = make_float4(gxl[0], gxr[0], gxl[1], gxr[1]);
        *reinterpret_cast<float4*>(gx + ro + 4) = make_float4(gxl[2], gxr[2], gxl[3], gxr[3]);
    } else {
        gx[rw + P8.xj] = gxl[0];
        *reinterpret_cast<float4*>(gx + ro) = make_float4(gxr[0], gxl[1], gxr[1], gxl[2]);
        gx[ro + 4] = gxr[2];
        gx[ro + 5] = gxl[3];
        gx[ro + 6] = gxr[3];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t x = 2 * u + P8.par;
        gy[ro + x] = gyd[u];
        gy[ru + x] = gyu[u];
    }
    // whole spans, as in the forward: the adjoints and the state before
    // this pass at the own sites, the other colour's values unchanged
    store_span(g + ro, G, o, gout);
    store_span(s + ro, S, o, sold);
}

__global__ void __launch_bounds__(256) k_dmc_back8(DmcArgs a, int c, uint32_t p,
                                                   const float* save, float* gs, float* gJx,
                                                   float* gJy, const float* tin, float* tout) {
    const int n_blocks = a.Ly * (a.Lx >> 3);
    const int b = (int)blockIdx.x * 256 + (int)threadIdx.x;
    if (b >= n_blocks) return;
    back8_block(a, c, p, save, gs, gJx, gJy, tin, tout, blockIdx.y, b, n_blocks);
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
    const float tr = tw[d.y * W + (xr >> 1)], tl = tw[d.y * W + (xl >> 1)];
    const float td = tw[yd * W + (d.x >> 1)], tu = tw[yu * W + (d.x >> 1)];
    const size_t row = (size_t)d.y * Lx;
    const float acc = Jx[row + d.x] * tr + Jx[row + xl] * tl + Jy[row + d.x] * td +
                      Jy[(size_t)yu * Lx + d.x] * tu;
    gs[off + d.i] += acc;
}

namespace {

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }


}  // namespace

hipError_t launch_dmc_forward(const DmcArgs& a, uint64_t t0, int n_sweeps, float* save,
                              hipStream_t s) {
    const int n_sites = a.Ly * (a.Lx >> 1);
    const bool v8 = (a.Lx & 7) == 0 && aligned16(a.s) && aligned16(a.Jx) && aligned16(a.Jy) &&
                    aligned16(save);
    const int n_blocks = (n_sites + 3) >> 2;
    const dim3 grid((n_blocks + 255) / 256, a.R), block(256);
    for (int i = 0; i < n_sweeps; ++i)
        for (int c = 0; c < 2; ++c) {
            const uint32_t p = (uint32_t)(2 * (t0 + (uint64_t)i) + (uint64_t)c);
            float* sv = save + (size_t)(2 * i + c) * a.R * n_sites;
            if (v8)
                hipLaunchKernelGGL(k_dmc_pass8, grid, block, 0, s, a, c, p, sv);
            else
                hipLaunchKernelGGL(k_dmc_pass, grid, block, 0, s, a, c, p, sv);
        }
    return hipGetLastError();
}

hipError_t launch_dmc_backward(const DmcArgs& a, uint64_t t0, int n_sweeps, const float* save,
                               float* gs, float* gJx, float* gJy, float* work, hipStream_t s) {
    const int n_sites = a.Ly * (a.Lx >> 1);
    const size_t plane = (size_t)a.R * n_sites;
    const bool v8 = (a.Lx & 7) == 0 && aligned16(a.s) && aligned16(a.Jx) && aligned16(a.Jy) &&
                    aligned16(save) && aligned16(gs) && aligned16(gJx) && aligned16(gJy) &&
                    aligned16(work);
    const int n_blocks = (n_sites + 3) >> 2;
    const dim3 grid((n_blocks + 255) / 256, a.R), gridg((n_sites + 255) / 256, a.R), block(256);
    // pass m = 2 i + c writes its t to plane m & 1 and folds in the t of
    // pass m + 1 from the other plane
    for (int m = 2 * n_sweeps - 1; m >= 0; --m) {
        const int i = m >> 1, c = m & 1;
        const uint32_t p = (uint32_t)(2 * (t0 + (uint64_t)i) + (uint64_t)c);
        const float* sv = save + (size_t)m * plane;
        const float* tin = m == 2 * n_sweeps - 1 ? nullptr : work + (size_t)((m + 1) & 1) * plane;
        float* tout = work + (size_t)(m & 1) * plane;
        if (v8)
            hipLaunchKernelGGL(k_dmc_back8, grid, block, 0, s, a, c, p, sv, gs, gJx, gJy,
                               tin, tout);
        else
            hipLaunchKernelGGL(k_dmc_back, grid, block, 0, s, a, c, p, sv, gs, gJx, gJy, tin,
                               tout);
    }
    if (n_sweeps > 0)  // pass 0 (colour 0): its t reach the colour-1 sites
        hipLaunchKernelGGL(k_dmc_gather, gridg, block, 0, s, a, 0, gs, work);
    return hipGetLastError();
}

}  // namespace spinmc

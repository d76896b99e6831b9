// Triangular-lattice Ising (the triangular kernels of the Methods): the
// checkerboard Metropolis chain of Algorithm 1 on the six-neighbour lattice.
//
// Sites sit on an Ly x Lx array (int8 spins, natural row-major); the
// neighbours of (y, x) are (y, x+-1), (y+-1, x), (y-1, x+1) and (y+1, x-1)
// (periodic), one coupling J for every bond, H = -J sum s s' - h sum s.
// Three colours c = (x + 2y) mod 3 -- no bond joins two sites of one colour
// when Lx and Ly are multiples of 3 -- make a sweep of three passes
// p = 3t + c.  The sites of colour c in row y are x = 3i + (c + y) mod 3; the
// within-colour index k = y Lx/3 + i selects word k & 3 of Philox4x32-10
// block (k >> 2, p, rid, 0), used whole as W; the flip is accepted iff
// W < T[7 [s > 0] + (S6 + 6) / 2] with the FP64 host thresholds
// T = ceil(2^32 exp(-beta 2 s (J S6 + h))) (2^32 when that change is <= 0).
// A lane takes the four sites of one Philox block.
#include "tri_internal.hpp"

namespace spinmc {

namespace {
constexpr uint32_t kTriTagMain = 0u, kTriTagInit = 2u;

__device__ __forceinline__ int wrapt(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
}  // namespace

// Initial spins from the init stream of the Ising model: site n = y Lx + x
// takes word n & 3 of block (n >> 2, 0, rid, 2); +1 iff it is < 2^31.
__global__ void __launch_bounds__(256) k_tri_init(TriArgs a) {
    const RepDev D = a.reps[blockIdx.y];
    const int n = D.Lx * D.Ly * (D.model == kModelIsingHC ? D.q : 1);
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * b >= n) return;
    uint32_t w[4];
    philox4x32_10((uint32_t)b, 0u, D.rid, kTriTagInit, a.key0, a.key1, w);
    int8_t* lat = a.lat + D.lat_off;
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (4 * b + u < n) lat[4 * b + u] = w[u] < 0x80000000u ? (int8_t)1 : (int8_t)-1;
}

__global__ void __launch_bounds__(256) k_tri_pass(TriArgs a, int c, int sweep_off) {
    __shared__ uint64_t lt[kTriClasses];
    const int r = blockIdx.y;
    if (threadIdx.x < kTriClasses) lt[threadIdx.x] = a.tab[(size_t)r * kTriClasses + threadIdx.x];
    __syncthreads();
    const RepDev D = a.reps[r];
    const int Lx = D.Lx, Ly = D.Ly, W3 = Lx / 3;
    const int nk = Ly * W3;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * b >= nk) return;
    const uint64_t t = *a.t_base + (uint64_t)sweep_off;
    const uint32_t p = (uint32_t)(3 * t + (uint64_t)c);
    uint32_t w[4];
    philox4x32_10((uint32_t)b, p, D.rid, kTriTagMain, a.key0, a.key1, w);
    int8_t* lat = a.lat + D.lat_off;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = 4 * b + u;
        if (k >= nk) break;
        const int y = k / W3;
        const int x = 3 * (k - y * W3) + (c + y) % 3;
        const int yu = wrapt(y - 1, Ly), yd = wrapt(y + 1, Ly);
        const int xl = wrapt(x - 1, Lx), xr = wrapt(x + 1, Lx);
        const int8_t* row = lat + (size_t)y * Lx;
        const int8_t* up = lat + (size_t)yu * Lx;
        const int8_t* dn = lat + (size_t)yd * Lx;
        const int s = row[x];
        const int S6 = row[xl] + row[xr] + up[x] + dn[x] + up[xr] + dn[xl];
        const int idx = 7 * (s > 0) + (S6 + 6) / 2;
        if ((uint64_t)w[u] < lt[idx]) lat[(size_t)y * Lx + x] = (int8_t)(-s);
    }
}

// Lx a multiple of 12: the four sites of a Philox block lie in one row,
// x = 12 j + xc + 3u (xc = (c + y) mod 3), inside the 12-byte span
// [12 j, 12 j + 12) of rows y - 1, y, y + 1, which come in as dwords (plus one
// halo byte at either end of row y, the right one of row y - 1 and the left
// one of row y + 1).  The row-y span is written back whole: no other lane
// writes it during the pass, and the other colours' bytes are unchanged.
namespace {
__device__ __forceinline__ int sbyte(const uint32_t (&v)[3], int i) {
    return (int)(int8_t)(v[i >> 2] >> (8 * (i & 3)));
}
}  // namespace

__global__ void __launch_bounds__(256) k_tri_pass12(TriArgs a, int c, int sweep_off) {
    __shared__ uint64_t lt[kTriClasses];
    const int r = blockIdx.y;
    if (threadIdx.x < kTriClasses) lt[threadIdx.x] = a.tab[(size_t)r * kTriClasses + threadIdx.x];
    __syncthreads();
    const RepDev D = a.reps[r];
    const int Lx = D.Lx, Ly = D.Ly, G = Lx / 12;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= Ly * G) return;
    const int y = b / G, x0 = 12 * (b - y * G);
    const int xc = (c + y) % 3;
    const int yu = y == 0 ? Ly - 1 : y - 1, yd = y + 1 == Ly ? 0 : y + 1;
    const int xl = x0 == 0 ? Lx - 1 : x0 - 1, xr = x0 + 12 == Lx ? 0 : x0 + 12;
    int8_t* lat = a.lat + D.lat_off;
    const uint32_t* row = reinterpret_cast<const uint32_t*>(lat + (size_t)y * Lx + x0);
    const uint32_t* up = reinterpret_cast<const uint32_t*>(lat + (size_t)yu * Lx + x0);
    const uint32_t* dn = reinterpret_cast<const uint32_t*>(lat + (size_t)yd * Lx + x0);
    uint32_t S[3] = {row[0], row[1], row[2]};
    const uint32_t U[3] = {up[0], up[1], up[2]};
    const uint32_t Dn[3] = {dn[0], dn[1], dn[2]};
    const int sl = lat[(size_t)y * Lx + xl], sr = lat[(size_t)y * Lx + xr];
    const int ur = lat[(size_t)yu * Lx + xr], dl = lat[(size_t)yd * Lx + xl];
    const uint64_t t = *a.t_base + (uint64_t)sweep_off;
    const uint32_t p = (uint32_t)(3 * t + (uint64_t)c);
    uint32_t w[4];
    philox4x32_10((uint32_t)b, p, D.rid, 0u, a.key0, a.key1, w);
    uint32_t flip[3] = {0u, 0u, 0u};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int o = xc + 3 * u;  // offset of the site in the span, 0..11
        const int s = sbyte(S, o);
        const int left = o == 0 ? sl : sbyte(S, o - 1);
        const int right = o == 11 ? sr : sbyte(S, o + 1);
        const int upr = o == 11 ? ur : sbyte(U, o + 1);
        const int dnl = o == 0 ? dl : sbyte(Dn, o - 1);
        const int S6 = left + right + sbyte(U, o) + sbyte(Dn, o) + upr + dnl;
        const int idx = 7 * (s > 0) + (S6 + 6) / 2;
        // a flip negates the byte: s -> -s is s ^ 0xFE for s = +-1
        if ((uint64_t)w[u] < lt[idx]) flip[o >> 2] |= 0xFEu << (8 * (o & 3));
    }
    uint32_t* rw = reinterpret_cast<uint32_t*>(lat + (size_t)y * Lx + x0);
    rw[0] = S[0] ^ flip[0];
    rw[1] = S[1] ^ flip[1];
    rw[2] = S[2] ^ flip[2];
}

// [M, Bh, Bv, Bd]: wave sums of each lane's sites, one atomic per wave and
// statistic (integers, so the order does not matter).
__global__ void __launch_bounds__(256) k_tri_stats(TriArgs a, int rec_row) {
    const int r = blockIdx.y;
    const RepDev D = a.reps[r];
    const int Lx = D.Lx, Ly = D.Ly, n = Lx * Ly;
    const int8_t* lat = a.lat + D.lat_off;
    int M = 0, Bh = 0, Bv = 0, Bd = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int y = i / Lx, x = i - y * Lx;
        const int yd = wrapt(y + 1, Ly), xr = wrapt(x + 1, Lx), xl = wrapt(x - 1, Lx);
        const int s = lat[i];
        M += s;
        Bh += s * lat[(size_t)y * Lx + xr];
        Bv += s * lat[(size_t)yd * Lx + x];
        Bd += s * lat[(size_t)yd * Lx + xl];
    }
    for (int o = 32; o > 0; o >>= 1) {
        M += __shfl_xor(M, o);
        Bh += __shfl_xor(Bh, o);
        Bv += __shfl_xor(Bv, o);
        Bd += __shfl_xor(Bd, o);
    }
    if ((threadIdx.x & 63) == 0) {
        int32_t* row = a.stats + ((size_t)rec_row * a.R + r) * a.width;
        atomicAdd(&row[0], M);
        atomicAdd(&row[1], Bh);
        atomicAdd(&row[2], Bv);
        atomicAdd(&row[3], Bd);
    }
}

// Chain / square / simple cubic (Lz = D.q): the colour-c site of the pair
// (2k, 2k + 1) -- both in one row since Lx is even -- for the four k of a
// Philox block; neighbours x +- 1 and, where the extent exceeds 1, y +- 1 and
// z +- 1.
__global__ void __launch_bounds__(256) k_hc_pass(TriArgs a, int c, int sweep_off) {
    __shared__ uint64_t lt[kTriClasses];
    const int r = blockIdx.y;
    if (threadIdx.x < kTriClasses) lt[threadIdx.x] = a.tab[(size_t)r * kTriClasses + threadIdx.x];
    __syncthreads();
    const RepDev D = a.reps[r];
    const int Lx = D.Lx, Ly = D.Ly, Lz = D.q, plane = Lx * Ly;
    const int nk = plane * Lz / 2;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * b >= nk) return;
    const uint64_t t = *a.t_base + (uint64_t)sweep_off;
    const uint32_t p = (uint32_t)(2 * t + (uint64_t)c);
    uint32_t w[4];
    philox4x32_10((uint32_t)b, p, D.rid, kTriTagMain, a.key0, a.key1, w);
    int8_t* lat = a.lat + D.lat_off;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = 4 * b + u;
        if (k >= nk) break;
        const int row = (2 * k) / Lx;  // z Ly + y
        const int z = row / Ly, y = row - z * Ly;
        const int x = 2 * k - row * Lx + ((c + y + z) & 1);
        const size_t rb = (size_t)row * Lx;
        const int s = lat[rb + x];
        int S = lat[rb + wrapt(x - 1, Lx)] + lat[rb + wrapt(x + 1, Lx)];
        if (Ly > 1)
            S += lat[(size_t)(z * Ly + wrapt(y - 1, Ly)) * Lx + x] +
                 lat[(size_t)(z * Ly + wrapt(y + 1, Ly)) * Lx + x];
        if (Lz > 1)
            S += lat[(size_t)wrapt(z - 1, Lz) * plane + (size_t)y * Lx + x] +
                 lat[(size_t)wrapt(z + 1, Lz) * plane + (size_t)y * Lx + x];
        const int idx = 7 * (s > 0) + (S + 6) / 2;
        if ((uint64_t)w[u] < lt[idx]) lat[rb + x] = (int8_t)(-s);
    }
}

// Lx a multiple of 8: the four sites of a Philox block are the colour-c
// bytes of one 8-byte row span [x0, x0 + 8), offsets o = 2u + par with
// par = (c + y + z) & 1; the spans of the neighbouring rows (y +- 1) and
// planes (z +- 1) come in as dword pairs, plus the halo bytes x0 - 1 and
// x0 + 8 of the own row.  The own span is written back whole (its other
// colour's bytes unchanged; no other lane writes it during the pass).
namespace {
__device__ __forceinline__ int sbyte2(uint2 v, int i) {
    return (int)(int8_t)((i < 4 ? v.x : v.y) >> (8 * (i & 3)));
}
}  // namespace

__global__ void __launch_bounds__(256) k_hc_pass8(TriArgs a, int c, int sweep_off) {
    __shared__ uint64_t lt[kTriClasses];
    const int r = blockIdx.y;
    if (threadIdx.x < kTriClasses) lt[threadIdx.x] = a.tab[(size_t)r * kTriClasses + threadIdx.x];
    __syncthreads();
    const RepDev D = a.reps[r];
    const int Lx = D.Lx, Ly = D.Ly, Lz = D.q, plane = Lx * Ly;
    const int nb = plane * Lz / 8;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int row = (8 * b) / Lx;  // z Ly + y
    const int z = row / Ly, y = row - z * Ly;
    const int x0 = 8 * b - row * Lx;
    const int par = (c + y + z) & 1;
    int8_t* lat = a.lat + D.lat_off;
    const size_t own = (size_t)row * Lx + x0;
    const uint2 S = *reinterpret_cast<const uint2*>(lat + own);
    const int hl = lat[(size_t)row * Lx + (x0 == 0 ? Lx - 1 : x0 - 1)];
    const int hr = lat[(size_t)row * Lx + (x0 + 8 == Lx ? 0 : x0 + 8)];
    uint2 Yu = make_uint2(0u, 0u), Yd = Yu, Zu = Yu, Zd = Yu;
    if (Ly > 1) {
        Yu = *reinterpret_cast<const uint2*>(lat + (size_t)(z * Ly + wrapt(y - 1, Ly)) * Lx + x0);
        Yd = *reinterpret_cast<const uint2*>(lat + (size_t)(z * Ly + wrapt(y + 1, Ly)) * Lx + x0);
    }
    if (Lz > 1) {
        Zu = *reinterpret_cast<const uint2*>(lat + (size_t)wrapt(z - 1, Lz) * plane + own - (size_t)z * plane);
        Zd = *reinterpret_cast<const uint2*>(lat + (size_t)wrapt(z + 1, Lz) * plane + own - (size_t)z * plane);
    }
    const uint64_t t = *a.t_base + (uint64_t)sweep_off;
    const uint32_t p = (uint32_t)(2 * t + (uint64_t)c);
    uint32_t w[4];
    philox4x32_10((uint32_t)b, p, D.rid, kTriTagMain, a.key0, a.key1, w);
    uint32_t flip[2] = {0u, 0u};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int o = 2 * u + par;
        const int s = sbyte2(S, o);
        int Sn = (o == 0 ? hl : sbyte2(S, o - 1)) + (o == 7 ? hr : sbyte2(S, o + 1));
        if (Ly > 1) Sn += sbyte2(Yu, o) + sbyte2(Yd, o);
        if (Lz > 1) Sn += sbyte2(Zu, o) + sbyte2(Zd, o);
        const int idx = 7 * (s > 0) + (Sn + 6) / 2;
        if ((uint64_t)w[u] < lt[idx]) flip[o >> 2] |= 0xFEu << (8 * (o & 3));
    }
    *reinterpret_cast<uint2*>(lat + own) = make_uint2(S.x ^ flip[0], S.y ^ flip[1]);
}

// [M, Bx, By, Bz] of the chain / square / cubic lattices.
__global__ void __launch_bounds__(256) k_hc_stats(TriArgs a, int rec_row) {
    const int r = blockIdx.y;
    const RepDev D = a.reps[r];
    const int Lx = D.Lx, Ly = D.Ly, Lz = D.q, plane = Lx * Ly, n = plane * Lz;
    const int8_t* lat = a.lat + D.lat_off;
    int M = 0, Bx = 0, By = 0, Bz = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int row = i / Lx, x = i - row * Lx;
        const int z = row / Ly, y = row - z * Ly;
        const int s = lat[i];
        M += s;
        Bx += s * lat[(size_t)row * Lx + wrapt(x + 1, Lx)];
        if (Ly > 1) By += s * lat[(size_t)(z * Ly + wrapt(y + 1, Ly)) * Lx + x];
        if (Lz > 1) Bz += s * lat[(size_t)wrapt(z + 1, Lz) * plane + (size_t)y * Lx + x];
    }
    for (int o = 32; o > 0; o >>= 1) {
        M += __shfl_xor(M, o);
        Bx += __shfl_xor(Bx, o);
        By += __shfl_xor(By, o);
        Bz += __shfl_xor(Bz, o);
    }
    if ((threadIdx.x & 63) == 0) {
        int32_t* rw = a.stats + ((size_t)rec_row * a.R + r) * a.width;
        atomicAdd(&rw[0], M);
        atomicAdd(&rw[1], Bx);
        atomicAdd(&rw[2], By);
        atomicAdd(&rw[3], Bz);
    }
}

// (e, |m|, m^2, m) per replica from [M, B1, B2, B3] (either lattice).
__global__ void k_tri_observables(TriArgs a, double* obs) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.R) return;
    const RepDev D = a.reps[r];
    const int32_t* s = a.stats + (size_t)r * a.width;
    const double N = (double)D.Lx * (double)D.Ly * (D.model == kModelIsingHC ? (double)D.q : 1.0);
    const double M = s[0];
    const double H = -((double)D.Jx * ((double)s[1] + (double)s[2] + (double)s[3]) +
                       (double)D.h * M);
    double* o = obs + (size_t)r * 4;
    o[0] = H / N;
    o[1] = fabs(M) / N;
    o[2] = (M / N) * (M / N);
    o[3] = M / N;
}

// All n_sweeps unrecorded sweeps in one launch, one workgroup per replica
// with its lattice in LDS (the layout of global memory) and a barrier after
// every colour pass: the same decisions as the streamed passes, without the
// per-pass launches and lattice round trips.  Needs Lx % 12 == 0 for the
// triangular lattice (the four sites of a Philox block in one row) and
// Lx % 8 == 0 for the chain / cubic lattices.
template <int MODEL>
__global__ void __launch_bounds__(1024) k_nat_resident(TriArgs a, int n_sweeps) {
    extern __shared__ __align__(16) int8_t ls[];
    __shared__ uint64_t lt[kTriClasses];
    const int r = blockIdx.x;
    const RepDev D = a.reps[r];
    const int Lx = D.Lx, Ly = D.Ly, Lz = MODEL == kModelIsingHC ? D.q : 1;
    const int n = Lx * Ly * Lz;
    int8_t* lat = a.lat + D.lat_off;
    if (threadIdx.x < kTriClasses) lt[threadIdx.x] = a.tab[(size_t)r * kTriClasses + threadIdx.x];
    for (int i = threadIdx.x; i < n / 4; i += blockDim.x)
        reinterpret_cast<uint32_t*>(ls)[i] = reinterpret_cast<const uint32_t*>(lat)[i];
    __syncthreads();
    const uint64_t t0 = *a.t_base;
    constexpr int ncol = MODEL == kModelIsingHC ? 2 : 3;
    const int nb = MODEL == kModelIsingHC ? n / 8 : n / 12;  // Philox blocks per pass
    const int plane = Lx * Ly;
    for (int sw = 0; sw < n_sweeps; ++sw) {
        const uint64_t t = t0 + (uint64_t)sw;
        for (int c = 0; c < ncol; ++c) {
            const uint32_t p = (uint32_t)((uint64_t)ncol * t + (uint64_t)c);
            for (int b = threadIdx.x; b < nb; b += blockDim.x) {
                uint32_t w[4];
                philox4x32_10((uint32_t)b, p, D.rid, kTriTagMain, a.key0, a.key1, w);
                if (MODEL == kModelIsingTri) {
                    const int G = Lx / 12;
                    const int y = b / G, x0 = 12 * (b - y * G), xc = (c + y) % 3;
                    const int yu = y == 0 ? Ly - 1 : y - 1, yd = y + 1 == Ly ? 0 : y + 1;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int x = x0 + xc + 3 * u;
                        const int xl = x == 0 ? Lx - 1 : x - 1, xr = x + 1 == Lx ? 0 : x + 1;
                        const int s = ls[y * Lx + x];
                        const int S6 = ls[y * Lx + xl] + ls[y * Lx + xr] + ls[yu * Lx + x] +
                                       ls[yd * Lx + x] + ls[yu * Lx + xr] + ls[yd * Lx + xl];
                        if ((uint64_t)w[u] < lt[7 * (s > 0) + (S6 + 6) / 2])
                            ls[y * Lx + x] = (int8_t)(-s);
                    }
                } else {
                    const int row = (8 * b) / Lx;
                    const int z = row / Ly, y = row - z * Ly;
                    const int x0 = 8 * b - row * Lx, par = (c + y + z) & 1;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int x = x0 + 2 * u + par;
                        const int i = row * Lx + x;
                        const int s = ls[i];
                        int S = ls[row * Lx + (x == 0 ? Lx - 1 : x - 1)] +
                                ls[row * Lx + (x + 1 == Lx ? 0 : x + 1)];
                        if (Ly > 1)
                            S += ls[(z * Ly + (y == 0 ? Ly - 1 : y - 1)) * Lx + x] +
                                 ls[(z * Ly + (y + 1 == Ly ? 0 : y + 1)) * Lx + x];
                        if (Lz > 1)
                            S += ls[(z == 0 ? Lz - 1 : z - 1) * plane + y * Lx + x] +
                                 ls[(z + 1 == Lz ? 0 : z + 1) * plane + y * Lx + x];
                        if ((uint64_t)w[u] < lt[7 * (s > 0) + (S + 6) / 2]) ls[i] = (int8_t)(-s);
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n / 4; i += blockDim.x)
        reinterpret_cast<uint32_t*>(lat)[i] = reinterpret_cast<const uint32_t*>(ls)[i];
}

hipError_t launch_nat_resident(const TriArgs& a, int n_sweeps, int lds_bytes, hipStream_t s) {
    if (a.model == kModelIsingHC) {
        hipFuncSetAttribute((const void*)k_nat_resident<kModelIsingHC>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        hipLaunchKernelGGL(k_nat_resident<kModelIsingHC>, dim3(a.R), dim3(1024), lds_bytes, s, a,
                           n_sweeps);
    } else {
        hipFuncSetAttribute((const void*)k_nat_resident<kModelIsingTri>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        hipLaunchKernelGGL(k_nat_resident<kModelIsingTri>, dim3(a.R), dim3(1024), lds_bytes, s, a,
                           n_sweeps);
    }
    return hipGetLastError();
}

hipError_t launch_tri_init(const TriArgs& a, hipStream_t s) {
    const int nb = (a.max_sites + 3) / 4;
    hipLaunchKernelGGL(k_tri_init, dim3((nb + 255) / 256, a.R), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tri_pass(const TriArgs& a, int c, int sweep_off, hipStream_t s) {
    if (a.model == kModelIsingHC && a.all_lx8)
        hipLaunchKernelGGL(k_hc_pass8, dim3((a.max_blocks + 255) / 256, a.R), dim3(256), 0, s, a,
                           c, sweep_off);
    else if (a.model == kModelIsingHC)
        hipLaunchKernelGGL(k_hc_pass, dim3((a.max_blocks + 255) / 256, a.R), dim3(256), 0, s, a,
                           c, sweep_off);
    else if (a.all_lx12)
        hipLaunchKernelGGL(k_tri_pass12, dim3((a.max_blocks + 255) / 256, a.R), dim3(256), 0, s,
                           a, c, sweep_off);
    else
        hipLaunchKernelGGL(k_tri_pass, dim3((a.max_blocks + 255) / 256, a.R), dim3(256), 0, s, a,
                           c, sweep_off);
    return hipGetLastError();
}

hipError_t launch_tri_stats(const TriArgs& a, int rec_row, hipStream_t s) {
    const int per = (a.max_sites + 255) / 256;
    if (a.model == kModelIsingHC)
        hipLaunchKernelGGL(k_hc_stats, dim3(per < 64 ? per : 64, a.R), dim3(256), 0, s, a, rec_row);
    else
        hipLaunchKernelGGL(k_tri_stats, dim3(per < 64 ? per : 64, a.R), dim3(256), 0, s, a,
                           rec_row);
    return hipGetLastError();
}

hipError_t launch_tri_observables(const TriArgs& a, double* obs, hipStream_t s) {
    hipLaunchKernelGGL(k_tri_observables, dim3((a.R + 127) / 128), dim3(128), 0, s, a, obs);
    return hipGetLastError();
}

}  // namespace spinmc

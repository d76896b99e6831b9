// Multispin-coded square-lattice Ising (1-bit spins): 32 replicas with the
// same lattice shape, couplings, field and temperature packed bit by bit in
// one uint32 per site (bit b = 1 is s = +1 in replica b).  On the device a
// group's words sit in two colour planes, as the byte planes of the square
// lattice: site (y, x) is word (y, x >> 1) of plane (x + y) & 1, each plane
// Ly rows of W = Lx / 2 words.  The replicas share the random numbers, so
// one Philox word decides 32 attempts: in pass p = 2t + c (colour
// c = (x + y) & 1) the site with within-colour index k = (y Lx + x) >> 1 --
// its plane word index y W + (x >> 1) -- takes W = word k & 3 of block
// (k >> 2, p, rid, 0), and every bit whose class idx = 9 [s > 0] +
// 3 (Sx/2 + 1) + (Sy/2 + 1) has W < T[idx] flips (Algorithm 1; the
// thresholds are the FP64 host table of the square lattice).  The classes of
// all 32 bits come from bitwise logic: a neighbour bit agrees with the own
// bit where their xor is 0, and counts of 0, 1 or 2 agreeing horizontal
// (vertical) neighbours are ~(a | b), a ^ b and a & b.
//
// Lx is a multiple of 8: a lane takes the four sites of one Philox block,
// four consecutive words of a row of plane c, and reads the other plane's
// same row (its horizontal neighbours, with one halo word on the side of the
// row parity) and rows y - 1, y + 1 (vertical neighbours) as 16-byte loads;
// only the own plane is written.
#include "msc_internal.hpp"

namespace spinmc {

namespace {
constexpr uint32_t kMscTagMain = 0u, kMscTagInit = 2u;

__device__ __forceinline__ uint32_t e4(const uint4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// Word index of site (y, x) of a group's lattice in its colour planes.
__device__ __forceinline__ size_t plane_word(int y, int x, int Lx, int Ly) {
    const int W = Lx >> 1;
    return (size_t)((x + y) & 1) * Ly * W + (size_t)y * W + (x >> 1);
}
}  // namespace

// Bit b of site n: 1 iff word n & 3 of block (n >> 2, b, rid, 2) is < 2^31.
__global__ void __launch_bounds__(256) k_msc_init(MscArgs a) {
    const RepDev D = a.reps[blockIdx.y];
    const int n = D.Lx * D.Ly;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;  // block of 4 sites
    if (4 * q >= n) return;
    uint32_t v[4] = {0u, 0u, 0u, 0u};
    for (int b = 0; b < 32; ++b) {
        uint32_t w[4];
        philox4x32_10((uint32_t)q, (uint32_t)b, D.rid, kMscTagInit, a.key0, a.key1, w);
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] |= (w[u] < 0x80000000u ? 1u : 0u) << b;
    }
    uint32_t* lat = reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(a.lat) + D.lat_off);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int i = 4 * q + u;
        if (i < n) {
            const int y = i / D.Lx;
            lat[plane_word(y, i - y * D.Lx, D.Lx, D.Ly)] = v[u];
        }
    }
}

__global__ void __launch_bounds__(256) k_msc_pass4(MscArgs a, int c, int sweep_off) {
    const int g = blockIdx.y;
    // W < T as a 32-bit compare: W <= T - 1 for 1 <= T <= 2^32, and never
    // for T = 0 (uniform per class: scalar registers and scalar logic)
    uint32_t tm1[kMscClasses];
    bool never[kMscClasses];
    const uint64_t* tg = a.tab + (size_t)g * kMscClasses;
#pragma unroll
    for (int i = 0; i < kMscClasses; ++i) {
        const uint64_t T = tg[i];
        never[i] = T == 0;
        tm1[i] = T == 0 ? 0u : (uint32_t)(T - 1);
    }
    const RepDev D = a.reps[g];
    const int Lx = D.Lx, Ly = D.Ly, W = Lx >> 1, qpr = W >> 2;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;  // Philox block = word (y W + j0) / 4
    if (b >= Ly * qpr) return;
    const int y = b / qpr, j0 = 4 * (b - y * qpr);
    const int par = (c + y) & 1;  // own site of word j: x = 2 j + par
    const int yu = y == 0 ? Ly - 1 : y - 1, yd = y + 1 == Ly ? 0 : y + 1;
    uint32_t* lat = reinterpret_cast<uint32_t*>(reinterpret_cast<uint8_t*>(a.lat) + D.lat_off);
    uint32_t* own = lat + (size_t)c * Ly * W;
    const uint32_t* oth = lat + (size_t)(1 - c) * Ly * W;
    const uint4 S = *reinterpret_cast<const uint4*>(own + (size_t)y * W + j0);
    const uint4 M = *reinterpret_cast<const uint4*>(oth + (size_t)y * W + j0);
    const uint4 U = *reinterpret_cast<const uint4*>(oth + (size_t)yu * W + j0);
    const uint4 Dn = *reinterpret_cast<const uint4*>(oth + (size_t)yd * W + j0);
    // the horizontal neighbour outside the four words: word j0 - 1 (par 0)
    // or j0 + 4 (par 1) of the other plane's row, periodic
    const uint32_t halo =
        oth[(size_t)y * W + (par ? (j0 + 4 == W ? 0 : j0 + 4) : (j0 == 0 ? W - 1 : j0 - 1))];
    const uint64_t t = *a.t_base + (uint64_t)sweep_off;
    const uint32_t p = (uint32_t)(2 * t + (uint64_t)c);
    uint32_t w[4];
    philox4x32_10((uint32_t)b, p, D.rid, kMscTagMain, a.key0, a.key1, w);
    uint32_t nv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t s = e4(S, u);
        // left (x - 1) and right (x + 1) neighbours: words j - 1 + par and j + par
        const uint32_t l = par ? e4(M, u) : (u == 0 ? halo : e4(M, u - 1));
        const uint32_t r = par ? (u == 3 ? halo : e4(M, u + 1)) : e4(M, u);
        const uint32_t up = e4(U, u), dn = e4(Dn, u);
        // agreeing neighbours per bit
        const uint32_t al = ~(s ^ l), ar = ~(s ^ r), au = ~(s ^ up), ad = ~(s ^ dn);
        const uint32_t ax[3] = {~(al | ar), al ^ ar, al & ar};
        const uint32_t ay[3] = {~(au | ad), au ^ ad, au & ad};
        // for s = +1, Sx/2 + 1 is the agreeing count; for s = -1, 2 minus it
        const uint32_t Wd = w[u];
        uint32_t fp = 0u, fn = 0u;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const uint32_t m = ax[i] & ay[j];
                const int cp = 9 + 3 * i + j, cn = 3 * (2 - i) + (2 - j);
                fp |= (Wd <= tm1[cp] && !never[cp]) ? m : 0u;
                fn |= (Wd <= tm1[cn] && !never[cn]) ? m : 0u;
            }
        nv[u] = s ^ ((s & fp) | (~s & fn));
    }
    *reinterpret_cast<uint4*>(own + (size_t)y * W + j0) = make_uint4(nv[0], nv[1], nv[2], nv[3]);
}

// Per bit b: M = 2 ones - N, Bx = N - 2 (ones of s ^ right), By likewise;
// wave ballots count the bits, one LDS atomic per wave, bit and statistic.
__global__ void __launch_bounds__(256) k_msc_stats(MscArgs a, int rec_row) {
    __shared__ int cnt[3][32];
    const int g = blockIdx.y;
    const RepDev D = a.reps[g];
    const int Lx = D.Lx, Ly = D.Ly, n = Lx * Ly;
    if (threadIdx.x < 96) (&cnt[0][0])[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t* lat =
        reinterpret_cast<const uint32_t*>(reinterpret_cast<const uint8_t*>(a.lat) + D.lat_off);
    for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
        const int i = base + threadIdx.x;
        uint32_t s = 0u, xr = 0u, xd = 0u;
        const bool in = i < n;
        if (in) {
            const int y = i / Lx, x = i - y * Lx;
            s = lat[plane_word(y, x, Lx, Ly)];
            xr = s ^ lat[plane_word(y, x + 1 == Lx ? 0 : x + 1, Lx, Ly)];
            xd = s ^ lat[plane_word(y + 1 == Ly ? 0 : y + 1, x, Lx, Ly)];
        }
        for (int bit = 0; bit < 32; ++bit) {
            const int c0 = __popcll(__ballot(in && ((s >> bit) & 1u)));
            const int c1 = __popcll(__ballot(in && ((xr >> bit) & 1u)));
            const int c2 = __popcll(__ballot(in && ((xd >> bit) & 1u)));
            if ((threadIdx.x & 63) == 0) {
                atomicAdd(&cnt[0][bit], c0);
                atomicAdd(&cnt[1][bit], c1);
                atomicAdd(&cnt[2][bit], c2);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < 32) {
        const int bit = threadIdx.x;
        int32_t* row = a.stats + ((size_t)rec_row * (32 * a.G) + 32 * g + bit) * a.width;
        // partial counts of this workgroup; every workgroup adds its share of
        // 2 ones - N as 2 ones - n_visited
        int visited = 0;
        for (int base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x)
            visited += min((int)blockDim.x, n - base);
        atomicAdd(&row[0], 2 * cnt[0][bit] - visited);
        atomicAdd(&row[1], visited - 2 * cnt[1][bit]);
        atomicAdd(&row[2], visited - 2 * cnt[2][bit]);
    }
}

hipError_t launch_msc_init(const MscArgs& a, hipStream_t s) {
    const int nq = (a.max_sites + 3) / 4;
    hipLaunchKernelGGL(k_msc_init, dim3((nq + 255) / 256, a.G), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_msc_pass(const MscArgs& a, int c, int sweep_off, hipStream_t s) {
    hipLaunchKernelGGL(k_msc_pass4, dim3((a.max_blocks + 255) / 256, a.G), dim3(256), 0, s, a, c,
                       sweep_off);
    return hipGetLastError();
}

hipError_t launch_msc_stats(const MscArgs& a, int rec_row, hipStream_t s) {
    const int per = (a.max_sites + 255) / 256;
    hipLaunchKernelGGL(k_msc_stats, dim3(per < 64 ? per : 64, a.G), dim3(256), 0, s, a, rec_row);
    return hipGetLastError();
}

}  // namespace spinmc

// Triangular-lattice Ising (the triangular kernels of the Methods): the
// checkerboard Metropolis chain of Algorithm 1 on the six-neighbour lattice.
//
// Sites sit on an Ly x Lx lattice of int8 spins; the neighbours of (y, x)
// are (y, x+-1), (y+-1, x), (y-1, x+1) and (y+1, x-1) (periodic), one
// coupling J for every bond, H = -J sum s s' - h sum s.  Three colours
// c = (x + 2y) mod 3 -- no bond joins two sites of one colour when Lx and Ly
// are multiples of 3 -- make a sweep of three passes p = 3t + c.  The sites
// of colour c in row y are x = 3i + (c + y) mod 3; on the device each colour
// has a plane of Ly rows of Lx/3 bytes, site (y, x) at byte (y, x / 3) of
// plane (x + 2y) mod 3, so that byte k of plane c is the site with
// within-colour index k = y Lx/3 + i.  It selects word k & 3 of Philox4x32-10
// block (k >> 2, p, rid, 0), used whole as W; the flip is accepted iff
// W < T[7 [s > 0] + (S6 + 6) / 2] with the FP64 host thresholds
// T = ceil(2^32 exp(-beta 2 s (J S6 + h))) (2^32 when that change is <= 0).
// A lane takes the four sites of one Philox block.
#include "tri_internal.hpp"

namespace spinmc {

namespace {
constexpr uint32_t kTriTagMain = 0u, kTriTagInit = 2u;

__device__ __forceinline__ int wrapt(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Byte of site (y, x) of a triangular lattice in its colour planes.
__device__ __forceinline__ size_t tri_byte(int y, int x, int Lx, int Ly) {
    const size_t W3 = (size_t)(Lx / 3);
    return (size_t)((x + 2 * y) % 3) * Ly * W3 + (size_t)y * W3 + (size_t)(x / 3);
}

// Chain / square / cubic lattices sit in two colour planes on the device:
// site (z, y, x) of row z Ly + y is byte (row, x >> 1) of plane
// (x + y + z) & 1, each plane Ly Lz rows of W = Lx / 2 bytes.  The byte's
// offset in its plane is the site's within-colour index k = (row Lx + x) >> 1.
__device__ __forceinline__ size_t hc_byte(int z, int y, int x, int Lx, int Ly, int Lz) {
    const size_t W = (size_t)(Lx >> 1);
    return (size_t)((x + y + z) & 1) * Ly * Lz * W + ((size_t)z * Ly + y) * W + (x >> 1);
}
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
    for (int u = 0; u < 4; ++u) {
        const int i = 4 * b + u;
        if (i >= n) break;
        const int8_t v = w[u] < 0x80000000u ? (int8_t)1 : (int8_t)-1;
        if (D.model == kModelIsingHC) {
            const int row = i / D.Lx, x = i - row * D.Lx, z = row / D.Ly;
            lat[hc_byte(z, row - z * D.Ly, x, D.Lx, D.Ly, D.q)] = v;
        } else {
            const int y = i / D.Lx;
            lat[tri_byte(y, i - y * D.Lx, D.Lx, D.Ly)] = v;
        }
    }
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
        const int s = lat[(size_t)c * nk + k];
        const int S6 = lat[tri_byte(y, xl, Lx, Ly)] + lat[tri_byte(y, xr, Lx, Ly)] +
                       lat[tri_byte(yu, x, Lx, Ly)] + lat[tri_byte(yd, x, Lx, Ly)] +
                       lat[tri_byte(yu, xr, Lx, Ly)] + lat[tri_byte(yd, xl, Lx, Ly)];
        const int idx = 7 * (s > 0) + (S6 + 6) / 2;
        if ((uint64_t)w[u] < lt[idx]) lat[(size_t)c * nk + k] = (int8_t)(-s);
    }
}

// Span form of a pass (four sites of one Philox block per lane, byte
// arithmetic in 32-bit words).  A spin byte is 0x01 (+1) or 0xFF (-1), so
// v & 0x02020202 flags the -1 bytes of a word as 2 per byte.  Sums of such
// flags stay below 16 per byte (at most six neighbours), so whole words add
// without carries between bytes: one add chain gives 2n, n the number of -1
// neighbours, at every byte position of a span.  The threshold class
// 7 [s > 0] + (S + 6) / 2 (S the neighbour sum over the k neighbours present,
// S = k - 2n) is then keyed by j = n + 8 [s < 0], read from a 16-entry table.
namespace {
constexpr uint32_t kNegFlag = 0x02020202u;

__device__ __forceinline__ uint32_t abyte(uint32_t hi, uint32_t lo, uint32_t sel) {
    return __builtin_amdgcn_alignbyte(hi, lo, sel);  // ({hi, lo} >> 8 sel)[31:0]
}

// entry j = n + 8 neg of the keyed table from the 14 classes, k neighbours
__device__ __forceinline__ uint64_t keyed_threshold(const uint64_t* tab, int j, int k) {
    const int n = j & 7, neg = j >> 3;
    return n > k ? 0ull : tab[7 * (1 - neg) + (k + 6) / 2 - n];
}

// Triangular: S, U, Dn are the 12-byte spans [x0, x0 + 12) of rows y, y - 1,
// y + 1; the own sites are x0 + xc + 3u.  hl = flags of (y, x0 - 1) and
// (y + 1, x0 - 1) added, hr = those of (y, x0 + 12) and (y - 1, x0 + 12).
// Neighbour flags at position o: S[o -+ 1], U[o], U[o + 1], Dn[o], Dn[o - 1],
// i.e. (S + Dn) moved up one byte position, (S + U) moved down one, U + Dn
// in place.  A funnel shift by xc bytes brings the own sites to byte
// positions 0, 3, 6, 9; their flips are shifted back.  Bytes of other
// positions may read values another lane is writing: they never reach an
// own site's count.
__device__ __forceinline__ void tri_span(uint32_t (&S)[3], const uint32_t (&U)[3],
                                         const uint32_t (&Dn)[3], uint32_t hl, uint32_t hr,
                                         uint32_t xc, const uint32_t (&w)[4],
                                         const uint64_t* lt) {
    uint32_t m[4], A[3], B[3], C[4];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        m[i] = S[i] & kNegFlag;
        const uint32_t mu = U[i] & kNegFlag, md = Dn[i] & kNegFlag;
        A[i] = m[i] + md;
        B[i] = m[i] + mu;
        C[i] = mu + md;
    }
    m[3] = 0u;
    C[0] += abyte(A[0], hl << 24, 3) + abyte(B[1], B[0], 1);
    C[1] += abyte(A[1], A[0], 3) + abyte(B[2], B[1], 1);
    C[2] += abyte(A[2], A[1], 3) + abyte(hr, B[2], 1);
    C[3] = 0u;
    // key bytes 2n + 16 [s < 0] with the own sites at bytes 0, 3, 6, 9
    uint32_t K[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) K[i] = abyte(C[i + 1], C[i], xc) | (abyte(m[i + 1], m[i], xc) << 3);
    const bool f0 = (uint64_t)w[0] < lt[(K[0] >> 1) & 15u];
    const bool f1 = (uint64_t)w[1] < lt[(K[0] >> 25) & 15u];
    const bool f2 = (uint64_t)w[2] < lt[(K[1] >> 17) & 15u];
    const bool f3 = (uint64_t)w[3] < lt[(K[2] >> 9) & 15u];
    // a flip negates the byte: s -> -s is s ^ 0xFE for s = +-1
    const uint32_t F0 = (f0 ? 0xFEu : 0u) | (f1 ? 0xFE000000u : 0u);
    const uint32_t F1 = f2 ? 0x00FE0000u : 0u;
    const uint32_t F2 = f3 ? 0x0000FE00u : 0u;
    if (xc == 0u) {
        S[0] ^= F0;
        S[1] ^= F1;
        S[2] ^= F2;
    } else {
        const uint32_t sh = 4u - xc;  // a left shift by xc bytes
        S[0] ^= abyte(F0, 0u, sh);
        S[1] ^= abyte(F1, F0, sh);
        S[2] ^= abyte(F2, F1, sh);
    }
}

// Chain / square / cubic in natural layout (the lattice the LDS-resident
// kernel holds): S the 8-byte span [x0, x0 + 8) of the own row, the own
// sites x0 + 2u + par; N0, N1 the added flags of the neighbouring rows and
// planes over the span; hl, hr the flags of (x0 - 1) and (x0 + 8).
__device__ __forceinline__ void hc_span(uint32_t (&S)[2], uint32_t N0, uint32_t N1, uint32_t hl,
                                        uint32_t hr, uint32_t par, const uint32_t (&w)[4],
                                        const uint64_t* lt) {
    const uint32_t m0 = S[0] & kNegFlag, m1 = S[1] & kNegFlag;
    const uint32_t K0 = (N0 + abyte(m0, hl << 24, 3) + abyte(m1, m0, 1)) | (m0 << 3);
    const uint32_t K1 = (N1 + abyte(m1, m0, 3) + abyte(hr, m1, 1)) | (m1 << 3);
    const uint32_t o0 = 8u * par, o1 = 16u + 8u * par;  // bit offsets of the own bytes
    const bool f0 = (uint64_t)w[0] < lt[(K0 >> (o0 + 1u)) & 15u];
    const bool f1 = (uint64_t)w[1] < lt[(K0 >> (o1 + 1u)) & 15u];
    const bool f2 = (uint64_t)w[2] < lt[(K1 >> (o0 + 1u)) & 15u];
    const bool f3 = (uint64_t)w[3] < lt[(K1 >> (o1 + 1u)) & 15u];
    const uint32_t e0 = 0xFEu << o0, e1 = 0xFEu << o1;
    S[0] ^= (f0 ? e0 : 0u) | (f1 ? e1 : 0u);
    S[1] ^= (f2 ? e0 : 0u) | (f3 ? e1 : 0u);
}

// Chain / square / cubic on the colour planes: S the four own bytes (plane
// bytes j0 .. j0 + 3 of a row, own sites x = 2 j + par), N the added -1 flags
// of the vertical partners (the other plane's rows y +- 1 and z +- 1, same
// bytes), M the other plane's word of the same row and hf the -1 flag of its
// halo byte (j0 - 1 for par = 0, j0 + 4 for par = 1): the horizontal partners
// of own byte j are the other plane's bytes j - 1 + par and j + par.
__device__ __forceinline__ uint32_t hc_word(uint32_t S, uint32_t N, uint32_t M, uint32_t hf,
                                            uint32_t par, const uint32_t (&w)[4],
                                            const uint64_t* lt) {
    const uint32_t mf = M & kNegFlag;
    const uint32_t H = mf + (par ? abyte(hf, mf, 1) : abyte(mf, hf << 24, 3));
    const uint32_t K = (N + H) | ((S & kNegFlag) << 3);  // 2n + 16 [s < 0] per byte
    uint32_t F = 0u;
#pragma unroll
    for (int u = 0; u < 4; ++u)
        F |= (uint64_t)w[u] < lt[(K >> (8 * u + 1)) & 15u] ? 0xFEu << (8 * u) : 0u;
    return S ^ F;  // a flip negates the byte: s -> -s is s ^ 0xFE for s = +-1
}

// b / d for 0 <= b < 2^22, d >= 1: the FP32 estimate b (1/d) is within one
// of the quotient there (relative error below 2^-22), one correction each way
__device__ __forceinline__ int qdiv(int b, int d, bool small) {
    if (!small) return b / d;
    int q = (int)((float)b * __builtin_amdgcn_rcpf((float)d));
    const int rem = b - (int)__umul24((uint32_t)q, (uint32_t)d);
    q += rem >= d ? 1 : 0;
    q -= rem < 0 ? 1 : 0;
    return q;
}

// Workgroup w of a 1-D grid of n runs on XCD w mod 8 (round-robin
// dispatch); the logical index (w mod 8) n/8 + w/8 keeps consecutive logical
// workgroups -- neighbouring spans of one replica -- on one XCD and its L2.
__device__ __forceinline__ int xcd_logical(int w, int n) {
    return (n & 7) ? w : (w & 7) * (n >> 3) + (w >> 3);
}

__device__ __forceinline__ uint32_t ld32(const int8_t* p) { return *reinterpret_cast<const uint32_t*>(p); }
__device__ __forceinline__ uint2 ld64(const int8_t* p) { return *reinterpret_cast<const uint2*>(p); }
__device__ __forceinline__ uint32_t negflag(const int8_t* p) { return (uint32_t)(uint8_t)*p & 2u; }
}  // namespace

// Lx a multiple of 12: the four sites of a Philox block are four consecutive
// bytes i0 .. i0 + 3 of row y of plane c (planes of W3 = Lx / 3 bytes per
// row).  With r = (c + y) mod 3 the six neighbours of own byte i are, in
// plane c + 1: row y at i + [r = 2] (x + 1), row y - 1 at i (y - 1, x) and
// row y + 1 at i - [r = 0] (y + 1, x - 1); in plane c + 2: row y at
// i - [r = 0] (x - 1), row y + 1 at i (y + 1, x) and row y - 1 at
// i + [r = 2] (y - 1, x + 1) -- six dwords, two of them with a halo byte
// on the side of the shift.  Only the own dword is stored.  A lane takes NB
// Philox blocks, 256 apart (a wave's loads of one block index stay
// contiguous), their loads all in flight together: NB = 2 for large passes
// (see launch_tri_pass), 1 otherwise.  The grid is 1-D: gx workgroups per
// replica, replica-major in logical order.
template <int NB>
__global__ void __launch_bounds__(256) k_tri_pass4(TriArgs a, int c, int sweep_off, int gx) {
    __shared__ uint64_t lt[16];
    const int wl = xcd_logical((int)blockIdx.x, (int)gridDim.x);
    const int r = wl / gx, wx = wl - r * gx;
    const RepDev D = a.reps[r];
    const int Lx = D.Lx, Ly = D.Ly, W3 = Lx / 3, qpr = W3 >> 2, nb = Ly * qpr;
    const int bt = NB * wx * 256 + (int)threadIdx.x;  // block k: bt + 256 k
    if (NB * wx * 256 >= nb) return;  // whole workgroup past the end
    const bool small = nb < (1 << 22);
    // 32-bit offsets from the replica's base (a lattice below 2^31 bytes)
    const uint32_t psz = (uint32_t)Ly * (uint32_t)W3;  // bytes per plane
    const int cp = c == 2 ? 0 : c + 1, cm = c == 0 ? 2 : c - 1;
    int8_t* own = a.lat + D.lat_off + (uint32_t)c * psz;
    const int8_t* pp = a.lat + D.lat_off + (uint32_t)cp * psz;
    const int8_t* pm = a.lat + D.lat_off + (uint32_t)cm * psz;
    // blocks past the end compute the last block and store nothing (every
    // lane reaches the barrier)
    uint32_t S[NB], N[NB], off[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int b = bt + 256 * k < nb ? bt + 256 * k : nb - 1;
        const int y = qdiv(b, qpr, small);
        const int i0 = 4 * (b - (int)__umul24((uint32_t)y, (uint32_t)qpr));
        const int yu = y == 0 ? Ly - 1 : y - 1, yd = y + 1 == Ly ? 0 : y + 1;
        const uint32_t o = __umul24((uint32_t)y, (uint32_t)W3);
        const uint32_t ou = __umul24((uint32_t)yu, (uint32_t)W3);
        const uint32_t od = __umul24((uint32_t)yd, (uint32_t)W3);
        const int rr = (c + y) % 3;
        off[k] = o + (uint32_t)i0;
        S[k] = ld32(own + off[k]);
        const uint32_t fa = ld32(pp + off[k]) & kNegFlag;           // (y, x + 1)
        const uint32_t fb = ld32(pp + (ou + i0)) & kNegFlag;        // (y - 1, x)
        const uint32_t fc = ld32(pp + (od + i0)) & kNegFlag;        // (y + 1, x - 1)
        const uint32_t fd = ld32(pm + off[k]) & kNegFlag;           // (y, x - 1)
        const uint32_t fe = ld32(pm + (od + i0)) & kNegFlag;        // (y + 1, x)
        const uint32_t ff = ld32(pm + (ou + i0)) & kNegFlag;        // (y - 1, x + 1)
        // halo bytes: r = 2 shifts (y, x + 1) and (y - 1, x + 1) by one byte
        // up (byte i0 + 4), r = 0 shifts (y + 1, x - 1) and (y, x - 1) down
        // (byte i0 - 1); r = 1 needs neither
        const int ir = i0 + 4 == W3 ? 0 : i0 + 4, il = i0 == 0 ? W3 - 1 : i0 - 1;
        const uint32_t h1 = negflag(rr == 2 ? pp + (o + ir) : pp + (od + il));
        const uint32_t h2 = negflag(rr == 2 ? pm + (ou + ir) : pm + (o + il));
        const uint32_t sa = rr == 2 ? abyte(h1, fa, 1) : fa;
        const uint32_t sf = rr == 2 ? abyte(h2, ff, 1) : ff;
        const uint32_t sc = rr == 0 ? abyte(fc, h1 << 24, 3) : fc;
        const uint32_t sd = rr == 0 ? abyte(fd, h2 << 24, 3) : fd;
        N[k] = sa + fb + sc + sd + fe + sf;  // 2n per byte, n <= 6 -1 neighbours
    }
    const uint64_t t = *a.t_base + (uint64_t)sweep_off;
    const uint32_t p = (uint32_t)(3 * t + (uint64_t)c);
    uint32_t w[NB][4];
#pragma unroll
    for (int k = 0; k < NB; ++k)
        philox4x32_10((uint32_t)(bt + 256 * k), p, D.rid, kTriTagMain, a.key0, a.key1, w[k]);
    // the table after the loads and the random words: its latency overlaps theirs
    if (threadIdx.x < 16)
        lt[threadIdx.x] = keyed_threshold(a.tab + (size_t)r * kTriClasses, threadIdx.x, 6);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const uint32_t K = N[k] | ((S[k] & kNegFlag) << 3);  // 2n + 16 [s < 0] per byte
        uint32_t F = 0u;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            F |= (uint64_t)w[k][u] < lt[(K >> (8 * u + 1)) & 15u] ? 0xFEu << (8 * u) : 0u;
        if (bt + 256 * k < nb) *reinterpret_cast<uint32_t*>(own + off[k]) = S[k] ^ F;
    }
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
        const int s = lat[tri_byte(y, x, Lx, Ly)];
        M += s;
        Bh += s * lat[tri_byte(y, xr, Lx, Ly)];
        Bv += s * lat[tri_byte(yd, x, Lx, Ly)];
        Bd += s * lat[tri_byte(yd, xl, Lx, Ly)];
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

// Chain / square / simple cubic (Lz = D.q) on the colour planes: the
// colour-c site with within-colour index k -- byte k of plane c -- for the
// four k of a Philox block; neighbours x +- 1 and, where the extent exceeds
// 1, y +- 1 and z +- 1, all in the other plane.
__global__ void __launch_bounds__(256) k_hc_pass(TriArgs a, int c, int sweep_off) {
    __shared__ uint64_t lt[kTriClasses];
    const int r = blockIdx.y;
    if (threadIdx.x < kTriClasses) lt[threadIdx.x] = a.tab[(size_t)r * kTriClasses + threadIdx.x];
    __syncthreads();
    const RepDev D = a.reps[r];
    const int Lx = D.Lx, Ly = D.Ly, Lz = D.q, W = Lx >> 1;
    const int nk = Ly * Lz * W;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * b >= nk) return;
    const uint64_t t = *a.t_base + (uint64_t)sweep_off;
    const uint32_t p = (uint32_t)(2 * t + (uint64_t)c);
    uint32_t w[4];
    philox4x32_10((uint32_t)b, p, D.rid, kTriTagMain, a.key0, a.key1, w);
    int8_t* own = a.lat + D.lat_off + (size_t)c * nk;
    const int8_t* oth = a.lat + D.lat_off + (size_t)(1 - c) * nk;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int k = 4 * b + u;
        if (k >= nk) break;
        const int row = k / W, j = k - row * W;  // row = z Ly + y
        const int z = row / Ly, y = row - z * Ly;
        const int x = 2 * j + ((c + y + z) & 1);
        const size_t rb = (size_t)row * W;
        const int s = own[k];
        int S = oth[rb + (wrapt(x - 1, Lx) >> 1)] + oth[rb + (wrapt(x + 1, Lx) >> 1)];
        if (Ly > 1)
            S += oth[(size_t)(z * Ly + wrapt(y - 1, Ly)) * W + j] +
                 oth[(size_t)(z * Ly + wrapt(y + 1, Ly)) * W + j];
        if (Lz > 1)
            S += oth[(size_t)(wrapt(z - 1, Lz) * Ly + y) * W + j] +
                 oth[(size_t)(wrapt(z + 1, Lz) * Ly + y) * W + j];
        const int idx = 7 * (s > 0) + (S + 6) / 2;
        if ((uint64_t)w[u] < lt[idx]) own[k] = (int8_t)(-s);
    }
}

// Lx a multiple of 8: the four sites of a Philox block are four consecutive
// bytes j0 .. j0 + 3 of a row of plane c (plane rows of W = Lx / 2 bytes, so
// a row holds W / 4 blocks); the other plane's word of the same row plus one
// halo byte, and its words of rows y +- 1 and z +- 1, come in as dwords, and
// only the own word is stored.  A lane takes NB Philox blocks, 256 apart, as
// k_tri_pass4.
template <int NB>
__global__ void __launch_bounds__(256) k_hc_pass4(TriArgs a, int c, int sweep_off, int gx) {
    __shared__ uint64_t lt[16];
    const int wl = xcd_logical((int)blockIdx.x, (int)gridDim.x);  // see k_tri_pass4
    const int r = wl / gx, wx = wl - r * gx;
    const RepDev D = a.reps[r];
    const int Lx = D.Lx, Ly = D.Ly, Lz = D.q, W = Lx >> 1, qpr = W >> 2;
    const int nb = Ly * Lz * qpr;  // Philox blocks per pass: Lx Ly Lz / 8
    const int bt = NB * wx * 256 + (int)threadIdx.x;  // block k: bt + 256 k
    if (NB * wx * 256 >= nb) return;  // whole workgroup past the end
    const bool small = nb < (1 << 22);
    // 32-bit offsets from the replica's base (a lattice below 2^31 bytes)
    const uint32_t psz = (uint32_t)(Ly * Lz) * (uint32_t)W;  // bytes per plane
    int8_t* own = a.lat + D.lat_off + (c ? psz : 0u);
    const int8_t* oth = a.lat + D.lat_off + (c ? 0u : psz);
    uint32_t S[NB], N[NB], M[NB], hf[NB], off[NB], par[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int b = bt + 256 * k < nb ? bt + 256 * k : nb - 1;  // see k_tri_pass4
        const int row = qdiv(b, qpr, small);  // z Ly + y
        const int j0 = 4 * (b - (int)__umul24((uint32_t)row, (uint32_t)qpr));
        const int z = qdiv(row, Ly, small), y = row - (int)__umul24((uint32_t)z, (uint32_t)Ly);
        const uint32_t ro = (uint32_t)row * (uint32_t)W;
        off[k] = ro + (uint32_t)j0;
        par[k] = (uint32_t)((c + y + z) & 1);
        S[k] = ld32(own + off[k]);
        M[k] = ld32(oth + off[k]);
        const int hb = par[k] ? (j0 + 4 == W ? 0 : j0 + 4) : (j0 == 0 ? W - 1 : j0 - 1);
        hf[k] = negflag(oth + (ro + (uint32_t)hb));
        N[k] = 0u;
        if (Ly > 1) {
            const uint32_t zr = (uint32_t)(z * Ly);
            N[k] += (ld32(oth + ((zr + wrapt(y - 1, Ly)) * (uint32_t)W + j0)) & kNegFlag) +
                    (ld32(oth + ((zr + wrapt(y + 1, Ly)) * (uint32_t)W + j0)) & kNegFlag);
        }
        if (Lz > 1) {
            N[k] += (ld32(oth + ((uint32_t)(wrapt(z - 1, Lz) * Ly + y) * (uint32_t)W + j0)) & kNegFlag) +
                    (ld32(oth + ((uint32_t)(wrapt(z + 1, Lz) * Ly + y) * (uint32_t)W + j0)) & kNegFlag);
        }
    }
    const uint64_t t = *a.t_base + (uint64_t)sweep_off;
    const uint32_t p = (uint32_t)(2 * t + (uint64_t)c);
    uint32_t w[NB][4];
#pragma unroll
    for (int k = 0; k < NB; ++k)
        philox4x32_10((uint32_t)(bt + 256 * k), p, D.rid, kTriTagMain, a.key0, a.key1, w[k]);
    if (threadIdx.x < 16)
        lt[threadIdx.x] = keyed_threshold(a.tab + (size_t)r * kTriClasses, threadIdx.x,
                                          2 + 2 * (Ly > 1) + 2 * (Lz > 1));
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const uint32_t v = hc_word(S[k], N[k], M[k], hf[k], par[k], w[k], lt);
        if (bt + 256 * k < nb) *reinterpret_cast<uint32_t*>(own + off[k]) = v;
    }
}

// [M, Bx, By, Bz] of the chain / square / cubic lattices.
__global__ void __launch_bounds__(256) k_hc_stats(TriArgs a, int rec_row) {
    const int r = blockIdx.y;
    const RepDev D = a.reps[r];
    const int Lx = D.Lx, Ly = D.Ly, Lz = D.q, n = Lx * Ly * Lz;
    const int8_t* lat = a.lat + D.lat_off;
    int M = 0, Bx = 0, By = 0, Bz = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int row = i / Lx, x = i - row * Lx;
        const int z = row / Ly, y = row - z * Ly;
        const int s = lat[hc_byte(z, y, x, Lx, Ly, Lz)];
        M += s;
        Bx += s * lat[hc_byte(z, y, wrapt(x + 1, Lx), Lx, Ly, Lz)];
        if (Ly > 1) By += s * lat[hc_byte(z, wrapt(y + 1, Ly), x, Lx, Ly, Lz)];
        if (Lz > 1) Bz += s * lat[hc_byte(wrapt(z + 1, Lz), y, x, Lx, Ly, Lz)];
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
// with its lattice in LDS in natural order (converted from the colour planes
// of global memory when loaded, and back when stored) and a barrier after
// every colour pass: the same decisions as the streamed passes, without the
// per-pass launches and lattice round trips.  Needs Lx % 12 == 0 for the
// triangular lattice (the four sites of a Philox block in one row) and
// Lx % 8 == 0 for the chain / cubic lattices.
// The statistics of k_tri_stats / k_hc_stats ([M, B1, B2, B3]) of an LDS
// lattice, this thread's share: four sites per 32-bit word.  A -1 byte has
// bit 7 set, so M = sites - 2 popc(v & 0x80808080); two +-1 bytes differ
// iff their xor is 0xFE (7 bits), so a bond sum is sites - 2 popc(v ^ w) / 7
// with w the word of the bond partners (byte funnel shifts for the x + 1
// and, on the triangular lattice, the down-left partners).
// The four sites (z, y, x0 .. x0 + 3) of natural index i = row Lx + x0
// (x0 % 4 == 0, Lx % 8 == 0) as one natural-order word, and back: sites x0
// and x0 + 2 are bytes (row, x0 / 2) and (row, x0 / 2 + 1) of plane
// (x0 + y + z) & 1, sites x0 + 1 and x0 + 3 the same bytes of the other plane.
__device__ __forceinline__ uint32_t hc_natural_word(const int8_t* lat, int i, int Lx, int Ly,
                                                    int Lz) {
    const int row = i / Lx, x0 = i - row * Lx, z = row / Ly, y = row - z * Ly;
    const size_t psz = (size_t)Ly * Lz * (Lx >> 1);
    const size_t pa = hc_byte(z, y, x0, Lx, Ly, Lz);
    const size_t pb = ((x0 + y + z) & 1) ? pa - psz : pa + psz;
    const uint32_t A = *reinterpret_cast<const uint16_t*>(lat + pa);
    const uint32_t B = *reinterpret_cast<const uint16_t*>(lat + pb);
    return __builtin_amdgcn_perm(B, A, 0x05010400u);  // bytes A0 B0 A1 B1
}

__device__ __forceinline__ void hc_store_natural_word(int8_t* lat, int i, uint32_t v, int Lx,
                                                      int Ly, int Lz) {
    const int row = i / Lx, x0 = i - row * Lx, z = row / Ly, y = row - z * Ly;
    const size_t psz = (size_t)Ly * Lz * (Lx >> 1);
    const size_t pa = hc_byte(z, y, x0, Lx, Ly, Lz);
    const size_t pb = ((x0 + y + z) & 1) ? pa - psz : pa + psz;
    *reinterpret_cast<uint16_t*>(lat + pa) = (uint16_t)__builtin_amdgcn_perm(0u, v, 0x0C0C0200u);
    *reinterpret_cast<uint16_t*>(lat + pb) = (uint16_t)__builtin_amdgcn_perm(0u, v, 0x0C0C0301u);
}

// The same for the triangular planes: sites (y, x0 .. x0 + 3), byte by byte.
__device__ __forceinline__ uint32_t tri_natural_word(const int8_t* lat, int i, int Lx, int Ly) {
    const int y = i / Lx, x0 = i - y * Lx;
    uint32_t v = 0u;
#pragma unroll
    for (int u = 0; u < 4; ++u) v |= (uint32_t)(uint8_t)lat[tri_byte(y, x0 + u, Lx, Ly)] << (8 * u);
    return v;
}

__device__ __forceinline__ void tri_store_natural_word(int8_t* lat, int i, uint32_t v, int Lx,
                                                       int Ly) {
    const int y = i / Lx, x0 = i - y * Lx;
#pragma unroll
    for (int u = 0; u < 4; ++u) lat[tri_byte(y, x0 + u, Lx, Ly)] = (int8_t)(v >> (8 * u));
}

template <int MODEL>
__device__ __forceinline__ int4 nat_stats(const int8_t* ls, int Lx, int Ly, int Lz) {
    const int plane = Lx * Ly, nq = (plane * Lz) >> 2;
    int cnt = 0;
    uint32_t pm = 0, p1 = 0, p2 = 0, p3 = 0;
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
        const int i = 4 * q;
        const int row = qdiv(i, Lx, true), x0 = i - row * Lx;  // i < 2^16
        const uint32_t v = ld32(ls + i);
        const uint32_t nx = ld32(ls + row * Lx + (x0 + 4 == Lx ? 0 : x0 + 4));
        pm += __popc(v & 0x80808080u);
        p1 += __popc(v ^ abyte(nx, v, 1));
        if (MODEL == kModelIsingTri) {
            const int yd = row + 1 == Ly ? 0 : row + 1;
            const uint32_t d = ld32(ls + yd * Lx + x0);
            const uint32_t dp = ld32(ls + yd * Lx + (x0 == 0 ? Lx - 4 : x0 - 4));
            p2 += __popc(v ^ d);
            p3 += __popc(v ^ abyte(d, dp, 3));
        } else {
            const int z = qdiv(row, Ly, true), y = row - z * Ly;
            if (Ly > 1) p2 += __popc(v ^ ld32(ls + (z * Ly + (y + 1 == Ly ? 0 : y + 1)) * Lx + x0));
            if (Lz > 1) p3 += __popc(v ^ ld32(ls + (z + 1 == Lz ? 0 : z + 1) * plane + y * Lx + x0));
        }
        cnt += 4;
    }
    const bool has2 = MODEL == kModelIsingTri || Ly > 1, has3 = MODEL == kModelIsingTri || Lz > 1;
    return make_int4(cnt - 2 * (int)pm, cnt - 2 * (int)(p1 / 7), has2 ? cnt - 2 * (int)(p2 / 7) : 0,
                     has3 ? cnt - 2 * (int)(p3 / 7) : 0);
}

// REC (re > 0): after sweep sw0 + sw + 1 = k re of the call the statistics
// of the LDS lattice go to stats row k - 1 (columns 0..3; the caller zeroes
// the rows).  The rows of the launch gather in LDS behind the lattice (LDS
// atomics of the waves) and are stored once at its end, so no sweep waits
// for global memory.
template <int MODEL, bool REC>
__global__ void __launch_bounds__(1024) k_nat_resident(TriArgs a, int n_sweeps, int sw0, int re) {
    extern __shared__ __align__(16) int8_t ls[];
    __shared__ uint64_t lt[16];
    const int r = blockIdx.x;
    const RepDev D = a.reps[r];
    const int Lx = D.Lx, Ly = D.Ly, Lz = MODEL == kModelIsingHC ? D.q : 1;
    const int n = Lx * Ly * Lz;
    int8_t* lat = a.lat + D.lat_off;
    if (threadIdx.x < 16)
        lt[threadIdx.x] = keyed_threshold(
            a.tab + (size_t)r * kTriClasses, threadIdx.x,
            MODEL == kModelIsingHC ? 2 + 2 * (Ly > 1) + 2 * (Lz > 1) : 6);
    for (int i = threadIdx.x; i < n / 4; i += blockDim.x)
        reinterpret_cast<uint32_t*>(ls)[i] = MODEL == kModelIsingHC
                                                 ? hc_natural_word(lat, 4 * i, Lx, Ly, Lz)
                                                 : tri_natural_word(lat, 4 * i, Lx, Ly);
    // recorded rows rec0 .. rec0 + n_rows - 1 (1-based) of this launch
    int* lrec = reinterpret_cast<int*>(ls + ((n + 15) & ~15));
    const int rec0 = REC ? sw0 / re + 1 : 0;
    const int n_rows = REC ? (sw0 + n_sweeps) / re - sw0 / re : 0;
    for (int i = threadIdx.x; i < 4 * n_rows; i += blockDim.x) lrec[i] = 0;
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
                    const int y = qdiv(b, G, true), x0 = 12 * (b - y * G);  // b < 2^16
                    const int yu = y == 0 ? Ly - 1 : y - 1, yd = y + 1 == Ly ? 0 : y + 1;
                    const int xl = x0 == 0 ? Lx - 1 : x0 - 1, xr = x0 + 12 == Lx ? 0 : x0 + 12;
                    int8_t* row = ls + y * Lx;
                    const int8_t* up = ls + yu * Lx;
                    const int8_t* dn = ls + yd * Lx;
                    uint32_t S[3] = {ld32(row + x0), ld32(row + x0 + 4), ld32(row + x0 + 8)};
                    const uint32_t U[3] = {ld32(up + x0), ld32(up + x0 + 4), ld32(up + x0 + 8)};
                    const uint32_t Dn[3] = {ld32(dn + x0), ld32(dn + x0 + 4), ld32(dn + x0 + 8)};
                    const uint32_t hl = negflag(row + xl) + negflag(dn + xl);
                    const uint32_t hr = negflag(row + xr) + negflag(up + xr);
                    tri_span(S, U, Dn, hl, hr, (uint32_t)((c + y) % 3), w, lt);
                    uint32_t* rw = reinterpret_cast<uint32_t*>(row + x0);
                    rw[0] = S[0];
                    rw[1] = S[1];
                    rw[2] = S[2];
                } else {
                    const int row = qdiv(8 * b, Lx, true);  // 8 b < 2^16
                    const int z = qdiv(row, Ly, true), y = row - z * Ly;
                    const int x0 = 8 * b - row * Lx;
                    int8_t* own = ls + row * Lx + x0;
                    const uint2 S2 = ld64(own);
                    uint32_t S[2] = {S2.x, S2.y};
                    const uint32_t hl = negflag(ls + row * Lx + (x0 == 0 ? Lx - 1 : x0 - 1));
                    const uint32_t hr = negflag(ls + row * Lx + (x0 + 8 == Lx ? 0 : x0 + 8));
                    uint32_t N0 = 0u, N1 = 0u;
                    if (Ly > 1) {
                        const uint2 vu = ld64(ls + (z * Ly + (y == 0 ? Ly - 1 : y - 1)) * Lx + x0);
                        const uint2 vd = ld64(ls + (z * Ly + (y + 1 == Ly ? 0 : y + 1)) * Lx + x0);
                        N0 += (vu.x & kNegFlag) + (vd.x & kNegFlag);
                        N1 += (vu.y & kNegFlag) + (vd.y & kNegFlag);
                    }
                    if (Lz > 1) {
                        const int ip = y * Lx + x0;
                        const uint2 vu = ld64(ls + (z == 0 ? Lz - 1 : z - 1) * plane + ip);
                        const uint2 vd = ld64(ls + (z + 1 == Lz ? 0 : z + 1) * plane + ip);
                        N0 += (vu.x & kNegFlag) + (vd.x & kNegFlag);
                        N1 += (vu.y & kNegFlag) + (vd.y & kNegFlag);
                    }
                    hc_span(S, N0, N1, hl, hr, (uint32_t)((c + y + z) & 1), w, lt);
                    *reinterpret_cast<uint2*>(own) = make_uint2(S[0], S[1]);
                }
            }
            __syncthreads();
        }
        if (REC && (sw0 + sw + 1) % re == 0) {
            int4 st = nat_stats<MODEL>(ls, Lx, Ly, Lz);
            // wave sums over the active lanes (every wave of the workgroup is
            // full and has reconverged after the loop)
            st.x = __ockl_wfred_add_i32(st.x);
            st.y = __ockl_wfred_add_i32(st.y);
            st.z = __ockl_wfred_add_i32(st.z);
            st.w = __ockl_wfred_add_i32(st.w);
            if ((threadIdx.x & 63) == 0) {
                int* row = lrec + 4 * ((sw0 + sw + 1) / re - rec0);
                atomicAdd(&row[0], st.x);
                atomicAdd(&row[1], st.y);
                atomicAdd(&row[2], st.z);
                atomicAdd(&row[3], st.w);
            }
            __syncthreads();  // the next sweep writes the lattice
        }
    }
    if (REC)
        for (int i = threadIdx.x; i < 4 * n_rows; i += blockDim.x)
            a.stats[((size_t)(rec0 - 1 + (i >> 2)) * a.R + r) * a.width + (i & 3)] = lrec[i];
    for (int i = threadIdx.x; i < n / 4; i += blockDim.x) {
        const uint32_t v = reinterpret_cast<const uint32_t*>(ls)[i];
        if (MODEL == kModelIsingHC)
            hc_store_natural_word(lat, 4 * i, v, Lx, Ly, Lz);
        else
            tri_store_natural_word(lat, 4 * i, v, Lx, Ly);
    }
}

hipError_t launch_nat_resident(const TriArgs& a, int n_sweeps, int sw0, int re, int lds_bytes,
                               hipStream_t s) {
    const bool hc = a.model == kModelIsingHC, rec = re > 0;
    const void* fn = hc ? (rec ? (const void*)k_nat_resident<kModelIsingHC, true>
                               : (const void*)k_nat_resident<kModelIsingHC, false>)
                        : (rec ? (const void*)k_nat_resident<kModelIsingTri, true>
                               : (const void*)k_nat_resident<kModelIsingTri, false>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess) return e;
    if (hc && rec)
        hipLaunchKernelGGL((k_nat_resident<kModelIsingHC, true>), dim3(a.R), dim3(1024), lds_bytes,
                           s, a, n_sweeps, sw0, re);
    else if (hc)
        hipLaunchKernelGGL((k_nat_resident<kModelIsingHC, false>), dim3(a.R), dim3(1024),
                           lds_bytes, s, a, n_sweeps, sw0, re);
    else if (rec)
        hipLaunchKernelGGL((k_nat_resident<kModelIsingTri, true>), dim3(a.R), dim3(1024),
                           lds_bytes, s, a, n_sweeps, sw0, re);
    else
        hipLaunchKernelGGL((k_nat_resident<kModelIsingTri, false>), dim3(a.R), dim3(1024),
                           lds_bytes, s, a, n_sweeps, sw0, re);
    return hipGetLastError();
}

hipError_t launch_tri_init(const TriArgs& a, hipStream_t s) {
    const int nb = (a.max_sites + 3) / 4;
    hipLaunchKernelGGL(k_tri_init, dim3((nb + 255) / 256, a.R), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tri_pass(const TriArgs& a, int c, int sweep_off, hipStream_t s) {
    // two blocks per lane from 1 M blocks per pass (two for every lane the
    // chip holds at once) when a replica has at least 2048 (four workgroups of
    // 512 blocks: little lost to a ragged last one)
    const bool two = (int64_t)a.max_blocks * a.R >= (int64_t)1 << 20 && a.max_blocks >= 2048;
    const int gx1 = (a.max_blocks + 255) / 256, gx2 = (a.max_blocks + 511) / 512;
    const dim3 g1((unsigned)gx1 * a.R), g2((unsigned)gx2 * a.R);
    if (a.model == kModelIsingHC && a.all_lx8) {
        if (two)
            hipLaunchKernelGGL(k_hc_pass4<2>, g2, dim3(256), 0, s, a, c, sweep_off, gx2);
        else
            hipLaunchKernelGGL(k_hc_pass4<1>, g1, dim3(256), 0, s, a, c, sweep_off, gx1);
    } else if (a.model == kModelIsingHC)
        hipLaunchKernelGGL(k_hc_pass, dim3((a.max_blocks + 255) / 256, a.R), dim3(256), 0, s, a,
                           c, sweep_off);
    else if (a.all_lx12 && two)
        hipLaunchKernelGGL(k_tri_pass4<2>, g2, dim3(256), 0, s, a, c, sweep_off, gx2);
    else if (a.all_lx12)
        hipLaunchKernelGGL(k_tri_pass4<1>, g1, dim3(256), 0, s, a, c, sweep_off, gx1);
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

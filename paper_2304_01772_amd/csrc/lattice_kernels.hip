// Ising and q-state Potts checkerboard Metropolis kernels for gfx950.
//
// Data layout (per replica): two int8 colour planes P0, P1, each Ly rows of
// W = Lx/2 bytes; site (y, x) lives in P[(x+y)&1][y][x>>1].  Ising stores
// the spin bit u = (s + 1)/2, Potts the label.  A colour pass updates every
// byte of P_c from its own value and four neighbours in P_{1-c}: the same
// column in rows y-1, y, y+1, and column j-1 (if x is even) or j+1 (if x is
// odd) in row y.  Colour-0 sites go first (Related Work, Fig. 1: sites of one
// colour have no interacting neighbour of that colour, so the pass is
// embarrassingly parallel).
//
// The fast ("chunk") path gives each lane 16 consecutive bytes of a plane row
// (one dwordx4 load per plane row), builds neighbour sums with byte-SWAR
// arithmetic, and consumes one 16-bit Philox prefix per site for the
// Metropolis test of Algorithm 1 (Ising: 8 sites per Philox4x32-10 call;
// Potts: 16-bit proposal + 16-bit accept prefix, 4 sites per call).  The low
// 16 bits of the uniform word are drawn from the fallback stream only when
// the prefix ties the threshold's high half (probability 2^-16), so the
// result equals comparing a full 32-bit uniform word with the FP64-built
// threshold T = ceil(2^32 exp(-beta dE)).
#include "spinmc_internal.hpp"

namespace spinmc {

namespace {

__device__ __forceinline__ uint32_t sad_u8(uint32_t a, uint32_t acc) {
    return __builtin_amdgcn_sad_u8(a, 0u, acc);
}

// Wave + workgroup sum of up to 4 ints, result valid in thread 0.
template <int N>
__device__ __forceinline__ void block_sum(int (&v)[N], int* lds /* >= 16*N */) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], o, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) lds[wave * N + i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nw; ++w) {
#pragma unroll
            for (int i = 0; i < N; ++i) v[i] += lds[w * N + i];
        }
    }
    __syncthreads();
}

struct IsingAcc {
    int M, Bx, By;
};

// 0xFF in byte i where d_i is negative (bit 31 set), else 0: v_perm_b32
// selectors 9 and 11 replicate bit 31 of its low and high source dword,
// 12 gives zero.
__device__ __forceinline__ uint32_t sign_bytes(uint32_t d0, uint32_t d1, uint32_t d2, uint32_t d3) {
    return __builtin_amdgcn_perm(d1, d0, 0x0C0C0B09u) | __builtin_amdgcn_perm(d3, d2, 0x0B090C0Cu);
}

// ---------------------------------------------------------------- Ising
// One 16-site chunk of plane row y starting at byte j0 (j0 % 16 == 0,
// W % 16 == 0): own bytes, the other plane's rows y-1, y, y+1, and the halo
// dword holding the horizontal neighbour of the first (PAR = 0) or last
// (PAR = 1) byte.  Loading is split from computing so that a lane can keep
// two chunks' loads in flight.
// 16-byte accesses of the own-colour plane; NT marks them nontemporal
// (streamed past the caches) for lattice sets larger than the last-level
// cache, where the own plane is read once and written once per pass.
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
template <bool NT>
__device__ __forceinline__ uint4 load_own(const uint8_t* p) {
    if (NT) {
        const u32x4_t t = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
        return make_uint4(t.x, t.y, t.z, t.w);
    }
    return *reinterpret_cast<const uint4*>(p);
}
template <bool NT>
__device__ __forceinline__ void store_own(uint8_t* p, uint32_t a, uint32_t b, uint32_t c,
                                          uint32_t d) {
    if (NT) {
        const u32x4_t t = {a, b, c, d};
        __builtin_nontemporal_store(t, reinterpret_cast<u32x4_t*>(p));
    } else {
        *reinterpret_cast<uint4*>(p) = make_uint4(a, b, c, d);
    }
}

struct ChunkIn {
    uint4 o, m, U, D;
    uint32_t e;
};

// Byte offsets within a plane: oo of the chunk (own row and the other
// plane's same row), uo / dof of the rows above / below, eo of the halo dword.
template <bool NT>
__device__ __forceinline__ ChunkIn chunk_load(const uint8_t* own, const uint8_t* oth, uint32_t oo,
                                              uint32_t uo, uint32_t dof, uint32_t eo) {
    ChunkIn in;
    in.o = load_own<NT>(own + oo);
    in.m = *reinterpret_cast<const uint4*>(oth + oo);
    in.U = *reinterpret_cast<const uint4*>(oth + uo);
    in.D = *reinterpret_cast<const uint4*>(oth + dof);
    in.e = *reinterpret_cast<const uint32_t*>(oth + eo);
    return in;
}

// Plane offsets of one chunk: row offset ro (= y W), column j0; the rows
// above and below wrap periodically, and so does the halo dword.
template <int PAR>
struct ChunkOff {
    uint32_t oo, uo, dof, eo;
    __device__ __forceinline__ ChunkOff(uint32_t ro, uint32_t j0, uint32_t W, uint32_t last) {
        oo = ro + j0;
        uo = (ro == 0u ? last : ro - W) + j0;
        dof = (ro == last ? 0u : ro + W) + j0;
        eo = ro + (PAR == 0 ? (j0 == 0u ? W - 4u : j0 - 4u) : (j0 + 16u == W ? 0u : j0 + 16u));
    }
};

// PAR = (y + c) & 1 selects which horizontal neighbour the shifted byte
// stream supplies.  thr: LDS [18 hi | 18 lo].
template <int PAR, bool REC, bool NT>
__device__ __forceinline__ void ising_compute(const ChunkIn& in, uint8_t* own, uint32_t oo,
                                              uint32_t p, uint32_t rid, uint32_t k0, uint32_t k1,
                                              const uint32_t* thr, IsingAcc& acc) {
    const uint32_t e = in.e;
    const uint32_t ov[4] = {in.o.x, in.o.y, in.o.z, in.o.w};
    const uint32_t mv[4] = {in.m.x, in.m.y, in.m.z, in.m.w};
    const uint32_t Uv[4] = {in.U.x, in.U.y, in.U.z, in.U.w};
    const uint32_t Dv[4] = {in.D.x, in.D.y, in.D.z, in.D.w};
    uint32_t sv[4];
    if (PAR == 0) {
        sv[0] = __builtin_amdgcn_alignbyte(mv[0], e, 3);
        sv[1] = __builtin_amdgcn_alignbyte(mv[1], mv[0], 3);
        sv[2] = __builtin_amdgcn_alignbyte(mv[2], mv[1], 3);
        sv[3] = __builtin_amdgcn_alignbyte(mv[3], mv[2], 3);
    } else {
        sv[0] = __builtin_amdgcn_alignbyte(mv[1], mv[0], 1);
        sv[1] = __builtin_amdgcn_alignbyte(mv[2], mv[1], 1);
        sv[2] = __builtin_amdgcn_alignbyte(mv[3], mv[2], 1);
        sv[3] = __builtin_amdgcn_alignbyte(e, mv[3], 1);
    }
    // class 9u + 3nx + ny per byte (< 18), times 4: the byte offset of its
    // threshold in LDS (< 72, still one byte)
    uint32_t idx4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t nx = mv[k] + sv[k];
        const uint32_t ny = Uv[k] + Dv[k];
        idx4[k] = ((ov[k] << 3) + ov[k] + (nx << 1) + nx + ny) << 2;
    }
    const uint32_t kb = oo;  // within-colour index of the first site
    uint32_t w[8];
    philox4x32_10(kb >> 3, p, rid, kTagMain, k0, k1, &w[0]);
    philox4x32_10((kb >> 3) + 1u, p, rid, kTagMain, k0, k1, &w[4]);
    // d = r - T_hi as unsigned: bit 31 set iff r < T_hi (accept on the prefix),
    // d == 0 iff the prefix ties; the smallest d flags a tie anywhere.
    const uint8_t* thb = reinterpret_cast<const uint8_t*>(thr);
    uint32_t d[16];
    uint32_t dmin = 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t off = (idx4[j >> 2] >> (8 * (j & 3))) & 0xFFu;
        const uint32_t r = (w[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
        d[j] = r - *reinterpret_cast<const uint32_t*>(thb + off);
        dmin = min(dmin, d[j]);
    }
    uint32_t flip[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) flip[k] = sign_bytes(d[4 * k], d[4 * k + 1], d[4 * k + 2], d[4 * k + 3]) & 0x01010101u;
    if (dmin == 0u) {
        // The prefix equals the threshold's high half: the low halves decide.
        for (int j = 0; j < 16; ++j) {
            if (d[j] != 0u) continue;
            const uint32_t cls = ((idx4[j >> 2] >> (8 * (j & 3))) & 0xFFu) >> 2;
            const uint32_t lo = thr[kIsingClasses + cls];
            if (lo == 0u) continue;
            uint32_t f[4];
            philox4x32_10(kb + (uint32_t)j, p, rid, kTagFallback, k0, k1, f);
            if ((f[0] & 0xFFFFu) < lo) flip[j >> 2] |= 1u << (8 * (j & 3));
        }
    }
    uint32_t nv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) nv[k] = ov[k] ^ flip[k];
    store_own<NT>(own + oo, nv[0], nv[1], nv[2], nv[3]);
    if (REC) {
        // Colour-1 pass of a recorded sweep: every bond has exactly one
        // colour-1 end, so summing over the updated sites counts each once.
        uint32_t up = 0u, dx = 0u, dy = 0u;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            up = sad_u8(nv[k], up);
            up = sad_u8(mv[k], up);
            dx = sad_u8((nv[k] ^ mv[k]) + (nv[k] ^ sv[k]), dx);
            dy = sad_u8((nv[k] ^ Uv[k]) + (nv[k] ^ Dv[k]), dy);
        }
        acc.M += 2 * (int)up - 32;
        acc.Bx += 32 - 2 * (int)dx;
        acc.By += 32 - 2 * (int)dy;
    }
}

// ---------------------------------------------------------------- Potts
struct PottsAcc {
    int Nx, Ny, S;
};

// Byte-wise "not equal" flags (bit 7 of each byte) for labels < 128.
__device__ __forceinline__ uint32_t ne_hi(uint32_t a, uint32_t b) {
    return ((a ^ b) + 0x7F7F7F7Fu) & 0x80808080u;
}

// 16-site Potts chunk.  thr: LDS [n hi | n lo], n = 9(2q-1); thr9: LDS
// [9 hi | 9 lo] by dn + 4 (used when HZ, i.e. h = 0).
// Byte offsets within a plane: oo of the chunk (own row and the other
// plane's same row), uo / dof of the rows above / below, eo of the halo dword.
template <int PAR, bool REC, bool HZ, bool NT>
__device__ __forceinline__ void potts_chunk(uint8_t* own, const uint8_t* oth, uint32_t oo,
                                            uint32_t uo, uint32_t dof, uint32_t eo, uint32_t p,
                                            uint32_t rid, uint32_t k0, uint32_t k1,
                                            const uint32_t* thr, const uint32_t* thr9, int q,
                                            int ntab, uint32_t lem_thr, PottsAcc& acc,
                                            int* lhist) {
    const uint4 o = load_own<NT>(own + oo);
    const uint4 m = *reinterpret_cast<const uint4*>(oth + oo);
    const uint4 U = *reinterpret_cast<const uint4*>(oth + uo);
    const uint4 D = *reinterpret_cast<const uint4*>(oth + dof);
    const uint32_t e = *reinterpret_cast<const uint32_t*>(oth + eo);
    const uint32_t ov[4] = {o.x, o.y, o.z, o.w};
    const uint32_t mv[4] = {m.x, m.y, m.z, m.w};
    const uint32_t Uv[4] = {U.x, U.y, U.z, U.w};
    const uint32_t Dv[4] = {D.x, D.y, D.z, D.w};
    uint32_t sv[4];
    if (PAR == 0) {
        sv[0] = __builtin_amdgcn_alignbyte(mv[0], e, 3);
        sv[1] = __builtin_amdgcn_alignbyte(mv[1], mv[0], 3);
        sv[2] = __builtin_amdgcn_alignbyte(mv[2], mv[1], 3);
        sv[3] = __builtin_amdgcn_alignbyte(mv[3], mv[2], 3);
    } else {
        sv[0] = __builtin_amdgcn_alignbyte(mv[1], mv[0], 1);
        sv[1] = __builtin_amdgcn_alignbyte(mv[2], mv[1], 1);
        sv[2] = __builtin_amdgcn_alignbyte(mv[3], mv[2], 1);
        sv[3] = __builtin_amdgcn_alignbyte(e, mv[3], 1);
    }
    const uint32_t kb = oo;
    uint32_t w[16];
#pragma unroll
    for (int b = 0; b < 4; ++b)
        philox4x32_10((kb >> 2) + (uint32_t)b, p, rid, kTagMain, k0, k1, &w[4 * b]);
    const uint32_t mq = (uint32_t)(q - 1);
    // proposals s' = s + 1 + off (mod q), off uniform in [0, q-1): off is
    // byte 2 of the 16-bit Lemire product (< 2^24), and the smallest low half
    // of the products flags a rejection anywhere
    uint32_t pr[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) pr[j] = __umul24(w[j] & 0xFFFFu, mq);  // full-rate 24-bit multiply
    // Bytewise: t = s + 1 + off <= 2q - 2 < 256; u = t + (128 - q) has bit 7
    // set iff t >= q (and stays below 256); those bytes take t - q.
    const uint32_t Cb = (uint32_t)(128 - q) * 0x01010101u;
    const uint32_t Cb1 = Cb + 0x01010101u;
    uint32_t s2v[4];
    if (q <= 64) {
        // t < 128: the bytes with t >= q take the low seven bits of u
        // (u - 128 = t - q), the others u - (128 - q) = t, in one select
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t offs = __builtin_amdgcn_perm(pr[4 * k + 1], pr[4 * k], 0x0C0C0602u) |
                                  __builtin_amdgcn_perm(pr[4 * k + 3], pr[4 * k + 2], 0x06020C0Cu);
            const uint32_t u = ov[k] + offs + Cb1;
            const uint32_t G = u & 0x80808080u;
            const uint32_t M = G - (G >> 7);  // 0x7F in the bytes with t >= q
            s2v[k] = (u & M) | ((u - Cb) & ~M);
        }
    } else {
        const uint32_t Qb = (uint32_t)q * 0x01010101u;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t offs = __builtin_amdgcn_perm(pr[4 * k + 1], pr[4 * k], 0x0C0C0602u) |
                                  __builtin_amdgcn_perm(pr[4 * k + 3], pr[4 * k + 2], 0x06020C0Cu);
            const uint32_t u = ov[k] + offs + Cb1;
            const uint32_t ge = u & 0x80808080u;
            const uint32_t wrap = ((ge << 1) - (ge >> 7)) & Qb;  // q in the bytes with t >= q
            s2v[k] = u - Cb - wrap;
        }
    }
    // a rejected 16-bit Lemire draw (low half of the product below
    // 2^16 mod (q - 1)) is redrawn from the fallback stream; none are
    // rejected when q - 1 divides 2^16
    uint32_t lmin = 0xFFFFFFFFu;
    if (lem_thr != 0u) {
        // low halves compared in pairs (one word-select min per pair)
#pragma unroll
        for (int j = 0; j < 16; j += 2) lmin = min(lmin, min(pr[j] & 0xFFFFu, pr[j + 1] & 0xFFFFu));
    }
    if (lmin < lem_thr) {
        for (int j = 0; j < 16; ++j) {
            const uint32_t prod = __umul24(w[j] & 0xFFFFu, mq);
            if ((prod & 0xFFFFu) >= lem_thr) continue;
            uint32_t f[4];
            philox4x32_10(kb + (uint32_t)j, p, rid, kTagFallback, k0, k1, f);
            const uint32_t s = (ov[j >> 2] >> (8 * (j & 3))) & 0xFFu;
            const uint32_t off = (uint32_t)(((uint64_t)f[1] * (uint64_t)mq) >> 32);
            const uint32_t s2 = s + 1u + off;
            const int sh = 8 * (j & 3);
            s2v[j >> 2] = (s2v[j >> 2] & ~(0xFFu << sh)) | (min(s2, s2 - (uint32_t)q) << sh);
        }
    }
    // dn + 4 = #ne(s) - #ne(s') + 4 = #ne(s) + #eq(s') per byte.  Labels
    // below 2^b (b <= 4): ((a ^ c) + (2^b - 1)) has bit b set iff a != c;
    // the eight flags (unequal to s, equal to s') sum to (4 + dn) 2^b < 256
    // in each byte, so no per-flag shift is needed.
    uint32_t dn4[4];
    if (q <= 16) {
        const int b = q <= 2 ? 1 : 32 - __clz(q - 1);
        const uint32_t F = 0x01010101u << b, A = F - 0x01010101u;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t neo = (((ov[k] ^ mv[k]) + A) & F) + (((ov[k] ^ sv[k]) + A) & F) +
                                 (((ov[k] ^ Uv[k]) + A) & F) + (((ov[k] ^ Dv[k]) + A) & F);
            const uint32_t eqn = (~((s2v[k] ^ mv[k]) + A) & F) + (~((s2v[k] ^ sv[k]) + A) & F) +
                                 (~((s2v[k] ^ Uv[k]) + A) & F) + (~((s2v[k] ^ Dv[k]) + A) & F);
            dn4[k] = (neo + eqn) >> b;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t neo = (ne_hi(ov[k], mv[k]) >> 7) + (ne_hi(ov[k], sv[k]) >> 7) +
                                 (ne_hi(ov[k], Uv[k]) >> 7) + (ne_hi(ov[k], Dv[k]) >> 7);
            const uint32_t nen = (ne_hi(s2v[k], mv[k]) >> 7) + (ne_hi(s2v[k], sv[k]) >> 7) +
                                 (ne_hi(s2v[k], Uv[k]) >> 7) + (ne_hi(s2v[k], Dv[k]) >> 7);
            dn4[k] = neo + 0x04040404u - nen;
        }
    }
    // Class: (dn+4)(2q-1) + (s'-s+q-1); with h = 0 the threshold depends on dn
    // only and thr9 holds the 9 (hi | lo) entries.  d = r - T_hi unsigned:
    // bit 31 set iff the prefix accepts, 0 iff it ties.
    const uint32_t wq = (uint32_t)(2 * q - 1);
    uint32_t d[16];
    uint32_t dmin = 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int sh = 8 * (j & 3);
        const uint32_t d4 = (dn4[j >> 2] >> sh) & 0xFFu;
        uint32_t th;
        if (HZ) {
            th = thr9[d4];
        } else {
            const uint32_t s = (ov[j >> 2] >> sh) & 0xFFu;
            const uint32_t s2 = (s2v[j >> 2] >> sh) & 0xFFu;
            th = thr[__umul24(d4, wq) + s2 + (uint32_t)(q - 1) - s];
        }
        d[j] = (w[j] >> 16) - th;
        dmin = min(dmin, d[j]);
    }
    uint32_t acc_sel[4];  // 0xFF in bytes that accept
#pragma unroll
    for (int k = 0; k < 4; ++k)
        acc_sel[k] = sign_bytes(d[4 * k], d[4 * k + 1], d[4 * k + 2], d[4 * k + 3]);
    if (dmin == 0u) {
        // a prefix equals the threshold's high half: the low halves decide
        for (int j = 0; j < 16; ++j) {
            if (d[j] != 0u) continue;
            const int sh = 8 * (j & 3);
            const uint32_t d4 = (dn4[j >> 2] >> sh) & 0xFFu;
            uint32_t lo;
            if (HZ) {
                lo = thr9[9 + d4];
            } else {
                const uint32_t s = (ov[j >> 2] >> sh) & 0xFFu;
                const uint32_t s2 = (s2v[j >> 2] >> sh) & 0xFFu;
                lo = thr[ntab + __umul24(d4, wq) + s2 + (uint32_t)(q - 1) - s];
            }
            if (lo == 0u) continue;
            uint32_t f[4];
            philox4x32_10(kb + (uint32_t)j, p, rid, kTagFallback, k0, k1, f);
            if ((f[0] & 0xFFFFu) < lo) acc_sel[j >> 2] |= 0xFFu << sh;
        }
    }
    uint32_t nv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) nv[k] = (s2v[k] & acc_sel[k]) | (ov[k] & ~acc_sel[k]);
    store_own<NT>(own + oo, nv[0], nv[1], nv[2], nv[3]);
    if (REC) {
        uint32_t nex = 0u, ney = 0u, ssum = 0u;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            nex = sad_u8((ne_hi(nv[k], mv[k]) >> 7) + (ne_hi(nv[k], sv[k]) >> 7), nex);
            ney = sad_u8((ne_hi(nv[k], Uv[k]) >> 7) + (ne_hi(nv[k], Dv[k]) >> 7), ney);
            ssum = sad_u8(nv[k], ssum);
            ssum = sad_u8(mv[k], ssum);
        }
        acc.Nx += 32 - (int)nex;
        acc.Ny += 32 - (int)ney;
        acc.S += (int)ssum;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            atomicAdd(&lhist[(nv[j >> 2] >> (8 * (j & 3))) & 0xFFu], 1);
            atomicAdd(&lhist[(mv[j >> 2] >> (8 * (j & 3))) & 0xFFu], 1);
        }
    }
}

// ------------------------------------------------- tile-level iteration
// Rows [y0, y0+rows) of plane c (y0, rows even), split over threads
// tid = 0..nthr-1 (a whole workgroup, or the share of one replica when a
// workgroup holds several).  Rows are visited by parity so that PAR is
// uniform across a wave.
template <bool REC, bool HZ, bool NT>
__device__ __forceinline__ void run_tile_potts(uint8_t* planes, int W, int Ly, int y0, int rows,
                                               int c, uint32_t p, uint32_t rid, uint32_t k0,
                                               uint32_t k1, const uint32_t* thr,
                                               const uint32_t* thr9, int q, int ntab,
                                               uint32_t lem_thr, PottsAcc& pa, int* lhist,
                                               int tid, int nthr) {
    uint8_t* own = planes + (size_t)c * Ly * W;
    const uint8_t* oth = planes + (size_t)(1 - c) * Ly * W;
    const int cpr = W >> 4;
    // item it = r * cpr + jc (row pair r, chunk column jc), advanced by nthr
    // without a division per item
    const int dr = nthr / cpr, dj = nthr - dr * cpr;
    const int r0 = tid / cpr, jc0 = tid - r0 * cpr;
    const uint32_t Wb = (uint32_t)W, W2 = 2u * Wb;
    const uint32_t last = (uint32_t)(Ly - 1) * Wb;
    // 32-bit plane offsets advanced per item: row offset ro by dr row pairs
    // (one more when the chunk column wraps), column j0 by dj chunks; the
    // row pairs of the tile end where ro reaches row y0 + rows
    const uint32_t dro = (uint32_t)dr * W2, dj0 = (uint32_t)dj << 4;
#pragma unroll
    for (int par = 0; par < 2; ++par) {
        const int yf = y0 + ((par ^ c) & 1);
        const uint32_t ro_end = (uint32_t)(yf + rows) * Wb;
        uint32_t ro = (uint32_t)(yf + 2 * r0) * Wb, j0 = (uint32_t)jc0 << 4;
        for (; ro < ro_end;) {
            if (par == 0) {
                const ChunkOff<0> f(ro, j0, Wb, last);
                potts_chunk<0, REC, HZ, NT>(own, oth, f.oo, f.uo, f.dof, f.eo, p, rid, k0, k1, thr,
                                        thr9, q, ntab, lem_thr, pa, lhist);
            } else {
                const ChunkOff<1> f(ro, j0, Wb, last);
                potts_chunk<1, REC, HZ, NT>(own, oth, f.oo, f.uo, f.dof, f.eo, p, rid, k0, k1, thr,
                                        thr9, q, ntab, lem_thr, pa, lhist);
            }
            ro += dro;
            j0 += dj0;
            if (j0 >= Wb) {
                j0 -= Wb;
                ro += W2;
            }
        }
    }
}

// Ising rows [y0, y0+rows) of plane c.  DUAL: each lane takes one chunk of
// each row parity per iteration and issues both chunks' loads before
// computing (latency hiding for the HBM stream); otherwise one chunk per
// iteration, parity by parity (fewer registers for the LDS-resident path).
template <bool REC, bool DUAL, bool NT>
__device__ __forceinline__ void run_tile_ising(uint8_t* planes, int W, int Ly, int y0, int rows,
                                               int c, uint32_t p, uint32_t rid, uint32_t k0,
                                               uint32_t k1, const uint32_t* thr, IsingAcc& ia,
                                               int tid, int nthr) {
    uint8_t* own = planes + (size_t)c * Ly * W;
    const uint8_t* oth = planes + (size_t)(1 - c) * Ly * W;
    const int cpr = W >> 4;
    const int ya = y0 + (c & 1);        // rows with (y + c) & 1 == 0
    const int yb = y0 + ((c & 1) ^ 1);  // rows with (y + c) & 1 == 1
    // item it = r * cpr + jc (row pair r, chunk column jc), advanced by nthr
    // without a division per item: the 32-bit row offset by dr row pairs (one
    // more when the column wraps), the column by dj chunks; the row pairs of
    // the tile end where the row offset reaches row y0 + rows
    const int dr = nthr / cpr, dj = nthr - dr * cpr;
    const int r0 = tid / cpr, jc0 = tid - r0 * cpr;
    const uint32_t Wb = (uint32_t)W, W2 = 2u * Wb;
    const uint32_t last = (uint32_t)(Ly - 1) * Wb;
    const uint32_t dro = (uint32_t)dr * W2, dj0 = (uint32_t)dj << 4;
    if (DUAL) {
        // ra: row of parity 0, ra + db: the row of parity 1 in the same pair
        const int db = yb - ya;  // +1 or -1
        const uint32_t ra_end = (uint32_t)(ya + rows) * Wb;
        uint32_t ra = (uint32_t)(ya + 2 * r0) * Wb, j0 = (uint32_t)jc0 << 4;
        for (; ra < ra_end;) {
            const uint32_t rb = ra + (uint32_t)db * Wb;
            const ChunkOff<0> fa(ra, j0, Wb, last);
            const ChunkOff<1> fb(rb, j0, Wb, last);
            const ChunkIn A = chunk_load<NT>(own, oth, fa.oo, fa.uo, fa.dof, fa.eo);
            const ChunkIn B = chunk_load<NT>(own, oth, fb.oo, fb.uo, fb.dof, fb.eo);
            ising_compute<0, REC, NT>(A, own, fa.oo, p, rid, k0, k1, thr, ia);
            ising_compute<1, REC, NT>(B, own, fb.oo, p, rid, k0, k1, thr, ia);
            ra += dro;
            j0 += dj0;
            if (j0 >= Wb) {
                j0 -= Wb;
                ra += W2;
            }
        }
    } else {
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            const int yf = par == 0 ? ya : yb;
            const uint32_t ro_end = (uint32_t)(yf + rows) * Wb;
            uint32_t ro = (uint32_t)(yf + 2 * r0) * Wb, j0 = (uint32_t)jc0 << 4;
            for (; ro < ro_end;) {
                if (par == 0) {
                    const ChunkOff<0> f(ro, j0, Wb, last);
                    const ChunkIn A = chunk_load<NT>(own, oth, f.oo, f.uo, f.dof, f.eo);
                    ising_compute<0, REC, NT>(A, own, f.oo, p, rid, k0, k1, thr, ia);
                } else {
                    const ChunkOff<1> f(ro, j0, Wb, last);
                    const ChunkIn B = chunk_load<NT>(own, oth, f.oo, f.uo, f.dof, f.eo);
                    ising_compute<1, REC, NT>(B, own, f.oo, p, rid, k0, k1, thr, ia);
                }
                ro += dro;
                j0 += dj0;
                if (j0 >= Wb) {
                    j0 -= Wb;
                    ro += W2;
                }
            }
        }
    }
}

__device__ __forceinline__ void load_table(const uint32_t* tab, const RepDev& R, uint32_t* lthr,
                                           int tid, int nthr) {
    const int n2 = 2 * R.tab_n;
    for (int i = tid; i < n2; i += nthr) lthr[i] = tab[R.tab_off + i];
}

__device__ __forceinline__ uint32_t lemire_threshold(int q) {
    return 65536u % (uint32_t)(q - 1);
}

// The 9 Potts thresholds of the dn classes (hi | lo) for h = 0, where the
// class no longer depends on s' - s (column s' = s of the full table).
__device__ __forceinline__ void load_table9(const uint32_t* tab, const RepDev& R, uint32_t* t9,
                                            int tid) {
    if (R.model != kModelPotts) return;
    const int wq = 2 * R.q - 1;
    if (tid < 18) {
        const int i = tid % 9, half = tid / 9;
        t9[tid] = tab[R.tab_off + half * R.tab_n + i * wq + R.q - 1];
    }
}

// Potts tile with the h = 0 specialisation chosen per replica.
template <bool REC, bool NT>
__device__ __forceinline__ void potts_tile(const RepDev& R, uint8_t* planes, int y0, int rows,
                                           int c, uint32_t p, uint32_t k0, uint32_t k1,
                                           const uint32_t* thr, const uint32_t* thr9,
                                           PottsAcc& pa, int* lhist, int tid, int nthr) {
    const uint32_t lt = lemire_threshold(R.q);
    if (R.h == 0.0f)
        run_tile_potts<REC, true, NT>(planes, R.W, R.Ly, y0, rows, c, p, R.rid, k0, k1, thr, thr9, R.q,
                                  R.tab_n, lt, pa, lhist, tid, nthr);
    else
        run_tile_potts<REC, false, NT>(planes, R.W, R.Ly, y0, rows, c, p, R.rid, k0, k1, thr, thr9,
                                   R.q, R.tab_n, lt, pa, lhist, tid, nthr);
}

// XCD-aware block order: consecutive logical units land on one XCD (blocks
// are dispatched round-robin over the 8 XCDs), so neighbouring row tiles of a
// replica share that XCD's L2.
__device__ __forceinline__ int logical_block(int n) {
    const int b = blockIdx.x;
    if ((n & 7) != 0) return b;
    return (b & 7) * (n >> 3) + (b >> 3);
}


}  // namespace

// ---------------------------------------------------------------- kernels
// One colour pass over the row tiles [tile0, tile0 + n) of one model.  The
// two models have separate kernels so that each gets its own register
// budget (Ising needs about half of Potts's, hence twice the waves per SIMD).
template <int MODEL, bool NT>
__device__ __forceinline__ void stream_pass_body(const SweepArgs& a, int tile0, int n, int c,
                                                 int sweep_off, int rec_row, uint32_t* lthr,
                                                 uint32_t* lthr9, int* lhist, int* lred) {
    const TileDev T = a.tiles[tile0 + logical_block(n)];
    const RepDev R = a.reps[T.rep];
    load_table(a.tab, R, lthr, threadIdx.x, blockDim.x);
    if (MODEL == kModelPotts) load_table9(a.tab, R, lthr9, threadIdx.x);
    const bool rec = (rec_row >= 0) && (c == 1);
    if (MODEL == kModelPotts && rec)
        for (int i = threadIdx.x; i < R.q; i += blockDim.x) lhist[i] = 0;
    __syncthreads();
    const uint64_t t = *a.t_base + (uint64_t)sweep_off;
    const uint32_t p = (uint32_t)(2 * t + (uint64_t)c);
    uint8_t* planes = a.lat + R.lat_off;
    IsingAcc ia{0, 0, 0};
    PottsAcc pa{0, 0, 0};
    if (MODEL == kModelIsing) {
        if (rec)
            run_tile_ising<true, true, NT>(planes, R.W, R.Ly, T.y0, T.rows, c, p, R.rid, a.key0, a.key1,
                                 lthr, ia, threadIdx.x, blockDim.x);
        else
            run_tile_ising<false, true, NT>(planes, R.W, R.Ly, T.y0, T.rows, c, p, R.rid, a.key0, a.key1,
                                  lthr, ia, threadIdx.x, blockDim.x);
    } else {
        if (rec)
            potts_tile<true, NT>(R, planes, T.y0, T.rows, c, p, a.key0, a.key1, lthr, lthr9, pa,
                             lhist, threadIdx.x, blockDim.x);
        else
            potts_tile<false, NT>(R, planes, T.y0, T.rows, c, p, a.key0, a.key1, lthr, lthr9, pa,
                              lhist, threadIdx.x, blockDim.x);
    }
    if (rec) {
        int v[3];
        if (MODEL == kModelIsing) {
            v[0] = ia.M; v[1] = ia.Bx; v[2] = ia.By;
        } else {
            v[0] = pa.Nx; v[1] = pa.Ny; v[2] = pa.S;
        }
        block_sum<3>(v, lred);
        int32_t* row = a.stats + ((size_t)rec_row * a.R + T.rep) * a.width;
        if (threadIdx.x == 0) {
            atomicAdd(&row[0], v[0]);
            atomicAdd(&row[1], v[1]);
            atomicAdd(&row[2], v[2]);
        }
        if (MODEL == kModelPotts) {
            __syncthreads();
            for (int i = threadIdx.x; i < R.q; i += blockDim.x)
                if (lhist[i]) atomicAdd(&a.hist[R.hist_off + i], lhist[i]);
        }
    }
}

// Occupancy targets: the Ising pass is memory-streaming and wants many
// waves in flight; the Potts pass is VALU-heavy and keeps more registers.
template <bool NT>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_stream_pass_ising(SweepArgs a, int tile0, int n, int c, int sweep_off, int rec_row) {
    extern __shared__ uint32_t lthr[];  // [2 * tab_n] thresholds of this tile's replica
    __shared__ uint32_t lthr9[18];
    __shared__ int lhist[kMaxPottsQ];
    __shared__ int lred[64];
    stream_pass_body<kModelIsing, NT>(a, tile0, n, c, sweep_off, rec_row, lthr, lthr9, lhist, lred);
}

template <bool NT>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_stream_pass_potts(SweepArgs a, int tile0, int n, int c, int sweep_off, int rec_row) {
    extern __shared__ uint32_t lthr[];
    __shared__ uint32_t lthr9[18];
    __shared__ int lhist[kMaxPottsQ];
    __shared__ int lred[64];
    stream_pass_body<kModelPotts, NT>(a, tile0, n, c, sweep_off, rec_row, lthr, lthr9, lhist, lred);
}

// ------------------------------------------------- persistent streamed passes
// One launch runs every colour pass of a chunk of unrecorded sweeps over the
// streamed replicas of one model (the batched scheduler without a launch per
// pass).  Workgroup g owns its items for the whole launch: whole replicas,
// which no other workgroup touches, so the workgroup's barrier between
// passes orders their passes, or one row slab of a replica cut into slabs
// owned by different workgroups.  A slab's pass j (counted from 0 within the
// launch) reads the other plane's rows just above and below it, which the
// neighbouring slabs write in their pass j - 1, and writes rows that they
// read in their pass j - 1; so it starts once both neighbours have published
// pass j - 1 (flag >= j), and a slab never runs more than one pass ahead of
// its neighbours.  Publishing: every lane waits for its stores, the
// workgroup meets at a barrier, lane 0 stores flag = j + 1 with agent-scope
// release (write-back of the XCD's L2).  Waiting: lane 0 polls the
// neighbours' flags, then takes an agent-scope acquire (invalidation of its
// L1 and L2) before the barrier that lets the other lanes read.  All slab
// workgroups must be resident at once: the host keeps their number within
// the occupancy of the whole chip and numbers them first, so that in-order
// dispatch places them before any whole-replica workgroup.  A wait that
// exceeds its bound (about two seconds) raises *abort, and every waiting
// workgroup then leaves: a launch always ends.
constexpr uint32_t kPersistSpinCap = 1u << 25;  // polls of ~128 cycles each

// every store of this lane has completed (vmcnt 0; exp and lgkm counts
// left at their maxima)
__device__ __forceinline__ void wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Agent-scope release of a pass flag: the fence writes the L2 back (the
// workgroup's rows reach memory for the other XCDs), the explicit vmcnt(0)
// waits for that write-back to finish, then the flag is stored.  (The
// release store alone compiles to the write-back directly followed by the
// flag store, with no wait between them, when the workgroup's stores were
// already waited for, so the flag could be seen before the rows.)
__device__ __forceinline__ void persist_publish(uint32_t* flag, uint32_t v) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    wait_stores();
    __hip_atomic_store(flag, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ int persist_wait(uint32_t* flags, int up, int down, uint32_t need, uint32_t* abort_flag) {
    for (uint32_t spin = 0;; ++spin) {
        const uint32_t u = __hip_atomic_load(&flags[up], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t d = __hip_atomic_load(&flags[down], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (u >= need && d >= need) break;
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return 0;
        if (spin >= kPersistSpinCap) {
            __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return 0;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return 1;
}

template <int MODEL, bool NT>
__device__ __forceinline__ void persist_body(const SweepArgs& a, const PersistItem* items,
                                             const int32_t* item_off, uint32_t* flags,
                                             uint32_t* abort_flag, int slot_words, uint32_t* lds,
                                             int* go) {
    const int i0 = item_off[blockIdx.x], i1 = item_off[blockIdx.x + 1];
    // threshold tables of the items' replicas (Potts: the h = 0 table of 9
    // entries in the last 18 words of the slot)
    for (int k = i0; k < i1; ++k) {
        const RepDev R = a.reps[items[k].rep];
        uint32_t* t = lds + (k - i0) * slot_words;
        load_table(a.tab, R, t, threadIdx.x, blockDim.x);
        if (MODEL == kModelPotts) load_table9(a.tab, R, t + slot_words - 18, threadIdx.x);
    }
    __syncthreads();
    const uint64_t t0 = *a.t_base + (uint64_t)a.sweep_off;
    for (int sw = 0; sw < a.n_sweeps; ++sw) {
        for (int c = 0; c < 2; ++c) {
            const uint32_t j = (uint32_t)(2 * sw + c);
            const uint32_t p = (uint32_t)(2 * (t0 + (uint64_t)sw) + (uint64_t)c);
            for (int k = i0; k < i1; ++k) {
                const PersistItem it = items[k];
                if (it.slab >= 0 && j > 0) {
                    if (threadIdx.x == 0) *go = persist_wait(flags, it.up, it.down, j, abort_flag);
                    __syncthreads();
                    if (!*go) return;  // uniform: the whole workgroup leaves
                }
                const RepDev R = a.reps[it.rep];
                uint32_t* tab = lds + (k - i0) * slot_words;
                uint8_t* planes = a.lat + R.lat_off;
                if (MODEL == kModelIsing) {
                    IsingAcc ia{0, 0, 0};
                    run_tile_ising<false, true, NT>(planes, R.W, R.Ly, it.y0, it.rows, c, p, R.rid,
                                                    a.key0, a.key1, tab, ia, threadIdx.x,
                                                    blockDim.x);
                } else {
                    PottsAcc pa{0, 0, 0};
                    potts_tile<false, NT>(R, planes, it.y0, it.rows, c, p, a.key0, a.key1, tab,
                                          tab + slot_words - 18, pa, nullptr, threadIdx.x,
                                          blockDim.x);
                }
                if (it.slab >= 0) {
                    wait_stores();
                    __syncthreads();
                    if (threadIdx.x == 0) persist_publish(&flags[it.slab], j + 1u);
                }
            }
            __syncthreads();  // the workgroup's pass boundary
        }
    }
}

template <bool NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_persist_ising(SweepArgs a, const PersistItem* items, const int32_t* item_off, uint32_t* flags,
                uint32_t* abort_flag, int slot_words) {
    extern __shared__ uint32_t ptab[];
    __shared__ int go;
    persist_body<kModelIsing, NT>(a, items, item_off, flags, abort_flag, slot_words, ptab, &go);
}

template <bool NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_persist_potts(SweepArgs a, const PersistItem* items, const int32_t* item_off, uint32_t* flags,
                uint32_t* abort_flag, int slot_words) {
    extern __shared__ uint32_t ptab[];
    __shared__ int go;
    persist_body<kModelPotts, NT>(a, items, item_off, flags, abort_flag, slot_words, ptab, &go);
}

// nmax of each Potts replica from its histogram; clears the histogram.
__global__ void k_potts_hist_finalize(SweepArgs a, const int32_t* list, int n, int rec_row) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = list[i];
    const RepDev R = a.reps[r];
    int mx = 0;
    for (int k = 0; k < R.q; ++k) {
        const int v = a.hist[R.hist_off + k];
        mx = v > mx ? v : mx;
        a.hist[R.hist_off + k] = 0;
    }
    a.stats[((size_t)rec_row * a.R + r) * a.width + 3] = mx;
}

// ------------------------------------------------------ generic (any L)
namespace {

__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// One site of colour c, within-colour index k, in planes (LDS or global).
__device__ __forceinline__ void generic_site(int model, uint8_t* planes, int W, int Ly, int c,
                                             int k, uint32_t p, uint32_t rid, uint32_t k0,
                                             uint32_t k1, const uint32_t* thr, int q, int ntab) {
    const int y = k / W;
    const int j = k - y * W;
    const int off = (y + c) & 1;
    uint8_t* own = planes + (size_t)c * Ly * W;
    const uint8_t* oth = planes + (size_t)(1 - c) * Ly * W;
    const int ym = wrapi(y - 1, Ly), yp = wrapi(y + 1, Ly);
    const int js = wrapi(off ? j + 1 : j - 1, W);
    const uint32_t s = own[(size_t)y * W + j];
    const uint32_t a0 = oth[(size_t)y * W + j], a1 = oth[(size_t)y * W + js];
    const uint32_t b0 = oth[(size_t)ym * W + j], b1 = oth[(size_t)yp * W + j];
    uint32_t w[4];
    if (model == kModelIsing) {
        philox4x32_10((uint32_t)k >> 3, p, rid, kTagMain, k0, k1, w);
        const uint32_t h = (uint32_t)k & 7u;
        const uint32_t r = (w[h >> 1] >> (16 * (h & 1))) & 0xFFFFu;
        const uint32_t cls = 9u * s + 3u * (a0 + a1) + (b0 + b1);
        const uint32_t hi = thr[cls];
        bool acc = r < hi;
        if (r == hi && thr[kIsingClasses + cls] != 0u) {
            uint32_t f[4];
            philox4x32_10((uint32_t)k, p, rid, kTagFallback, k0, k1, f);
            acc = (f[0] & 0xFFFFu) < thr[kIsingClasses + cls];
        }
        if (acc) own[(size_t)y * W + j] = (uint8_t)(s ^ 1u);
    } else {
        philox4x32_10((uint32_t)k >> 2, p, rid, kTagMain, k0, k1, w);
        const uint32_t word = w[k & 3];
        const uint32_t mq = (uint32_t)(q - 1);
        const uint32_t prod = (word & 0xFFFFu) * mq;
        uint32_t off2 = prod >> 16;
        uint32_t f[4];
        bool have_f = false;
        if ((prod & 0xFFFFu) < 65536u % mq) {
            philox4x32_10((uint32_t)k, p, rid, kTagFallback, k0, k1, f);
            have_f = true;
            off2 = (uint32_t)(((uint64_t)f[1] * (uint64_t)mq) >> 32);
        }
        uint32_t s2 = s + 1u + off2;
        s2 = s2 >= (uint32_t)q ? s2 - (uint32_t)q : s2;
        const int dn = (int)(a0 == s2) + (int)(a1 == s2) + (int)(b0 == s2) + (int)(b1 == s2) -
                       (int)(a0 == s) - (int)(a1 == s) - (int)(b0 == s) - (int)(b1 == s);
        const uint32_t cls = (uint32_t)(dn + 4) * (uint32_t)(2 * q - 1) + s2 + (uint32_t)(q - 1) - s;
        const uint32_t hi = thr[cls];
        const uint32_t r = word >> 16;
        bool acc = r < hi;
        if (r == hi && thr[ntab + cls] != 0u) {
            if (!have_f) philox4x32_10((uint32_t)k, p, rid, kTagFallback, k0, k1, f);
            acc = (f[0] & 0xFFFFu) < thr[ntab + cls];
        }
        if (acc) own[(size_t)y * W + j] = (uint8_t)s2;
    }
}

__device__ __forceinline__ uint32_t site_at(const uint8_t* planes, int W, int Ly, int y, int x) {
    return planes[(size_t)((x + y) & 1) * Ly * W + (size_t)y * W + (x >> 1)];
}

// Integer statistics of a whole lattice (Ising: M, Bx, By; Potts: Nx, Ny, S
// and the label histogram into hist).  Thread-strided over natural sites.
__device__ __forceinline__ void lattice_stats(int model, const uint8_t* planes, int Lx, int Ly,
                                              int W, int n0, int n1, int (&v)[3], int* hist) {
    for (int n = n0 + (int)threadIdx.x; n < n1; n += blockDim.x) {
        const int y = n / Lx, x = n - y * Lx;
        const int s = (int)site_at(planes, W, Ly, y, x);
        const int r = (int)site_at(planes, W, Ly, y, x + 1 == Lx ? 0 : x + 1);
        const int d = (int)site_at(planes, W, Ly, y + 1 == Ly ? 0 : y + 1, x);
        if (model == kModelIsing) {
            const int ss = 2 * s - 1;
            v[0] += ss;
            v[1] += ss * (2 * r - 1);
            v[2] += ss * (2 * d - 1);
        } else {
            v[0] += (s == r);
            v[1] += (s == d);
            v[2] += s;
            atomicAdd(&hist[s], 1);
        }
    }
}

}  // namespace

// Resident kernel: a workgroup owns a.rpb replicas of one shape for the
// whole call, each with its thresholds and both planes in LDS, and
// blockDim/rpb threads; colour passes are separated by workgroup barriers.
// KIND selects the path: kResIsing / kResPotts run the 16-byte SWAR chunks
// (W % 16 == 0, every replica of the launch of that model), kResGeneric the
// per-site code for any model and width.  Separate instantiations keep the
// Ising path's register count (and so its waves per SIMD) free of Potts's.
template <int KIND>
__device__ __forceinline__ void resident_body(const SweepArgs& a) {
    constexpr bool CHUNK = KIND != kResGeneric;
    // dynamic LDS: rpb slots of [thresholds (tab_lds_bytes) | plane 0 | plane 1]
    extern __shared__ __align__(16) uint8_t dyn[];
    __shared__ uint32_t lthr9[kMaxRpb][18];
    __shared__ int lhist[kMaxPottsQ];
    __shared__ int lred[64];
    __shared__ int lsum[kMaxRpb][3];  // Ising: per-slot (M, Bx, By) of a recorded sweep
    const int P = a.rpb;
    const int nt = blockDim.x / P;
    const int g = threadIdx.x / nt, lt = threadIdx.x - g * nt;
    const int first = blockIdx.x * P;
    const bool active = g < P && first + g < a.n_list;
    const int rep = a.rep_list[active ? first + g : first];
    const RepDev R = a.reps[rep];
    uint8_t* slot = dyn + (size_t)(active ? g : 0) * a.res_slot_bytes;
    uint32_t* lthr = reinterpret_cast<uint32_t*>(slot);
    uint8_t* lds = slot + a.tab_lds_bytes;
    const int plane = R.Ly * R.W;
    const int bytes = 2 * plane;
    uint8_t* gmem = a.lat + R.lat_off;
    if (active) {
        if ((bytes & 15) == 0) {
            for (int i = lt; i < (bytes >> 4); i += nt)
                reinterpret_cast<uint4*>(lds)[i] = reinterpret_cast<const uint4*>(gmem)[i];
        } else {
            for (int i = lt; i < bytes; i += nt) lds[i] = gmem[i];
        }
        load_table(a.tab, R, lthr, lt, nt);
        load_table9(a.tab, R, lthr9[g], lt);
    }
    __syncthreads();
    const uint64_t t0 = *a.t_base;
    for (int i = 0; i < a.n_sweeps; ++i) {
        const int sw = a.sweep_off + i;  // sweep index within the call
        const uint64_t t = t0 + (uint64_t)sw;
        const bool rec = a.record_every > 0 && ((sw + 1) % a.record_every) == 0;
        for (int c = 0; c < 2; ++c) {
            const uint32_t p = (uint32_t)(2 * t + (uint64_t)c);
            if (KIND == kResIsing && rec && c == 1) {
                if (threadIdx.x < 3 * kMaxRpb) (&lsum[0][0])[threadIdx.x] = 0;
                __syncthreads();
            }
            if (active) {
                if (KIND == kResIsing) {
                    IsingAcc ia{0, 0, 0};
                    if (rec && c == 1) {
                        // statistics fused into the colour-1 pass: every bond has
                        // exactly one colour-1 end
                        run_tile_ising<true, false, false>(lds, R.W, R.Ly, 0, R.Ly, c, p, R.rid,
                                                           a.key0, a.key1, lthr, ia, lt, nt);
                        atomicAdd(&lsum[g][0], ia.M);
                        atomicAdd(&lsum[g][1], ia.Bx);
                        atomicAdd(&lsum[g][2], ia.By);
                    } else {
                        run_tile_ising<false, false, false>(lds, R.W, R.Ly, 0, R.Ly, c, p, R.rid,
                                                            a.key0, a.key1, lthr, ia, lt, nt);
                    }
                } else if (KIND == kResPotts) {
                    PottsAcc pa{0, 0, 0};
                    potts_tile<false, false>(R, lds, 0, R.Ly, c, p, a.key0, a.key1, lthr, lthr9[g], pa,
                                      lhist, lt, nt);
                } else {
                    for (int k = lt; k < plane; k += nt)
                        generic_site(R.model, lds, R.W, R.Ly, c, k, p, R.rid, a.key0, a.key1,
                                     lthr, R.q, R.tab_n);
                }
            }
            __syncthreads();
        }
        if (KIND == kResIsing && rec) {
            if (active && lt == 0) {
                int32_t* row =
                    a.stats + ((size_t)((sw + 1) / a.record_every - 1) * a.R + rep) * a.width;
                row[0] = lsum[g][0];
                row[1] = lsum[g][1];
                row[2] = lsum[g][2];
                for (int k = 3; k < a.width; ++k) row[k] = 0;
            }
        } else if (rec) {
            // statistics of each replica of the workgroup, all threads per replica
            for (int gg = 0; gg < P && first + gg < a.n_list; ++gg) {
                const int rg = a.rep_list[first + gg];
                const RepDev Q = a.reps[rg];
                const uint8_t* lq = dyn + (size_t)gg * a.res_slot_bytes + a.tab_lds_bytes;
                if (Q.model == kModelPotts) {
                    for (int k = threadIdx.x; k < Q.q; k += blockDim.x) lhist[k] = 0;
                    __syncthreads();
                }
                int v[3] = {0, 0, 0};
                lattice_stats(Q.model, lq, Q.Lx, Q.Ly, Q.W, 0, Q.Lx * Q.Ly, v, lhist);
                block_sum<3>(v, lred);
                int32_t* row =
                    a.stats + ((size_t)((sw + 1) / a.record_every - 1) * a.R + rg) * a.width;
                if (threadIdx.x == 0) {
                    row[0] = v[0];
                    row[1] = v[1];
                    row[2] = v[2];
                    int mx = 0;
                    if (Q.model == kModelPotts)
                        for (int k = 0; k < Q.q; ++k) mx = lhist[k] > mx ? lhist[k] : mx;
                    row[3] = mx;
                    for (int k = 4; k < a.width; ++k) row[k] = 0;
                }
                __syncthreads();
            }
        }
    }
    if (active) {
        if ((bytes & 15) == 0) {
            for (int i = lt; i < (bytes >> 4); i += nt)
                reinterpret_cast<uint4*>(gmem)[i] = reinterpret_cast<const uint4*>(lds)[i];
        } else {
            for (int i = lt; i < bytes; i += nt) gmem[i] = lds[i];
        }
    }
}

__global__ void __launch_bounds__(512) k_resident_generic(SweepArgs a) {
    resident_body<kResGeneric>(a);
}

__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_resident_ising(SweepArgs a) {
    resident_body<kResIsing>(a);
}

__global__ void __launch_bounds__(512) k_resident_potts(SweepArgs a) {
    resident_body<kResPotts>(a);
}

// Initial state from the init stream: natural index n, block n >> 2, word n & 3.
__global__ void k_init(const RepDev* reps, const int32_t* list, uint8_t* lat, uint32_t k0,
                       uint32_t k1) {
    const RepDev R = reps[list[blockIdx.y]];
    const int N = R.Lx * R.Ly;
    uint8_t* planes = lat + R.lat_off;
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; 4 * b < N; b += gridDim.x * blockDim.x) {
        uint32_t w[4];
        philox4x32_10((uint32_t)b, 0u, R.rid, kTagInit, k0, k1, w);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int n = 4 * b + i;
            if (n >= N) break;
            const int y = n / R.Lx, x = n - y * R.Lx;
            uint8_t v;
            if (R.model == kModelIsing)
                v = (w[i] < 0x80000000u) ? 1 : 0;
            else
                v = (uint8_t)(((uint64_t)w[i] * (uint64_t)R.q) >> 32);
            planes[(size_t)((x + y) & 1) * R.Ly * R.W + (size_t)y * R.W + (x >> 1)] = v;
        }
    }
}

// Statistics of the current state: grid (tiles of natural sites, replicas).
__global__ void k_measure(const RepDev* reps, const int32_t* list, const uint8_t* lat,
                          int32_t* stats, int32_t* hist, int width) {
    __shared__ int lred[64];
    const int r = list[blockIdx.y];
    const RepDev R = reps[r];
    const int N = R.Lx * R.Ly;
    const int per = 4096;
    const int n0 = blockIdx.x * per;
    if (n0 >= N) return;
    const int n1 = min(N, n0 + per);
    int v[3] = {0, 0, 0};
    lattice_stats(R.model, lat + R.lat_off, R.Lx, R.Ly, R.W, n0, n1, v, hist + R.hist_off);
    block_sum<3>(v, lred);
    if (threadIdx.x == 0) {
        atomicAdd(&stats[(size_t)r * width + 0], v[0]);
        atomicAdd(&stats[(size_t)r * width + 1], v[1]);
        atomicAdd(&stats[(size_t)r * width + 2], v[2]);
    }
}

__global__ void k_fill_i32(int32_t* p, size_t n, int32_t v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_advance(uint64_t* t, uint64_t n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *t += n;
}

__global__ void k_copy_counter(uint64_t* t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) t[1] = t[0];
}

// FP64 observables from integer statistics (one thread per replica).
__global__ void k_observables(const RepDev* reps, int R, const int32_t* stats, int width,
                              double* obs) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    const RepDev D = reps[r];
    const int32_t* s = stats + (size_t)r * width;
    const double N = (double)D.Lx * (double)D.Ly;
    double* o = obs + (size_t)r * 4;
    if (D.model == kModelIsing) {
        const double M = s[0], Bx = s[1], By = s[2];
        const double H = -((double)D.Jx * Bx + (double)D.Jy * By + (double)D.h * M);
        o[0] = H / N;
        o[1] = fabs(M) / N;
        o[2] = (M / N) * (M / N);
        o[3] = M / N;
    } else if (D.model == kModelPotts) {
        const double Nx = s[0], Ny = s[1], S = s[2], nm = s[3];
        const double H = -((double)D.Jx * (Nx + Ny) + (double)D.h * S);
        o[0] = H / N;
        o[1] = ((double)D.q * nm / N - 1.0) / ((double)D.q - 1.0);
        o[2] = S / N;
        o[3] = 0.0;
    } else {
        const uint64_t lo = (uint32_t)s[10], hi = (uint32_t)s[11];
        const int64_t H = (int64_t)((hi << 32) | lo);
        o[0] = (double)H / (double)D.S;
        o[1] = 0.0;
        o[2] = 0.0;
        o[3] = 0.0;
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_init(const RepDev* reps, const int32_t* list, int n, uint8_t* lat,
                       uint32_t key0, uint32_t key1, int threads, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    dim3 grid(64, n);
    hipLaunchKernelGGL(k_init, grid, dim3(threads), 0, s, reps, list, lat, key0, key1);
    return hipGetLastError();
}

hipError_t resident_reserve_lds(size_t lds_bytes) {
    const void* fns[3] = {(const void*)k_resident_generic, (const void*)k_resident_ising,
                          (const void*)k_resident_potts};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 3 && e == hipSuccess; ++i)
        e = hipFuncSetAttribute(fns[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    return e;
}

hipError_t launch_resident(const SweepArgs& a, int n_list, int model, bool chunk, int threads,
                           size_t lds_bytes, hipStream_t s) {
    if (n_list <= 0) return hipSuccess;
    const int blocks = (n_list + a.rpb - 1) / a.rpb;
    if (!chunk)
        hipLaunchKernelGGL(k_resident_generic, dim3(blocks), dim3(threads), lds_bytes, s, a);
    else if (model == kModelIsing)
        hipLaunchKernelGGL(k_resident_ising, dim3(blocks), dim3(threads), lds_bytes, s, a);
    else
        hipLaunchKernelGGL(k_resident_potts, dim3(blocks), dim3(threads), lds_bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_stream_pass(const SweepArgs& a, int model, int tile0, int n_tiles, int c,
                              int sweep_off, int rec_row, int threads, size_t lds_tab_bytes,
                              bool nt, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    const dim3 g(n_tiles), b(threads);
    if (model == kModelIsing) {
        if (nt)
            hipLaunchKernelGGL(k_stream_pass_ising<true>, g, b, lds_tab_bytes, s, a, tile0, n_tiles,
                               c, sweep_off, rec_row);
        else
            hipLaunchKernelGGL(k_stream_pass_ising<false>, g, b, lds_tab_bytes, s, a, tile0,
                               n_tiles, c, sweep_off, rec_row);
    } else {
        if (nt)
            hipLaunchKernelGGL(k_stream_pass_potts<true>, g, b, lds_tab_bytes, s, a, tile0, n_tiles,
                               c, sweep_off, rec_row);
        else
            hipLaunchKernelGGL(k_stream_pass_potts<false>, g, b, lds_tab_bytes, s, a, tile0,
                               n_tiles, c, sweep_off, rec_row);
    }
    return hipGetLastError();
}

namespace {
const void* persist_fn(int model, bool nt) {
    if (model == kModelIsing)
        return nt ? (const void*)k_persist_ising<true> : (const void*)k_persist_ising<false>;
    return nt ? (const void*)k_persist_potts<true> : (const void*)k_persist_potts<false>;
}
}  // namespace

hipError_t persist_reserve_lds(size_t lds_bytes) {
    hipError_t e = hipSuccess;
    for (int m = 0; m < 2 && e == hipSuccess; ++m)
        for (int nt = 0; nt < 2 && e == hipSuccess; ++nt)
            e = hipFuncSetAttribute(persist_fn(m, nt != 0),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    return e;
}

hipError_t persist_occupancy(int model, bool nt, size_t lds_bytes, int* per_cu) {
    *per_cu = 0;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, persist_fn(model, nt), 256,
                                                        lds_bytes);
}

hipError_t launch_persist(const SweepArgs& a, int model, const PersistItem* items,
                          const int32_t* item_off, int n_wg, uint32_t* flags, uint32_t* abort_flag,
                          int slot_words, size_t lds_bytes, bool nt, hipStream_t s) {
    if (n_wg <= 0) return hipSuccess;
    const dim3 g(n_wg), b(256);
    if (model == kModelIsing) {
        if (nt)
            hipLaunchKernelGGL(k_persist_ising<true>, g, b, lds_bytes, s, a, items, item_off, flags,
                               abort_flag, slot_words);
        else
            hipLaunchKernelGGL(k_persist_ising<false>, g, b, lds_bytes, s, a, items, item_off,
                               flags, abort_flag, slot_words);
    } else {
        if (nt)
            hipLaunchKernelGGL(k_persist_potts<true>, g, b, lds_bytes, s, a, items, item_off, flags,
                               abort_flag, slot_words);
        else
            hipLaunchKernelGGL(k_persist_potts<false>, g, b, lds_bytes, s, a, items, item_off,
                               flags, abort_flag, slot_words);
    }
    return hipGetLastError();
}

hipError_t launch_potts_hist_finalize(const SweepArgs& a, const int32_t* list, int n, int rec_row,
                                      hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_potts_hist_finalize, dim3((n + 255) / 256), dim3(256), 0, s, a, list, n,
                       rec_row);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy_counter(uint64_t* t, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_counter, dim3(1), dim3(64), 0, s, t);
    return hipGetLastError();
}

hipError_t launch_advance(uint64_t* t, uint64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, t, n);
    return hipGetLastError();
}

hipError_t launch_measure(const RepDev* reps, const int32_t* list, int n, int max_sites,
                          const uint8_t* lat, int32_t* stats, int32_t* hist, int width,
                          hipStream_t s) {
    if (n <= 0) return hipSuccess;
    // grid.x covers the largest replica in 4096-site tiles; extra blocks exit
    const int gx = (max_sites + 4095) / 4096;
    hipLaunchKernelGGL(k_measure, dim3(gx, n), dim3(256), 0, s, reps, list, lat, stats, hist,
                       width);
    return hipGetLastError();
}

hipError_t launch_observables(const RepDev* reps, int R, const int32_t* stats, int width,
                              double* obs, hipStream_t s) {
    hipLaunchKernelGGL(k_observables, dim3((R + 127) / 128), dim3(128), 0, s, reps, R, stats,
                       width, obs);
    return hipGetLastError();
}

}  // namespace spinmc

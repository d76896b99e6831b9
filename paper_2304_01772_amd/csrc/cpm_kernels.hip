// Cellular Potts model (Eq. (3)) copy-attempt kernels for gfx950.
//
// Cell ids are int32 in natural row-major layout.  The Moore neighbourhood
// has range one in both axes, so a 2x2 sublattice colouring
// c = 2 (y & 1) + (x & 1) makes the sites of one colour independent (the
// colouring criterion of the Related-Work section: no site interacts with
// another site of its own colour); a Monte Carlo step is the four colour
// passes in order.  Each attempt picks a target site and one of its eight
// neighbours (Methods, Cellular Potts model), and copies the neighbour's id
// through the Algorithm-1 test.  Energies are integers in a fixed-point
// scale S; the area term reads a snapshot of the cell areas taken at the
// start of the pass (so the outcome does not depend on the order in which
// the sites of one pass are visited), and accepted copies update the areas
// with integer atomics, which commute.  The streamed passes keep the
// snapshot without a copy launch: pass P reads it as S[P & 1] + D[(P-1) % 3]
// (the previous snapshot plus the previous pass's changes), adds its own
// changes into D[P % 3], and on the side writes its snapshot to S[(P+1) & 1]
// and clears D[(P+1) % 3] for pass P + 1 (buffers no other pass of the
// launch touches).
#include "cpm_internal.hpp"

namespace spinmc {

namespace {
__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// The rotating snapshot / change buffers of pass P for cells at offset off.
struct PassAreas {
    const int32_t* s_rd;  // previous snapshot
    const int32_t* d_rd;  // previous pass's changes
    int32_t* d_wr;        // this pass's changes
};
__device__ __forceinline__ PassAreas pass_areas(const CpmArgs& a, uint64_t P, int off) {
    const size_t n = (size_t)a.total_cells;
    PassAreas r;
    r.s_rd = a.sbuf + (size_t)(P & 1u) * n + off;
    r.d_rd = a.dbuf + (size_t)((P + 2u) % 3u) * n + off;
    r.d_wr = a.dbuf + (size_t)(P % 3u) * n + off;
    return r;
}

// Side work of pass P, spread over the launch's threads: the snapshot it
// reads goes to S[(P+1) & 1] and D[(P+1) % 3] is cleared.
__device__ __forceinline__ void pass_rotate(const CpmArgs& a, uint64_t P) {
    const size_t n = (size_t)a.total_cells;
    const int32_t* s_rd = a.sbuf + (size_t)(P & 1u) * n;
    const int32_t* d_rd = a.dbuf + (size_t)((P + 2u) % 3u) * n;
    int32_t* s_wr = a.sbuf + (size_t)((P + 1u) & 1u) * n;
    int32_t* d_clr = a.dbuf + (size_t)((P + 1u) % 3u) * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        s_wr[i] = s_rd[i] + d_rd[i];
        d_clr[i] = 0;
    }
}
}  // namespace

__global__ void __launch_bounds__(256) k_cpm_pass(CpmArgs a, int c, int sweep_off) {
    extern __shared__ uint32_t lthr[];  // [2 * tab_n]: hi16 | lo16 of T(k), k = 1..K1-1
    __shared__ int32_t ljs[kMaxCpmTypes * kMaxCpmTypes];
    const TileDev T = a.tiles[blockIdx.x];
    const RepDev R = a.reps[T.rep];
    for (int i = threadIdx.x; i < 2 * R.tab_n; i += blockDim.x) lthr[i] = a.tab[R.tab_off + i];
    for (int i = threadIdx.x; i < R.n_types * R.n_types; i += blockDim.x)
        ljs[i] = a.js[R.js_off + i];
    __syncthreads();
    const uint64_t t = *a.t_base + (uint64_t)sweep_off;
    const uint64_t P = 4 * t + (uint64_t)c;
    const uint32_t p = (uint32_t)P;
    pass_rotate(a, P);
    const PassAreas pa = pass_areas(a, P, R.cell_off);
    const int cy = c >> 1, cx = c & 1;
    const int Lx = R.Lx, Ly = R.Ly, Wc = Lx >> 1, nt = R.n_types;
    int32_t* ids = a.lat + R.lat_off;
    const int8_t* ty = a.ctype + R.cell_off;
    const int32_t* A = a.target + R.cell_off;
    int32_t* area = pa.d_wr;
    const auto snap_of = [&](int i) -> int64_t { return (int64_t)pa.s_rd[i] + pa.d_rd[i]; };
    const int total = (T.rows >> 1) * Wc;
    for (int it = threadIdx.x; it < total; it += blockDim.x) {
        const int r = it / Wc;
        const int i = it - r * Wc;
        const int y = T.y0 + 2 * r + cy;
        const int x = 2 * i + cx;
        const uint32_t k = (uint32_t)((y >> 1) * Wc + i);
        uint32_t w[4];
        philox4x32_10(k >> 2, p, R.rid, kTagMain, a.key0, a.key1, w);
        const uint32_t word = w[k & 3u];
        const int jn = (int)(word & 7u);
        // Moore order (dy, dx): (-1,-1) (-1,0) (-1,1) (0,-1) (0,1) (1,-1) (1,0) (1,1)
        const int ndy = jn < 3 ? -1 : (jn < 5 ? 0 : 1);
        const int ndx = (jn == 0 || jn == 3 || jn == 5) ? -1 : ((jn == 1 || jn == 6) ? 0 : 1);
        const int ym = wrapc(y - 1, Ly), yp = wrapc(y + 1, Ly);
        const int xm = wrapc(x - 1, Lx), xp = wrapc(x + 1, Lx);
        const int s = ids[(size_t)y * Lx + x];
        const int tg = ids[(size_t)wrapc(y + ndy, Ly) * Lx + wrapc(x + ndx, Lx)];
        if (tg == s) continue;
        const int nb[8] = {ids[(size_t)ym * Lx + xm], ids[(size_t)ym * Lx + x],
                           ids[(size_t)ym * Lx + xp], ids[(size_t)y * Lx + xm],
                           ids[(size_t)y * Lx + xp], ids[(size_t)yp * Lx + xm],
                           ids[(size_t)yp * Lx + x], ids[(size_t)yp * Lx + xp]};
        const int ts = ty[s] * nt, tt = ty[tg] * nt;
        int kadh = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int m = nb[j];
            const int tm = ty[m];
            kadh += (tg != m) ? ljs[tt + tm] : 0;
            kadh -= (s != m) ? ljs[ts + tm] : 0;
        }
        int64_t karea = 0;
        if (tg != 0) karea += 2 * (snap_of(tg) - (int64_t)A[tg]) + 1;
        if (s != 0) karea += -2 * (snap_of(s) - (int64_t)A[s]) + 1;
        const int64_t kk = (int64_t)kadh + R.LS * karea;
        bool acc;
        if (kk <= 0) {
            acc = true;
        } else if (kk >= R.K0) {
            acc = false;
        } else {
            uint32_t hi = 0u, lo = 1u;  // T = 1 for K1 <= k < K0
            if (kk < (int64_t)R.K1) {
                hi = lthr[kk - 1];
                lo = lthr[R.tab_n + kk - 1];
            }
            const uint32_t rr = word >> 16;
            acc = rr < hi;
            if (rr == hi && lo != 0u) {
                uint32_t f[4];
                philox4x32_10(k, p, R.rid, kTagFallback, a.key0, a.key1, f);
                acc = (f[0] & 0xFFFFu) < lo;
            }
        }
        if (acc) {
            ids[(size_t)y * Lx + x] = tg;
            atomicAdd(&area[tg], 1);
            atomicAdd(&area[s], -1);
        }
    }
}

// The 5x5 neighbourhood (the Moore neighbourhood with its second shell):
// 24 neighbours in row-major order of (dy, dx) for both the adhesion sum and
// the copy source; the 3x3 sublattice c = 3 (y % 3) + x % 3 keeps the sites
// of one colour out of each other's neighbourhoods; pass p = 9t + c, within-
// colour index k = (y / 3) Lx/3 + x / 3.  The neighbour index is Lemire's
// multiply-shift of the low 16 bits of the main word into 24, and where
// that rejects (16 of the 65536 values) the 32-bit multiply-shift of word 1
// of the fallback block.
// The 5x5 copy attempt of site (y, x), within-colour index k, colour pass p:
// ty the cell types, sa(i) the pass-start area minus target of cell i (as
// int64); accepted copies update ids and area.
template <class SA>
__device__ __forceinline__ void cpm5_attempt(const CpmArgs& a, const RepDev& R, int32_t* ids,
                                             int32_t* area, int y, int x, uint32_t k, uint32_t p,
                                             const uint32_t* lthr, const int8_t* ty,
                                             const int32_t* ljs, SA sa) {
    const int Lx = R.Lx, Ly = R.Ly, nt = R.n_types;
    uint32_t w[4];
    philox4x32_10(k >> 2, p, R.rid, kTagMain, a.key0, a.key1, w);
    const uint32_t word = w[k & 3u];
    uint32_t f[4];
    bool have_f = false;
    const uint32_t l = (word & 0xFFFFu) * 24u;
    int jn = (int)(l >> 16);
    if ((l & 0xFFFFu) < 16u) {
        philox4x32_10(k, p, R.rid, kTagFallback, a.key0, a.key1, f);
        have_f = true;
        jn = (int)(((uint64_t)f[1] * 24u) >> 32);
    }
    // row-major offsets without the centre: jn < 12 lies before it
    const int jj = jn < 12 ? jn : jn + 1;
    const int ndy = jj / 5 - 2, ndx = jj % 5 - 2;
    int rows[5], cols[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) {
        rows[d] = wrapc(y + d - 2, Ly) * Lx;
        cols[d] = wrapc(x + d - 2, Lx);
    }
    const int s = ids[(size_t)rows[2] + x];
    const int tg = ids[(size_t)wrapc(y + ndy, Ly) * Lx + wrapc(x + ndx, Lx)];
    if (tg == s) return;
    int nb[25];
#pragma unroll
    for (int dy = 0; dy < 5; ++dy)
#pragma unroll
        for (int dx = 0; dx < 5; ++dx) nb[dy * 5 + dx] = ids[(size_t)rows[dy] + cols[dx]];
    const int ts = ty[s] * nt, tt = ty[tg] * nt;
    int kadh = 0;
#pragma unroll
    for (int j = 0; j < 25; ++j) {
        if (j == 12) continue;  // the site itself
        const int m = nb[j];
        const int tm = ty[m];
        kadh += (tg != m) ? ljs[tt + tm] : 0;
        kadh -= (s != m) ? ljs[ts + tm] : 0;
    }
    int64_t karea = 0;
    if (tg != 0) karea += 2 * sa(tg) + 1;
    if (s != 0) karea += -2 * sa(s) + 1;
    const int64_t kk = (int64_t)kadh + R.LS * karea;
    bool acc;
    if (kk <= 0) {
        acc = true;
    } else if (kk >= R.K0) {
        acc = false;
    } else {
        uint32_t hi = 0u, lo = 1u;  // T = 1 for K1 <= k < K0
        if (kk < (int64_t)R.K1) {
            hi = lthr[kk - 1];
            lo = lthr[R.tab_n + kk - 1];
        }
        const uint32_t rr = word >> 16;
        acc = rr < hi;
        if (rr == hi && lo != 0u) {
            if (!have_f) philox4x32_10(k, p, R.rid, kTagFallback, a.key0, a.key1, f);
            acc = (f[0] & 0xFFFFu) < lo;
        }
    }
    if (acc) {
        ids[(size_t)rows[2] + x] = tg;
        atomicAdd(&area[tg], 1);
        atomicAdd(&area[s], -1);
    }
}

__global__ void __launch_bounds__(256) k_cpm_pass5(CpmArgs a, int c, int sweep_off) {
    extern __shared__ uint32_t lthr[];  // [2 * tab_n]: hi16 | lo16 of T(k), k = 1..K1-1
    __shared__ int32_t ljs[kMaxCpmTypes * kMaxCpmTypes];
    const TileDev T = a.tiles[blockIdx.x];
    const RepDev R = a.reps[T.rep];
    for (int i = threadIdx.x; i < 2 * R.tab_n; i += blockDim.x) lthr[i] = a.tab[R.tab_off + i];
    for (int i = threadIdx.x; i < R.n_types * R.n_types; i += blockDim.x)
        ljs[i] = a.js[R.js_off + i];
    __syncthreads();
    const uint64_t t = *a.t_base + (uint64_t)sweep_off;
    const uint64_t P = 9 * t + (uint64_t)c;
    const uint32_t p = (uint32_t)P;
    pass_rotate(a, P);
    const PassAreas pa = pass_areas(a, P, R.cell_off);
    const int cy = c / 3, cx = c - 3 * cy;
    const int Lx = R.Lx, Wc = Lx / 3;
    int32_t* ids = a.lat + R.lat_off;
    const int8_t* ty = a.ctype + R.cell_off;
    const int32_t* A = a.target + R.cell_off;
    int32_t* area = pa.d_wr;
    const int32_t* s_rd = pa.s_rd;
    const int32_t* d_rd = pa.d_rd;
    const auto sa = [=](int i) -> int64_t {
        return (int64_t)s_rd[i] + (int64_t)d_rd[i] - (int64_t)A[i];
    };
    const int total = (T.rows / 3) * Wc;
    for (int it = threadIdx.x; it < total; it += blockDim.x) {
        const int r = it / Wc;
        const int i = it - r * Wc;
        const int y = T.y0 + 3 * r + cy;
        const int x = 3 * i + cx;
        const uint32_t k = (uint32_t)((y / 3) * Wc + i);
        cpm5_attempt(a, R, ids, area, y, x, k, p, lthr, ty, ljs, sa);
    }
}

// The same pass with four consecutive same-colour sites of one row per lane
// (Lx a multiple of 8): their attempts share one Philox call (words 0..3 of
// counter k >> 2), their 3 x 9 id window comes in with six 16-byte loads and
// three halo loads, and the per-cell tables (type, pass-start area minus
// target) sit in LDS, so that a lane's attempts wait for one round of
// global loads.
__device__ __forceinline__ int sel8(const int (&v)[8], uint32_t j) {
    const int a0 = (j & 1u) ? v[1] : v[0], a1 = (j & 1u) ? v[3] : v[2];
    const int a2 = (j & 1u) ? v[5] : v[4], a3 = (j & 1u) ? v[7] : v[6];
    const int b0 = (j & 2u) ? a1 : a0, b1 = (j & 2u) ? a3 : a2;
    return (j & 4u) ? b1 : b0;
}

// The copy attempt of site x (id s, Moore neighbours nb in the order
// (dy, dx) = (-1,-1) (-1,0) (-1,1) (0,-1) (0,1) (1,-1) (1,0) (1,1)) with main
// word `word` (bits 0..2 the neighbour, bits 16..31 the prefix r of W) and
// within-colour index k (the fallback counter): the id to copy, or -1.
__device__ __forceinline__ int cpm_decide(const CpmArgs& a, const RepDev& R, const int (&nb)[8],
                                          int s, uint32_t word, uint32_t k, uint32_t p,
                                          const uint32_t* qthr, const int32_t* lsa,
                                          const int8_t* lty, const int32_t* ljs) {
    const int nt = R.n_types;
    const int tg = sel8(nb, word & 7u);
    if (tg == s) return -1;
    const int ts = lty[s] * nt, tt = lty[tg] * nt;
    int kadh = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int m = nb[j];
        const int tm = lty[m];
        kadh += (tg != m) ? ljs[tt + tm] : 0;
        kadh -= (s != m) ? ljs[ts + tm] : 0;
    }
    int64_t karea = 0;
    if (tg != 0) karea += 2 * (int64_t)lsa[tg] + 1;
    if (s != 0) karea += -2 * (int64_t)lsa[s] + 1;
    const int64_t kk = (int64_t)kadh + R.LS * karea;
    bool acc;
    if (kk <= 0) {
        acc = true;
    } else if (kk >= R.K0) {
        acc = false;
    } else {
        uint32_t hi = 0u, lo = 1u;  // T = 1 for K1 <= k < K0
        if (kk < (int64_t)R.K1) {
            hi = qthr[kk - 1];
            lo = qthr[R.tab_n + kk - 1];
        }
        const uint32_t rr = word >> 16;
        acc = rr < hi;
        if (rr == hi && lo != 0u) {
            uint32_t f[4];
            philox4x32_10(k, p, R.rid, kTagFallback, a.key0, a.key1, f);
            acc = (f[0] & 0xFFFFu) < lo;
        }
    }
    return acc ? tg : -1;
}

// ids / area: the replica's cell ids and live areas (global memory for the
// streamed pass, LDS for the resident kernel); rows y0 .. y0 + rows - 1.

// Per-cell tables of replica R into LDS for one pass of a tile: thresholds,
// adhesion, types and pass-start area minus target.  Each thread issues up
// to 4 items' loads before storing any, so that the tables arrive in one
// round of global loads.
__device__ __forceinline__ void cpm_stage(const CpmArgs& a, const RepDev& R, const PassAreas& pa,
                                          uint32_t* qthr, int32_t* lsa, int8_t* lty,
                                          int32_t* ljs) {
    const int ncell = R.q + 1;
    const int8_t* ty = a.ctype + R.cell_off;
    const int32_t* A = a.target + R.cell_off;
    const int nthr = blockDim.x;
    const int ntab = 2 * R.tab_n;
    for (int i0 = threadIdx.x; i0 < ntab; i0 += 4 * nthr) {
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * nthr;
            v[u] = i < ntab ? a.tab[R.tab_off + i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + u * nthr < ntab) qthr[i0 + u * nthr] = v[u];
    }
    for (int i = threadIdx.x; i < R.n_types * R.n_types; i += nthr) ljs[i] = a.js[R.js_off + i];
    for (int i0 = threadIdx.x; i0 < ncell; i0 += 4 * nthr) {
        int32_t sv[4], av[4];
        int8_t tv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * nthr;
            const bool in = i < ncell;
            sv[u] = in ? pa.s_rd[i] + pa.d_rd[i] : 0;
            av[u] = in ? A[i] : 0;
            tv[u] = in ? ty[i] : (int8_t)0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + u * nthr;
            if (i < ncell) {
                lsa[i] = sv[u] - av[u];
                lty[i] = tv[u];
            }
        }
    }
}


// The copy attempt of site (y, x) of colour pass p, word u of Philox block kq
// (the quad of four consecutive same-colour sites of the row): its Moore
// window from ids, the decision, and on acceptance the id and area updates.
__device__ __forceinline__ void cpm_moore_site(const CpmArgs& a, const RepDev& R, int32_t* ids,
                                               int32_t* area, int y, int x, uint32_t kq, int u,
                                               uint32_t p, const uint32_t* qthr,
                                               const int32_t* lsa, const int8_t* lty,
                                               const int32_t* ljs) {
    const int Lx = R.Lx, Ly = R.Ly;
    const int yu = y == 0 ? Ly - 1 : y - 1, yd = y + 1 == Ly ? 0 : y + 1;
    const int xl = x == 0 ? Lx - 1 : x - 1, xr = x + 1 == Lx ? 0 : x + 1;
    // int offsets: a replica holds fewer than 2^31 sites
    const int32_t* ru = ids + yu * Lx;
    const int32_t* ry = ids + y * Lx;
    const int32_t* rd = ids + yd * Lx;
    const int nb[8] = {ru[xl], ru[x], ru[xr], ry[xl], ry[xr], rd[xl], rd[x], rd[xr]};
    const int s = ry[x];
    uint32_t w[4];
    philox4x32_10(kq, p, R.rid, kTagMain, a.key0, a.key1, w);
    const uint32_t word = (u & 2) ? ((u & 1) ? w[3] : w[2]) : ((u & 1) ? w[1] : w[0]);
    const int tg = cpm_decide(a, R, nb, s, word, 4u * kq + (uint32_t)u, p, qthr, lsa, lty, ljs);
    if (tg >= 0) {
        ids[y * Lx + x] = tg;
        atomicAdd(&area[tg], 1);
        atomicAdd(&area[s], -1);
    }
}

// The colour-c sites of rows y0 .. y0 + rows - 1 (rows even), one per thread
// of the loop: site j is word j & 3 of quad j >> 2.  (Streamed from global
// memory the quad form is faster: its window loads serve four sites.)
__device__ __forceinline__ void cpm_sites(const CpmArgs& a, const RepDev& R, int32_t* ids,
                                          int32_t* area, int y0, int rows, int c, uint32_t p,
                                          const uint32_t* qthr, const int32_t* lsa,
                                          const int8_t* lty, const int32_t* ljs) {
    const int Q = R.Lx >> 3, cy = c >> 1, cx = c & 1;
    const int n = (rows >> 1) * (R.Lx >> 1);
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const int it = j >> 2, u = j & 3;
        const int r = it / Q, qi = it - r * Q;
        const int y = y0 + 2 * r + cy, x = 8 * qi + 2 * u + cx;
        cpm_moore_site(a, R, ids, area, y, x, (uint32_t)((y >> 1) * Q + qi), u, p, qthr, lsa,
                       lty, ljs);
    }
}

// One quad's inputs: its 3 x 9 id window (rows y - 1, y, y + 1; the halo
// column on the side of colour CX) and its Philox block.
struct QuadIn {
    int win[3][9];
    uint32_t w[4];
    int y, x0;
    uint32_t kq;
};

// Loads of quad `it` of the colour-(2 cy + CX) sites of rows y0 ..: six
// 16-byte loads, three halo loads and the Philox block (k >> 2 of the four
// sites); nothing here reads the staged tables.
template <int CX>
__device__ __forceinline__ void quad_load(const CpmArgs& a, const RepDev& R, const int32_t* ids,
                                          int y0, int cy, uint32_t p, int it, QuadIn& q) {
    const int Lx = R.Lx, Ly = R.Ly, Q = Lx >> 3;
    const int r = it / Q;
    const int qi = it - r * Q;
    q.y = y0 + 2 * r + cy;
    q.x0 = 8 * qi;
    q.kq = (uint32_t)((q.y >> 1) * Q + qi);
    const int yr[3] = {wrapc(q.y - 1, Ly), q.y, wrapc(q.y + 1, Ly)};
    const int xh = CX == 0 ? wrapc(q.x0 - 1, Lx) : wrapc(q.x0 + 8, Lx);
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
        const int32_t* row = ids + (size_t)yr[rr] * Lx;
        const int4 u = *reinterpret_cast<const int4*>(row + q.x0);
        const int4 v = *reinterpret_cast<const int4*>(row + q.x0 + 4);
        const int h = row[xh];
        constexpr int o = CX == 0 ? 1 : 0;
        q.win[rr][o + 0] = u.x;
        q.win[rr][o + 1] = u.y;
        q.win[rr][o + 2] = u.z;
        q.win[rr][o + 3] = u.w;
        q.win[rr][o + 4] = v.x;
        q.win[rr][o + 5] = v.y;
        q.win[rr][o + 6] = v.z;
        q.win[rr][o + 7] = v.w;
        q.win[rr][CX == 0 ? 0 : 8] = h;
    }
    philox4x32_10(q.kq, p, R.rid, kTagMain, a.key0, a.key1, q.w);
}

// The quad's four attempts (site 2u + CX of the quad is word u) and, on
// acceptance, the id update and the area changes (LDS atomics into the
// workgroup's per-cell sums).
template <int CX>
__device__ __forceinline__ void quad_decide(const CpmArgs& a, const RepDev& R, int32_t* ids,
                                            int32_t* area, uint32_t p, const QuadIn& q,
                                            const uint32_t* qthr, const int32_t* lsa,
                                            const int8_t* lty, const int32_t* ljs) {
    const int Lx = R.Lx;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        // Moore order (dy, dx): (-1,-1) (-1,0) (-1,1) (0,-1) (0,1) (1,-1) (1,0) (1,1)
        const int nb[8] = {q.win[0][2 * u], q.win[0][2 * u + 1], q.win[0][2 * u + 2],
                           q.win[1][2 * u], q.win[1][2 * u + 2],
                           q.win[2][2 * u], q.win[2][2 * u + 1], q.win[2][2 * u + 2]};
        const int s = q.win[1][2 * u + 1];
        const int tg = cpm_decide(a, R, nb, s, q.w[u], 4u * q.kq + (uint32_t)u, p, qthr, lsa, lty,
                                  ljs);
        if (tg >= 0) {
            ids[(size_t)q.y * Lx + q.x0 + 2 * u + CX] = tg;
            atomicAdd(&area[tg], 1);
            atomicAdd(&area[s], -1);
        }
    }
}

// A lane's first quad is loaded (window and Philox block) before the
// per-cell tables are staged, so that the two rounds of global loads
// overlap; the other quads of the lane follow the table barrier.  Area
// changes gather in LDS (one sum per cell of the replica) and go to the
// pass's change buffer as one global atomic per touched cell at the end:
// integer sums, so the buffer ends equal to one atomic per copy, with far
// fewer atomics on the cells' words.
template <int CX>
__device__ __forceinline__ void quad_pass(const CpmArgs& a, int c, int sweep_off,
                                          uint32_t* qthr, int32_t* lsa, int8_t* lty,
                                          int32_t* ljs, int32_t* ldel) {
    const TileDev T = a.tiles[blockIdx.x];
    const RepDev R = a.reps[T.rep];
    const uint64_t t = *a.t_base + (uint64_t)sweep_off;
    const uint64_t P = 4 * t + (uint64_t)c;
    const uint32_t p = (uint32_t)P;
    const PassAreas pa = pass_areas(a, P, R.cell_off);
    int32_t* ids = a.lat + R.lat_off;
    const int cy = c >> 1;
    const int total = (T.rows >> 1) * (R.Lx >> 3);
    const int it0 = (int)threadIdx.x;
    QuadIn q;
    if (it0 < total) quad_load<CX>(a, R, ids, T.y0, cy, p, it0, q);
    cpm_stage(a, R, pa, qthr, lsa, lty, ljs);
    pass_rotate(a, P);
    const int ncell = R.q + 1;
    for (int i = (int)threadIdx.x; i < ncell; i += (int)blockDim.x) ldel[i] = 0;
    __syncthreads();
    if (it0 < total) quad_decide<CX>(a, R, ids, ldel, p, q, qthr, lsa, lty, ljs);
    for (int it = it0 + (int)blockDim.x; it < total; it += blockDim.x) {
        quad_load<CX>(a, R, ids, T.y0, cy, p, it, q);
        quad_decide<CX>(a, R, ids, ldel, p, q, qthr, lsa, lty, ljs);
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < ncell; i += (int)blockDim.x) {
        const int d = ldel[i];
        if (d != 0) atomicAdd(&pa.d_wr[i], d);
    }
}

// One lane per site (the "site" form of the quad pass): lane u of each
// group of four takes site 2u + CX of a quad, computes the quad's Philox
// block itself and keeps word u, loads its own 3 x 3 window and decides one
// attempt, so that a workgroup of 1024 lanes carries four times the
// attempts in flight of the quad form at the same tile, each lane's
// chain of table lookups a quarter as long.  Same decisions, same stores;
// area changes gather in LDS as in the quad form.
struct SiteIn {
    int nb[8];
    int s;
    uint32_t w;
    int y, x;
    uint32_t kq;
};

template <int CX>
__device__ __forceinline__ void site_load(const CpmArgs& a, const RepDev& R, const int32_t* ids,
                                          int y0, int cy, uint32_t p, int it, int u, SiteIn& q) {
    const int Lx = R.Lx, Ly = R.Ly, Q = Lx >> 3;
    const int r = it / Q;
    const int qi = it - r * Q;
    q.y = y0 + 2 * r + cy;
    q.x = 8 * qi + 2 * u + CX;
    q.kq = (uint32_t)((q.y >> 1) * Q + qi);
    const int yu = wrapc(q.y - 1, Ly), yd = wrapc(q.y + 1, Ly);
    const int xl = wrapc(q.x - 1, Lx), xr = wrapc(q.x + 1, Lx);
    const int32_t* ru = ids + (size_t)yu * Lx;
    const int32_t* ry = ids + (size_t)q.y * Lx;
    const int32_t* rd = ids + (size_t)yd * Lx;
    // Moore order (dy, dx): (-1,-1) (-1,0) (-1,1) (0,-1) (0,1) (1,-1) (1,0) (1,1)
    q.nb[0] = ru[xl];
    q.nb[1] = ru[q.x];
    q.nb[2] = ru[xr];
    q.nb[3] = ry[xl];
    q.nb[4] = ry[xr];
    q.nb[5] = rd[xl];
    q.nb[6] = rd[q.x];
    q.nb[7] = rd[xr];
    q.s = ry[q.x];
    uint32_t w[4];
    philox4x32_10(q.kq, p, R.rid, kTagMain, a.key0, a.key1, w);
    q.w = u == 0 ? w[0] : (u == 1 ? w[1] : (u == 2 ? w[2] : w[3]));
}

template <int CX>
__device__ __forceinline__ void site_pass(const CpmArgs& a, int c, int sweep_off,
                                          uint32_t* qthr, int32_t* lsa, int8_t* lty,
                                          int32_t* ljs, int32_t* ldel) {
    const TileDev T = a.tiles[blockIdx.x];
    const RepDev R = a.reps[T.rep];
    const uint64_t t = *a.t_base + (uint64_t)sweep_off;
    const uint64_t P = 4 * t + (uint64_t)c;
    const uint32_t p = (uint32_t)P;
    const PassAreas pa = pass_areas(a, P, R.cell_off);
    int32_t* ids = a.lat + R.lat_off;
    const int cy = c >> 1;
    const int total = (T.rows >> 1) * (R.Lx >> 3);  // quads of the tile
    const int u = (int)threadIdx.x & 3, qs = (int)blockDim.x >> 2;
    int it = (int)threadIdx.x >> 2;
    SiteIn q;
    if (it < total) site_load<CX>(a, R, ids, T.y0, cy, p, it, u, q);
    cpm_stage(a, R, pa, qthr, lsa, lty, ljs);
    pass_rotate(a, P);
    const int ncell = R.q + 1;
    for (int i = (int)threadIdx.x; i < ncell; i += (int)blockDim.x) ldel[i] = 0;
    __syncthreads();
    while (it < total) {
        const int tg = cpm_decide(a, R, q.nb, q.s, q.w, 4u * q.kq + (uint32_t)u, p, qthr, lsa,
                                  lty, ljs);
        if (tg >= 0) {
            ids[(size_t)q.y * R.Lx + q.x] = tg;
            atomicAdd(&ldel[tg], 1);
            atomicAdd(&ldel[q.s], -1);
        }
        it += qs;
        if (it < total) site_load<CX>(a, R, ids, T.y0, cy, p, it, u, q);
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < ncell; i += (int)blockDim.x) {
        const int d = ldel[i];
        if (d != 0) atomicAdd(&pa.d_wr[i], d);
    }
}

__global__ void __launch_bounds__(256) k_cpm_pass_quad(CpmArgs a, int c, int sweep_off,
                                                       int tab_lds_bytes, int cell_cap) {
    // dynamic LDS: [T hi | T lo] (tab_lds_bytes) | snap - A (int32) | type (int8) |
    // area changes of the pass (int32); cell_cap is a multiple of 16
    extern __shared__ __align__(16) uint8_t dyn[];
    uint32_t* qthr = reinterpret_cast<uint32_t*>(dyn);
    int32_t* lsa = reinterpret_cast<int32_t*>(dyn + tab_lds_bytes);
    int8_t* lty = reinterpret_cast<int8_t*>(lsa + cell_cap);
    int32_t* ldel = reinterpret_cast<int32_t*>(lty + cell_cap);
    __shared__ int32_t ljs[kMaxCpmTypes * kMaxCpmTypes];
    if (c & 1)
        quad_pass<1>(a, c, sweep_off, qthr, lsa, lty, ljs, ldel);
    else
        quad_pass<0>(a, c, sweep_off, qthr, lsa, lty, ljs, ldel);
}

__global__ void __launch_bounds__(1024) k_cpm_pass_site(CpmArgs a, int c, int sweep_off,
                                                        int tab_lds_bytes, int cell_cap) {
    // dynamic LDS as k_cpm_pass_quad
    extern __shared__ __align__(16) uint8_t dyn[];
    uint32_t* qthr = reinterpret_cast<uint32_t*>(dyn);
    int32_t* lsa = reinterpret_cast<int32_t*>(dyn + tab_lds_bytes);
    int8_t* lty = reinterpret_cast<int8_t*>(lsa + cell_cap);
    int32_t* ldel = reinterpret_cast<int32_t*>(lty + cell_cap);
    __shared__ int32_t ljs[kMaxCpmTypes * kMaxCpmTypes];
    if (c & 1)
        site_pass<1>(a, c, sweep_off, qthr, lsa, lty, ljs, ldel);
    else
        site_pass<0>(a, c, sweep_off, qthr, lsa, lty, ljs, ldel);
}

// All n_steps unrecorded Monte Carlo steps of every replica in one launch:
// one 1024-thread workgroup per replica with its ids, areas, cell tables and
// thresholds in LDS.  Per pass the snapshot (area minus target) is taken in
// LDS; then one site per thread.  Range 1 (Lx % 8 == 0): the four lanes of a
// quad (four consecutive same-colour sites of a row, one Philox block)
// compute the block alike and take one word each; range 2: the attempt of
// the streamed 5x5 pass on the LDS ids.  A replica has 16 waves to hide the
// latency of its table lookups; accepted copies update the areas with LDS
// atomics, and a barrier closes the pass.  The same
// decisions as the streamed passes; ids and areas are written back at the
// end (the stored snapshot equals the areas then).
template <int RANGE>
__global__ void __launch_bounds__(1024) k_cpm_resident(CpmArgs a, int n_steps,
                                                       int tab_lds_bytes, int cell_cap) {
    // dynamic LDS: [T hi | T lo] (tab_lds_bytes) | snap - A | area | A (int32 [cell_cap] each)
    // | type (int8 [cell_cap], padded to 16) | ids (int32 [Ly Lx])
    extern __shared__ __align__(16) uint8_t dyn[];
    uint32_t* qthr = reinterpret_cast<uint32_t*>(dyn);
    int32_t* lsa = reinterpret_cast<int32_t*>(dyn + tab_lds_bytes);
    int32_t* larea = lsa + cell_cap;
    int32_t* lA = larea + cell_cap;
    int8_t* lty = reinterpret_cast<int8_t*>(lA + cell_cap);
    int32_t* lids = reinterpret_cast<int32_t*>(lty + ((cell_cap + 15) & ~15));
    __shared__ int32_t ljs[kMaxCpmTypes * kMaxCpmTypes];
    const RepDev R = a.reps[blockIdx.x];
    const int Lx = R.Lx, Ly = R.Ly;
    const int ncell = R.q + 1, n = Lx * Ly, nthr = (int)blockDim.x;
    int32_t* gids = a.lat + R.lat_off;
    int32_t* garea = a.area + R.cell_off;
    for (int i = threadIdx.x; i < 2 * R.tab_n; i += nthr) qthr[i] = a.tab[R.tab_off + i];
    for (int i = threadIdx.x; i < R.n_types * R.n_types; i += nthr) ljs[i] = a.js[R.js_off + i];
    for (int i = threadIdx.x; i < ncell; i += nthr) {
        larea[i] = garea[i];
        lA[i] = a.target[R.cell_off + i];
        lty[i] = a.ctype[R.cell_off + i];
    }
    for (int i = threadIdx.x; i < n / 4; i += nthr)
        reinterpret_cast<int4*>(lids)[i] = reinterpret_cast<const int4*>(gids)[i];
    __syncthreads();
    const uint64_t t0 = *a.t_base;
    constexpr int ncol = RANGE == 2 ? 9 : 4;
    const int n_sites = n / ncol;  // sites of one colour
    const auto sa = [=](int i) -> int64_t { return (int64_t)lsa[i]; };
    for (int st = 0; st < n_steps; ++st) {
        for (int c = 0; c < ncol; ++c) {
            for (int i = threadIdx.x; i < ncell; i += nthr) lsa[i] = larea[i] - lA[i];
            __syncthreads();
            const uint32_t p = (uint32_t)(ncol * (t0 + (uint64_t)st) + (uint64_t)c);
            if (RANGE == 2) {
                // the 3x3 sublattice: colour c = 3 (y mod 3) + (x mod 3)
                const int cy = c / 3, cx = c - 3 * cy, Wc = Lx / 3;
                for (int j = threadIdx.x; j < n_sites; j += nthr) {
                    const int r = j / Wc, i = j - r * Wc;
                    cpm5_attempt(a, R, lids, larea, 3 * r + cy, 3 * i + cx, (uint32_t)j, p, qthr,
                                 lty, ljs, sa);
                }
                __syncthreads();
                continue;
            }
            cpm_sites(a, R, lids, larea, 0, Ly, c, p, qthr, lsa, lty, ljs);
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n / 4; i += nthr)
        reinterpret_cast<int4*>(gids)[i] = reinterpret_cast<const int4*>(lids)[i];
    for (int i = threadIdx.x; i < ncell; i += nthr) {
        garea[i] = larea[i];
        a.snap[R.cell_off + i] = larea[i];
    }
}

// ------------------------------------------- tiled persistent streamed passes
// All 4 G colour passes of G unrecorded Monte Carlo steps in one launch for
// lattices too large for one workgroup's LDS (range 1, Lx % 8 == 0): every
// replica is cut into TH x TW tiles, one workgroup per tile for the whole
// launch, its ids (with a one-cell halo) in LDS.  A pass: the tile's sites
// of the colour attempt their copies on the LDS ids (the decision of the
// streamed passes, cpm_decide), the tile's border cells go to the global
// lattice and its area changes to the pass's change buffer; then the
// replica's workgroups meet at a barrier (a counter per replica, agent-scope
// release / acquire), after which each reads its halo ring, which the
// neighbouring tiles wrote, and stages the next pass's snapshot.  Snapshots
// rotate as in the streamed passes (S[P & 1] + D[(P-1) % 3], the side work of
// pass P spread over the replica's tiles).  Every tile workgroup of the
// launch must be resident at once (the host sizes the grid within the chip's
// occupancy); a barrier wait beyond its bound (about two seconds) raises
// *abort and every waiting workgroup leaves, so a launch always ends.
constexpr uint32_t kCpmSpinCap = 1u << 25;

__device__ __forceinline__ void cpm_wait_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ int cpm_tile_barrier(uint32_t* bar, uint32_t need, uint32_t* abort_flag) {
    // release: the fence writes the L2 back (border ids, snapshot and change
    // buffers reach memory for the other XCDs), the explicit vmcnt(0) waits
    // for that write-back to finish, and only then is the arrival counted.
    // (A release add alone compiles to the write-back directly followed by
    // the add, with no wait between them, when the workgroup's stores were
    // already waited for, so a workgroup on another XCD could pass the
    // barrier and read memory the write-back had not reached.)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    cpm_wait_stores();
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (uint32_t spin = 0;; ++spin) {
        if (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) break;
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return 0;
        if (spin >= kCpmSpinCap) {
            __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return 0;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return 1;
}

__global__ void __launch_bounds__(256) k_cpm_tiled(CpmArgs a, int n_steps, int TH, int TW,
                                                   int tab_lds_bytes, int cell_cap,
                                                   uint32_t* bar, uint32_t* abort_flag) {
    // dynamic LDS: [T hi | T lo] (tab_lds_bytes) | snap - A (int32 [cell_cap]) |
    // type (int8 [cell_cap], padded to 16) | ids with halo (int32 [TH + 2][TW + 2])
    extern __shared__ __align__(16) uint8_t dyn[];
    uint32_t* qthr = reinterpret_cast<uint32_t*>(dyn);
    int32_t* lsa = reinterpret_cast<int32_t*>(dyn + tab_lds_bytes);
    int8_t* lty = reinterpret_cast<int8_t*>(lsa + cell_cap);
    int32_t* tile = reinterpret_cast<int32_t*>(lty + ((cell_cap + 15) & ~15));
    __shared__ int32_t ljs[kMaxCpmTypes * kMaxCpmTypes];
    __shared__ int go;
    // block b: replica b % R, tile b / R (with R a multiple of 8 a replica's
    // tiles share one XCD)
    const int r = (int)blockIdx.x % a.R, tix = (int)blockIdx.x / a.R;
    const RepDev R = a.reps[r];
    const int Lx = R.Lx, Ly = R.Ly, ntx = Lx / TW, n_tiles = ntx * (Ly / TH);
    const int y0 = (tix / ntx) * TH, x0 = (tix % ntx) * TW;
    const int ts = TW + 2, nthr = (int)blockDim.x, tid = (int)threadIdx.x;
    const int ncell = R.q + 1;
    int32_t* gids = a.lat + R.lat_off;
    const int32_t* A = a.target + R.cell_off;
    for (int i = tid; i < 2 * R.tab_n; i += nthr) qthr[i] = a.tab[R.tab_off + i];
    for (int i = tid; i < R.n_types * R.n_types; i += nthr) ljs[i] = a.js[R.js_off + i];
    for (int i = tid; i < ncell; i += nthr) lty[i] = a.ctype[R.cell_off + i];
    // the tile with its halo (periodic)
    for (int i = tid; i < (TH + 2) * ts; i += nthr) {
        const int ly = i / ts, lx = i - ly * ts;
        const int gy = wrapc(y0 + ly - 1, Ly), gx = wrapc(x0 + lx - 1, Lx);
        tile[i] = gids[gy * Lx + gx];
    }
    const uint64_t t0 = *a.t_base;
    const int Q = Lx >> 3;                 // quads per global row
    const int nq = (TH >> 1) * (TW >> 3);  // quads of one colour in the tile
    // this tile's share of the replica's cells for the side work
    const int per = (ncell + n_tiles - 1) / n_tiles;
    const int c0 = tix * per, c1 = min(ncell, c0 + per);
    for (int sw = 0; sw < n_steps; ++sw) {
        for (int c = 0; c < 4; ++c) {
            const uint32_t j = (uint32_t)(4 * sw + c);
            const uint64_t P = 4 * (t0 + (uint64_t)sw) + (uint64_t)c;
            const uint32_t p = (uint32_t)P;
            const PassAreas pa = pass_areas(a, P, R.cell_off);
            if (j > 0) {
                // the halo ring, written by the neighbouring tiles' last pass
                const int ring = 2 * ts + 2 * TH;
                for (int i = tid; i < ring; i += nthr) {
                    int ly, lx;
                    if (i < ts) {
                        ly = 0;
                        lx = i;
                    } else if (i < 2 * ts) {
                        ly = TH + 1;
                        lx = i - ts;
                    } else {
                        const int k = i - 2 * ts;
                        ly = 1 + (k >> 1);
                        lx = (k & 1) ? TW + 1 : 0;
                    }
                    tile[ly * ts + lx] =
                        gids[wrapc(y0 + ly - 1, Ly) * Lx + wrapc(x0 + lx - 1, Lx)];
                }
            }
            for (int i = tid; i < ncell; i += nthr) lsa[i] = pa.s_rd[i] + pa.d_rd[i] - A[i];
            // side work of pass P for this tile's cells
            {
                const size_t n = (size_t)a.total_cells;
                int32_t* s_wr = a.sbuf + (size_t)((P + 1u) & 1u) * n + R.cell_off;
                int32_t* d_clr = a.dbuf + (size_t)((P + 1u) % 3u) * n + R.cell_off;
                for (int i = c0 + tid; i < c1; i += nthr) {
                    s_wr[i] = pa.s_rd[i] + pa.d_rd[i];
                    d_clr[i] = 0;
                }
            }
            __syncthreads();
            // the colour's quads of the tile: four consecutive same-colour
            // sites of a row share Philox block k >> 2 (global counters)
            const int cy = c >> 1, cx = c & 1;
            for (int it = tid; it < nq; it += nthr) {
                const int rr = it / (TW >> 3), qi = it - rr * (TW >> 3);
                const int gy = y0 + 2 * rr + cy;
                const int gx0 = x0 + 8 * qi;
                const uint32_t kq = (uint32_t)((gy >> 1) * Q + (gx0 >> 3));
                uint32_t w[4];
                philox4x32_10(kq, p, R.rid, kTagMain, a.key0, a.key1, w);
                const int ly = gy - y0 + 1;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int lx = gx0 - x0 + 2 * u + cx + 1;
                    const int32_t* ru = tile + (ly - 1) * ts;
                    const int32_t* ry = tile + ly * ts;
                    const int32_t* rd = tile + (ly + 1) * ts;
                    const int nb[8] = {ru[lx - 1], ru[lx], ru[lx + 1], ry[lx - 1], ry[lx + 1],
                                       rd[lx - 1], rd[lx], rd[lx + 1]};
                    const int s = ry[lx];
                    const int tg = cpm_decide(a, R, nb, s, w[u], 4u * kq + (uint32_t)u, p, qthr,
                                              lsa, lty, ljs);
                    if (tg >= 0) {
                        tile[ly * ts + lx] = tg;
                        atomicAdd(&pa.d_wr[tg], 1);
                        atomicAdd(&pa.d_wr[s], -1);
                    }
                }
            }
            __syncthreads();
            // the tile's border cells for the neighbouring tiles
            for (int i = tid; i < 2 * TW + 2 * (TH - 2); i += nthr) {
                int ly, lx;
                if (i < TW) {
                    ly = 1;
                    lx = 1 + i;
                } else if (i < 2 * TW) {
                    ly = TH;
                    lx = 1 + i - TW;
                } else {
                    const int k = i - 2 * TW;
                    ly = 2 + (k >> 1);
                    lx = (k & 1) ? TW : 1;
                }
                gids[(y0 + ly - 1) * Lx + x0 + lx - 1] = tile[ly * ts + lx];
            }
            cpm_wait_stores();
            __syncthreads();
            if (tid == 0)
                go = cpm_tile_barrier(bar + r, (uint32_t)n_tiles * (j + 1u), abort_flag);
            __syncthreads();
            if (!go) return;  // uniform: the whole workgroup leaves
        }
    }
    // the tile's interior (its border is already in place)
    for (int i = tid; i < TH * TW; i += nthr) {
        const int ly = 1 + i / TW, lx = 1 + i % TW;
        gids[(y0 + ly - 1) * Lx + x0 + lx - 1] = tile[ly * ts + lx];
    }
}

size_t cpm_tiled_lds_bytes(int tab_lds_bytes, int cell_cap, int TH, int TW) {
    return (size_t)tab_lds_bytes + (size_t)4 * cell_cap + (size_t)((cell_cap + 15) & ~15) +
           (size_t)4 * (TH + 2) * (TW + 2);
}

hipError_t cpm_tiled_occupancy(int tab_lds_bytes, int cell_cap, int TH, int TW, int* per_cu) {
    const size_t lds = cpm_tiled_lds_bytes(tab_lds_bytes, cell_cap, TH, TW);
    hipError_t e = hipFuncSetAttribute((const void*)k_cpm_tiled,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, (const void*)k_cpm_tiled, 256, lds);
}

hipError_t launch_cpm_tiled(const CpmArgs& a, int n_steps, int TH, int TW, int tab_lds_bytes,
                            int cell_cap, int n_blocks, uint32_t* bar, uint32_t* abort_flag,
                            hipStream_t s) {
    const size_t lds = cpm_tiled_lds_bytes(tab_lds_bytes, cell_cap, TH, TW);
    hipLaunchKernelGGL(k_cpm_tiled, dim3(n_blocks), dim3(256), lds, s, a, n_steps, TH, TW,
                       tab_lds_bytes, cell_cap, bar, abort_flag);
    return hipGetLastError();
}

size_t cpm_resident_lds_bytes(int tab_lds_bytes, int cell_cap, int max_sites) {
    return (size_t)tab_lds_bytes + (size_t)12 * cell_cap + (size_t)((cell_cap + 15) & ~15) +
           (size_t)4 * max_sites;
}

hipError_t launch_cpm_resident(const CpmArgs& a, int n_steps, int tab_lds_bytes, int cell_cap,
                               int max_sites, hipStream_t s) {
    const size_t lds = cpm_resident_lds_bytes(tab_lds_bytes, cell_cap, max_sites);
    const void* fn = a.range == 2 ? (const void*)k_cpm_resident<2> : (const void*)k_cpm_resident<1>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (a.range == 2)
        hipLaunchKernelGGL(k_cpm_resident<2>, dim3(a.R), dim3(1024), lds, s, a, n_steps,
                           tab_lds_bytes, cell_cap);
    else
        hipLaunchKernelGGL(k_cpm_resident<1>, dim3(a.R), dim3(1024), lds, s, a, n_steps,
                           tab_lds_bytes, cell_cap);
    return hipGetLastError();
}

__global__ void k_cpm_copy(const int32_t* src, int32_t* dst, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__device__ __forceinline__ uint64_t first_pass(const CpmArgs& a, int sweep_off) {
    return (uint64_t)(a.range == 2 ? 9 : 4) * (*a.t_base + (uint64_t)sweep_off);
}

__global__ void k_cpm_pass_init(CpmArgs a, int sweep_off) {
    const uint64_t P = first_pass(a, sweep_off);
    const size_t n = (size_t)a.total_cells;
    int32_t* s_wr = a.sbuf + (size_t)(P & 1u) * n;
    int32_t* d0 = a.dbuf + (size_t)((P + 2u) % 3u) * n;
    int32_t* d1 = a.dbuf + (size_t)(P % 3u) * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        s_wr[i] = a.area[i];
        d0[i] = 0;
        d1[i] = 0;
    }
}

__global__ void k_cpm_pass_final(CpmArgs a, int sweep_off) {
    const uint64_t P = first_pass(a, sweep_off);
    const size_t n = (size_t)a.total_cells;
    const int32_t* s_rd = a.sbuf + (size_t)(P & 1u) * n;
    const int32_t* d_rd = a.dbuf + (size_t)((P + 2u) % 3u) * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        a.area[i] = s_rd[i] + d_rd[i];
}

// Areas from the lattice (after set_state): per tile, atomics into area
// (which the caller cleared).
__global__ void k_cpm_area_count(CpmArgs a) {
    const TileDev T = a.tiles[blockIdx.x];
    const RepDev R = a.reps[T.rep];
    const int32_t* ids = a.lat + R.lat_off;
    int32_t* area = a.area + R.cell_off;
    const int n = T.rows * R.Lx;
    const size_t base = (size_t)T.y0 * R.Lx;
    for (int i = threadIdx.x; i < n; i += blockDim.x) atomicAdd(&area[ids[base + i]], 1);
}

// Statistics: boundary bonds by type pair (von Neumann, right and down) and
// the adhesion energy over Moore pairs counted once (right, down,
// down-right, down-left), in fixed point; the area term is added by
// k_cpm_area_energy.  stats row: [10 pair counts, H lo, H hi, ...].
__global__ void __launch_bounds__(256) k_cpm_stats(CpmArgs a, int rec_row) {
    __shared__ int32_t ljs[kMaxCpmTypes * kMaxCpmTypes];
    __shared__ int lpair[10];
    __shared__ unsigned long long lH;
    const TileDev T = a.tiles[blockIdx.x];
    const RepDev R = a.reps[T.rep];
    const int nt = R.n_types;
    for (int i = threadIdx.x; i < nt * nt; i += blockDim.x) ljs[i] = a.js[R.js_off + i];
    if (threadIdx.x < 10) lpair[threadIdx.x] = 0;
    if (threadIdx.x == 0) lH = 0ull;
    __syncthreads();
    const int Lx = R.Lx, Ly = R.Ly;
    const int32_t* ids = a.lat + R.lat_off;
    const int8_t* ty = a.ctype + R.cell_off;
    long long H = 0;
    const int n = T.rows * Lx;
    for (int it = threadIdx.x; it < n; it += blockDim.x) {
        const int y = T.y0 + it / Lx, x = it % Lx;
        const int yp = wrapc(y + 1, Ly), xp = wrapc(x + 1, Lx), xm = wrapc(x - 1, Lx);
        const int s = ids[(size_t)y * Lx + x];
        const int ts = ty[s];
        const int r = ids[(size_t)y * Lx + xp], d = ids[(size_t)yp * Lx + x];
        const int dr = ids[(size_t)yp * Lx + xp], dl = ids[(size_t)yp * Lx + xm];
        if (r != s) {
            int p0 = ts, p1 = ty[r];
            if (p0 > p1) { const int tmp = p0; p0 = p1; p1 = tmp; }
            atomicAdd(&lpair[p0 * nt - p0 * (p0 - 1) / 2 + (p1 - p0)], 1);
            H += ljs[ts * nt + ty[r]];
        }
        if (d != s) {
            int p0 = ts, p1 = ty[d];
            if (p0 > p1) { const int tmp = p0; p0 = p1; p1 = tmp; }
            atomicAdd(&lpair[p0 * nt - p0 * (p0 - 1) / 2 + (p1 - p0)], 1);
            H += ljs[ts * nt + ty[d]];
        }
        if (dr != s) H += ljs[ts * nt + ty[dr]];
        if (dl != s) H += ljs[ts * nt + ty[dl]];
        if (a.range == 2) {
            // the second shell's forward half: (0,2), (1,+-2), (2,-2..2)
            const int x2 = wrapc(x + 2, Lx), xm2 = wrapc(x - 2, Lx), y2 = wrapc(y + 2, Ly);
            const int o[8] = {ids[(size_t)y * Lx + x2],   ids[(size_t)yp * Lx + xm2],
                              ids[(size_t)yp * Lx + x2],  ids[(size_t)y2 * Lx + xm2],
                              ids[(size_t)y2 * Lx + xm],  ids[(size_t)y2 * Lx + x],
                              ids[(size_t)y2 * Lx + xp],  ids[(size_t)y2 * Lx + x2]};
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (o[j] != s) H += ljs[ts * nt + ty[o[j]]];
        }
    }
    atomicAdd(&lH, (unsigned long long)H);
    __syncthreads();
    int32_t* row = a.stats + ((size_t)rec_row * a.R + T.rep) * a.width;
    if (threadIdx.x < 10 && lpair[threadIdx.x]) atomicAdd(&row[threadIdx.x], lpair[threadIdx.x]);
    if (threadIdx.x == 0) atomicAdd(reinterpret_cast<unsigned long long*>(row + 10), lH);
}

// lambda S sum over cells (not the medium) of (a - A)^2, one block per replica.
__global__ void k_cpm_area_energy(CpmArgs a, int rec_row) {
    __shared__ unsigned long long lH;
    const int r = blockIdx.x;
    const RepDev R = a.reps[r];
    if (threadIdx.x == 0) lH = 0ull;
    __syncthreads();
    const int32_t* area = a.area + R.cell_off;
    const int32_t* A = a.target + R.cell_off;
    long long H = 0;
    for (int i = 1 + threadIdx.x; i <= R.q; i += blockDim.x) {
        const long long d = (long long)area[i] - (long long)A[i];
        H += R.LS * d * d;
    }
    atomicAdd(&lH, (unsigned long long)H);
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t* row = a.stats + ((size_t)rec_row * a.R + r) * a.width;
        atomicAdd(reinterpret_cast<unsigned long long*>(row + 10), lH);
    }
}

hipError_t launch_cpm_pass(const CpmArgs& a, int n_tiles, int c, int sweep_off, int threads,
                           size_t lds_tab_bytes, hipStream_t s) {
    hipLaunchKernelGGL(k_cpm_pass, dim3(n_tiles), dim3(threads), lds_tab_bytes, s, a, c,
                       sweep_off);
    return hipGetLastError();
}

hipError_t launch_cpm_pass5(const CpmArgs& a, int n_tiles, int c, int sweep_off, int threads,
                            size_t lds_tab_bytes, hipStream_t s) {
    hipLaunchKernelGGL(k_cpm_pass5, dim3(n_tiles), dim3(threads), lds_tab_bytes, s, a, c,
                       sweep_off);
    return hipGetLastError();
}

size_t cpm_quad_lds_bytes(int tab_lds_bytes, int cell_cap) {
    return (size_t)tab_lds_bytes + (size_t)cell_cap * 9;
}

hipError_t launch_cpm_pass_quad(const CpmArgs& a, int n_tiles, int c, int sweep_off,
                                int threads, int tab_lds_bytes, int cell_cap, hipStream_t s) {
    const size_t lds = cpm_quad_lds_bytes(tab_lds_bytes, cell_cap);
    if (threads > 256)
        hipLaunchKernelGGL(k_cpm_pass_site, dim3(n_tiles), dim3(threads), lds, s, a, c, sweep_off,
                           tab_lds_bytes, cell_cap);
    else
        hipLaunchKernelGGL(k_cpm_pass_quad, dim3(n_tiles), dim3(threads), lds, s, a, c, sweep_off,
                           tab_lds_bytes, cell_cap);
    return hipGetLastError();
}

hipError_t cpm_reserve_lds(size_t lds_bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)k_cpm_pass_quad,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_cpm_pass_site,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    return e;
}

hipError_t launch_cpm_snapshot(const CpmArgs& a, int total_cells, hipStream_t s) {
    int blocks = (total_cells + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_cpm_copy, dim3(blocks), dim3(256), 0, s, a.area, a.snap, total_cells);
    return hipGetLastError();
}

hipError_t launch_cpm_pass_init(const CpmArgs& a, int sweep_off, hipStream_t s) {
    int blocks = (a.total_cells + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_cpm_pass_init, dim3(blocks), dim3(256), 0, s, a, sweep_off);
    return hipGetLastError();
}

hipError_t launch_cpm_pass_final(const CpmArgs& a, int sweep_off, hipStream_t s) {
    int blocks = (a.total_cells + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_cpm_pass_final, dim3(blocks), dim3(256), 0, s, a, sweep_off);
    return hipGetLastError();
}

hipError_t launch_cpm_area_recount(const CpmArgs& a, int n_tiles, int total_cells, hipStream_t s) {
    hipError_t e = launch_fill_i32(a.area, (size_t)total_cells, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cpm_area_count, dim3(n_tiles), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_cpm_snapshot(a, total_cells, s);
}

hipError_t launch_cpm_stats(const CpmArgs& a, int n_tiles, int rec_row, hipStream_t s) {
    hipLaunchKernelGGL(k_cpm_stats, dim3(n_tiles), dim3(256), 0, s, a, rec_row);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cpm_area_energy, dim3(a.R), dim3(256), 0, s, a, rec_row);
    return hipGetLastError();
}

}  // namespace spinmc

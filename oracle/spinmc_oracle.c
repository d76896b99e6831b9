/*
 * spinmc oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU implementation of the
 * checkerboard Metropolis-Hastings chain for the Ising, q-state Potts and
 * Cellular Potts models of "A differentiable programming framework for spin
 * models" (Farias, Schultz, Mombach, Maziero).  Only the test-suite, the
 * smoke entry point and the CPU-baseline leg of the benchmark may load this
 * library; the product path (the HIP library) never calls it and shares no
 * code with it.
 *
 * What is computed (paper references by section / equation / algorithm):
 *   - Ising energy, Eq. (1), with the ferromagnetic sign convention
 *     H = -Jx sum_h s s' - Jy sum_v s s' - h sum s (every bond once).
 *   - Potts energy, Eq. (2): H = -J sum delta(s,s') - h sum s (labels 0..q-1).
 *   - Cellular Potts energy, Eq. (3): adhesion over the Moore neighbourhood
 *     (each unordered pair once) plus lambda * sum_{cells} (a - A)^2,
 *     no area term for the medium (id 0).
 *   - Algorithm 1 (Methods, "Standard Metropolis-Hastings algorithm with
 *     parallelization"): propose, energy change from the neighbourhood,
 *     checkerboard colouring, accept when dE <= 0, else with exp(-beta dE).
 *     Checkerboard colouring as in the Related-Work section (Fig. 1): sites of
 *     one colour have no interacting neighbour of the same colour, so updating
 *     them one after another in place equals updating them all at once.
 *   - Potts proposals: a uniformly chosen state different from the current one
 *     (Methods, Potts model).
 *   - CPM copy attempts (Methods, Cellular Potts model): target site, random
 *     Moore neighbour, copy its id through the Algorithm-1 test.
 *
 * Readings where the paper is silent (the same readings bind the HIP path):
 *   - random numbers: Philox4x32-10 (Salmon et al., SC'11), counters below;
 *   - a uniform 32-bit word W is built as (main 16-bit prefix << 16) | 16-bit
 *     fallback half; accept iff W < T with T = ceil(2^32 exp(-beta dE)) built
 *     in FP64 (T = 2^32 when dE <= 0);
 *   - colour 0 = (x+y) even goes first (CPM: colour 2(y&1)+(x&1), 0..3);
 *   - CPM area terms read a snapshot of the areas taken at the start of every
 *     colour pass; energies are in fixed point with a power-of-two scale S.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOTREP -5

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, written from its published definition (SC'11, Sec. 4):
 * ten rounds of two 32x32->64 multiplies; round r uses key + r * Weyl.      */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int r;
    for (r = 0; r < 10; r++) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static void seed_key(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xffffffffu);
    key[1] = (uint32_t)(seed >> 32);
}

static void draw(uint32_t a, uint32_t b, uint32_t rid, uint32_t tag, const uint32_t key[2],
                 uint32_t out[4])
{
    uint32_t ctr[4];
    ctr[0] = a;
    ctr[1] = b;
    ctr[2] = rid;
    ctr[3] = tag;
    orc_philox4x32_10(ctr, key, out);
}

/* Stream tags (fourth counter word). */
#define TAG_MAIN 0u
#define TAG_FALLBACK 1u
#define TAG_INIT 2u

static int wrap(int i, int n) { return ((i % n) + n) % n; }

/* Square-lattice Ising and Potts passes of lattices from 2^16 sites on split
 * their rows over OpenMP threads when called outside a parallel region (the
 * batch runners below are one; nested regions stay on one thread).  A pass
 * updates only sites of one colour and reads only the other colour, so the
 * split changes no bit; orc_set_num_threads(1) runs every chain on one
 * thread.                                                                   */
#define PASS_THREADS(Lx, Ly) ((int64_t)(Lx) * (Ly) >= 65536)

/* Metropolis threshold: accept iff W < T, W uniform on [0, 2^32). */
static uint64_t threshold_from_dE(double dE, double beta)
{
    if (dE <= 0.0)
        return (uint64_t)1 << 32;
    return (uint64_t)ceil(ldexp(exp(-beta * dE), 32));
}

/* ------------------------------------------------------------------------ */
/* Ising, Eq. (1).  Class of a site: own spin s, Sx = left + right,
 * Sy = up + down; idx = 9*[s>0] + 3*(Sx/2+1) + (Sy/2+1).  Flipping s changes
 * the energy by dE = 2 s (Jx Sx + Jy Sy + h).                               */
int orc_ising_table(float Jx, float Jy, float h, double beta, uint64_t T[18])
{
    int si, a, b;
    if (!(beta >= 0.0) || !isfinite(beta) || !isfinite(Jx) || !isfinite(Jy) || !isfinite(h))
        return ORC_EINVAL;
    for (si = 0; si < 2; si++)
        for (a = 0; a < 3; a++)
            for (b = 0; b < 3; b++) {
                double s = si ? 1.0 : -1.0;
                double Sx = 2.0 * a - 2.0, Sy = 2.0 * b - 2.0;
                double u = (double)Jx * Sx;
                u = u + (double)Jy * Sy;
                u = u + (double)h;
                double dE = 2.0 * s * u;
                T[9 * si + 3 * a + b] = threshold_from_dE(dE, beta);
            }
    return ORC_OK;
}

void orc_ising_init(int Lx, int Ly, uint64_t seed, uint32_t rid, int8_t *sigma)
{
    uint32_t key[2], w[4];
    int y, x;
    seed_key(seed, key);
    for (y = 0; y < Ly; y++)
        for (x = 0; x < Lx; x++) {
            uint32_t n = (uint32_t)(y * Lx + x);
            draw(n >> 2, 0u, rid, TAG_INIT, key, w);
            sigma[n] = (w[n & 3] < 0x80000000u) ? (int8_t)1 : (int8_t)-1;
        }
}

/* Integer statistics of an Ising state: M, Bx = sum s(y,x)s(y,x+1),
 * By = sum s(y,x)s(y+1,x).                                                 */
void orc_ising_stats(int Lx, int Ly, const int8_t *sg, int32_t out[8])
{
    int32_t M = 0, Bx = 0, By = 0;
    int y, x;
    for (y = 0; y < Ly; y++)
        for (x = 0; x < Lx; x++) {
            int s = sg[y * Lx + x];
            M += s;
            Bx += s * sg[y * Lx + wrap(x + 1, Lx)];
            By += s * sg[wrap(y + 1, Ly) * Lx + x];
        }
    memset(out, 0, 8 * sizeof(int32_t));
    out[0] = M;
    out[1] = Bx;
    out[2] = By;
}

static int check_shape(int Lx, int Ly)
{
    return (Lx >= 2 && Ly >= 2 && (Lx % 2) == 0 && (Ly % 2) == 0);
}

/* One Ising run of n sweeps starting at global sweep t0.  A sweep is the
 * colour-0 pass then the colour-1 pass; pass index p = 2t + c.            */
int orc_ising_run(int Lx, int Ly, float Jx, float Jy, float h, double beta, uint64_t seed,
                  uint32_t rid, uint64_t t0, int n_sweeps, int record_every, int8_t *sg,
                  int32_t *stats)
{
    uint64_t T[18];
    uint32_t key[2];
    int i, c, y, rec = 0;
    if (!check_shape(Lx, Ly) || n_sweeps < 0 || record_every < 0)
        return ORC_EINVAL;
    if (orc_ising_table(Jx, Jy, h, beta, T) != ORC_OK)
        return ORC_EINVAL;
    seed_key(seed, key);
    for (i = 0; i < n_sweeps; i++) {
        uint64_t t = t0 + (uint64_t)i;
        for (c = 0; c < 2; c++) {
            uint32_t p = (uint32_t)(2 * t + (uint64_t)c);
            /* the colour's sites are independent (see the header): rows of a
             * large lattice may run on several threads, same result */
#pragma omp parallel for schedule(static) if (PASS_THREADS(Lx, Ly))
            for (y = 0; y < Ly; y++)
                for (int x = 0; x < Lx; x++) {
                    uint32_t w[4], f[4];
                    if (((x + y) & 1) != c)
                        continue;
                    uint32_t k = (uint32_t)(y * (Lx / 2) + (x >> 1));
                    draw(k >> 3, p, rid, TAG_MAIN, key, w);
                    uint32_t hw = k & 7u;
                    uint32_t ra = (w[hw >> 1] >> (16u * (hw & 1u))) & 0xFFFFu;
                    draw(k, p, rid, TAG_FALLBACK, key, f);
                    uint64_t W = ((uint64_t)ra << 16) | (uint64_t)(f[0] & 0xFFFFu);
                    int s = sg[y * Lx + x];
                    int Sx = sg[y * Lx + wrap(x - 1, Lx)] + sg[y * Lx + wrap(x + 1, Lx)];
                    int Sy = sg[wrap(y - 1, Ly) * Lx + x] + sg[wrap(y + 1, Ly) * Lx + x];
                    int idx = 9 * (s > 0) + 3 * (Sx / 2 + 1) + (Sy / 2 + 1);
                    if (W < T[idx])
                        sg[y * Lx + x] = (int8_t)(-s);
                }
        }
        if (record_every > 0 && ((i + 1) % record_every) == 0 && stats) {
            orc_ising_stats(Lx, Ly, sg, stats + 8 * rec);
            rec++;
        }
    }
    return rec;
}

/* ------------------------------------------------------------------------ */
/* Triangular-lattice Ising (the triangular kernels of the Methods): sites on
 * an Ly x Lx array, the six neighbours (y, x-1), (y, x+1), (y-1, x),
 * (y+1, x), (y-1, x+1), (y+1, x-1) (periodic), one coupling J for every
 * bond: H = -J sum_bonds s s' - h sum s.  Three colours c = (x + 2y) mod 3
 * (no bond joins two sites of one colour; Lx and Ly multiples of 3), passes
 * p = 3t + c; within-colour index k = y Lx/3 + x/3; W = word k & 3 of the
 * main block (k >> 2, p, rid, 0) as a whole 32-bit word; accept the flip iff
 * W < T(class), class idx = 7 [s > 0] + (S6 + 6) / 2 with S6 the sum of the
 * six neighbours, dE = 2 s (J S6 + h).                                      */
int orc_tri_table(float J, float h, double beta, uint64_t T[14])
{
    int si, a;
    if (!(beta >= 0.0) || !isfinite(beta) || !isfinite(J) || !isfinite(h))
        return ORC_EINVAL;
    for (si = 0; si < 2; si++)
        for (a = 0; a < 7; a++) {
            double s = si ? 1.0 : -1.0;
            double u = (double)J * (double)(2 * a - 6);
            u = u + (double)h;
            T[7 * si + a] = threshold_from_dE(2.0 * s * u, beta);
        }
    return ORC_OK;
}

/* M, Bh = sum s(y,x)s(y,x+1), Bv = sum s(y,x)s(y+1,x), Bd = sum s(y,x)s(y+1,x-1). */
void orc_tri_stats(int Lx, int Ly, const int8_t *sg, int32_t out[8])
{
    int32_t M = 0, Bh = 0, Bv = 0, Bd = 0;
    int y, x;
    for (y = 0; y < Ly; y++)
        for (x = 0; x < Lx; x++) {
            int s = sg[y * Lx + x];
            M += s;
            Bh += s * sg[y * Lx + wrap(x + 1, Lx)];
            Bv += s * sg[wrap(y + 1, Ly) * Lx + x];
            Bd += s * sg[wrap(y + 1, Ly) * Lx + wrap(x - 1, Lx)];
        }
    memset(out, 0, 8 * sizeof(int32_t));
    out[0] = M;
    out[1] = Bh;
    out[2] = Bv;
    out[3] = Bd;
}

int orc_tri_run(int Lx, int Ly, float J, float h, double beta, uint64_t seed, uint32_t rid,
                uint64_t t0, int n_sweeps, int record_every, int8_t *sg, int32_t *stats)
{
    uint64_t T[14];
    uint32_t key[2], w[4];
    int i, c, y, x, rec = 0;
    if (Lx < 3 || Ly < 3 || Lx % 3 != 0 || Ly % 3 != 0 || n_sweeps < 0 || record_every < 0)
        return ORC_EINVAL;
    if (orc_tri_table(J, h, beta, T) != ORC_OK)
        return ORC_EINVAL;
    seed_key(seed, key);
    for (i = 0; i < n_sweeps; i++) {
        uint64_t t = t0 + (uint64_t)i;
        for (c = 0; c < 3; c++) {
            uint32_t p = (uint32_t)(3 * t + (uint64_t)c);
            for (y = 0; y < Ly; y++)
                for (x = 0; x < Lx; x++) {
                    if ((x + 2 * y) % 3 != c)
                        continue;
                    uint32_t k = (uint32_t)(y * (Lx / 3) + x / 3);
                    draw(k >> 2, p, rid, TAG_MAIN, key, w);
                    uint32_t W = w[k & 3u];
                    int s = sg[y * Lx + x];
                    int S6 = sg[y * Lx + wrap(x - 1, Lx)] + sg[y * Lx + wrap(x + 1, Lx)] +
                             sg[wrap(y - 1, Ly) * Lx + x] + sg[wrap(y + 1, Ly) * Lx + x] +
                             sg[wrap(y - 1, Ly) * Lx + wrap(x + 1, Lx)] +
                             sg[wrap(y + 1, Ly) * Lx + wrap(x - 1, Lx)];
                    int idx = 7 * (s > 0) + (S6 + 6) / 2;
                    if ((uint64_t)W < T[idx])
                        sg[y * Lx + x] = (int8_t)(-s);
                }
        }
        if (record_every > 0 && ((i + 1) % record_every) == 0 && stats) {
            orc_tri_stats(Lx, Ly, sg, stats + 8 * rec);
            rec++;
        }
    }
    return rec;
}

/* ------------------------------------------------------------------------ */
/* Ising on the chain, square and simple-cubic lattices (the 1D, 2D and 3D
 * convolutions of the Methods) in one natural layout: an Lz x Ly x Lx array,
 * n = (z Ly + y) Lx + x; a dimension of extent 1 is absent, every other
 * extent is even and >= 2; the neighbours are x +- 1 and, where present,
 * y +- 1 and z +- 1 (periodic), one coupling J for every bond.  Two colours
 * c = (x + y + z) & 1, passes p = 2t + c; the colour-c site of the pair
 * (2k, 2k + 1) is the one with within-colour index k, and takes word k & 3 of
 * the main block (k >> 2, p, rid, 0) whole as W; flip iff W < T(class),
 * class idx = 7 [s > 0] + (S + 6) / 2 with S the sum of the neighbours,
 * dE = 2 s (J S + h) -- the same 14-entry table as the triangular lattice.  */
int orc_hc_table(float J, float h, double beta, uint64_t T[14])
{
    return orc_tri_table(J, h, beta, T);
}

/* M, Bx = sum s(n)s(n+x), By = sum s(n)s(n+y), Bz = sum s(n)s(n+z) (By, Bz
 * zero for absent dimensions).                                              */
void orc_hc_stats(int Lx, int Ly, int Lz, const int8_t *sg, int32_t out[8])
{
    int32_t M = 0, Bx = 0, By = 0, Bz = 0;
    int z, y, x;
    for (z = 0; z < Lz; z++)
        for (y = 0; y < Ly; y++)
            for (x = 0; x < Lx; x++) {
                int s = sg[(z * Ly + y) * Lx + x];
                M += s;
                Bx += s * sg[(z * Ly + y) * Lx + wrap(x + 1, Lx)];
                if (Ly > 1)
                    By += s * sg[(z * Ly + wrap(y + 1, Ly)) * Lx + x];
                if (Lz > 1)
                    Bz += s * sg[(wrap(z + 1, Lz) * Ly + y) * Lx + x];
            }
    memset(out, 0, 8 * sizeof(int32_t));
    out[0] = M;
    out[1] = Bx;
    out[2] = By;
    out[3] = Bz;
}

static int hc_extent_ok(int L) { return L == 1 || (L >= 2 && L % 2 == 0); }

int orc_hc_run(int Lx, int Ly, int Lz, float J, float h, double beta, uint64_t seed, uint32_t rid,
               uint64_t t0, int n_sweeps, int record_every, int8_t *sg, int32_t *stats)
{
    uint64_t T[14];
    uint32_t key[2], w[4];
    int i, c, z, y, x, rec = 0;
    if (Lx < 2 || Lx % 2 != 0 || !hc_extent_ok(Ly) || !hc_extent_ok(Lz) || n_sweeps < 0 ||
        record_every < 0)
        return ORC_EINVAL;
    if (orc_hc_table(J, h, beta, T) != ORC_OK)
        return ORC_EINVAL;
    seed_key(seed, key);
    for (i = 0; i < n_sweeps; i++) {
        uint64_t t = t0 + (uint64_t)i;
        for (c = 0; c < 2; c++) {
            uint32_t p = (uint32_t)(2 * t + (uint64_t)c);
            for (z = 0; z < Lz; z++)
                for (y = 0; y < Ly; y++)
                    for (x = 0; x < Lx; x++) {
                        if (((x + y + z) & 1) != c)
                            continue;
                        uint32_t n = (uint32_t)((z * Ly + y) * Lx + x);
                        uint32_t k = n >> 1;
                        draw(k >> 2, p, rid, TAG_MAIN, key, w);
                        uint32_t W = w[k & 3u];
                        int s = sg[n];
                        int S = sg[(z * Ly + y) * Lx + wrap(x - 1, Lx)] +
                                sg[(z * Ly + y) * Lx + wrap(x + 1, Lx)];
                        if (Ly > 1)
                            S += sg[(z * Ly + wrap(y - 1, Ly)) * Lx + x] +
                                 sg[(z * Ly + wrap(y + 1, Ly)) * Lx + x];
                        if (Lz > 1)
                            S += sg[(wrap(z - 1, Lz) * Ly + y) * Lx + x] +
                                 sg[(wrap(z + 1, Lz) * Ly + y) * Lx + x];
                        int idx = 7 * (s > 0) + (S + 6) / 2;
                        if ((uint64_t)W < T[idx])
                            sg[n] = (int8_t)(-s);
                    }
        }
        if (record_every > 0 && ((i + 1) % record_every) == 0 && stats) {
            orc_hc_stats(Lx, Ly, Lz, sg, stats + 8 * rec);
            rec++;
        }
    }
    return rec;
}

/* ------------------------------------------------------------------------ */
/* Multispin-coded square-lattice Ising: 32 replicas with the same Lx, Ly,
 * Jx, Jy, h and beta packed bit by bit in one uint32 per site (bit b = 1 is
 * s = +1 in replica b), natural layout n = y Lx + x.  The replicas share the
 * random numbers: in pass p = 2t + c every site of colour c = (x + y) & 1
 * takes W = word k & 3 (k = n >> 1) of the main block (k >> 2, p, rid, 0)
 * whole, and every bit of it flips iff W < T[idx] with the square lattice's
 * classes idx = 9 [s > 0] + 3 (Sx/2 + 1) + (Sy/2 + 1) of that bit.  Bit b of
 * the initial word of site n is 1 iff word n & 3 of the init block
 * (n >> 2, b, rid, 2) is < 2^31.                                            */
void orc_msc_init(int Lx, int Ly, uint64_t seed, uint32_t rid, uint32_t *w32)
{
    uint32_t key[2], w[4];
    int n, b;
    seed_key(seed, key);
    for (n = 0; n < Lx * Ly; n++) {
        uint32_t v = 0;
        for (b = 0; b < 32; b++) {
            draw((uint32_t)n >> 2, (uint32_t)b, rid, TAG_INIT, key, w);
            if (w[n & 3] < 0x80000000u)
                v |= 1u << b;
        }
        w32[n] = v;
    }
}

/* Statistics of bit b: [M, Bx, By] into out + 8 b (32 rows of 8).           */
void orc_msc_stats(int Lx, int Ly, const uint32_t *w32, int32_t *out)
{
    int b, y, x;
    memset(out, 0, 32 * 8 * sizeof(int32_t));
    for (b = 0; b < 32; b++)
        for (y = 0; y < Ly; y++)
            for (x = 0; x < Lx; x++) {
                int s = (w32[y * Lx + x] >> b) & 1u ? 1 : -1;
                int r = (w32[y * Lx + wrap(x + 1, Lx)] >> b) & 1u ? 1 : -1;
                int d = (w32[wrap(y + 1, Ly) * Lx + x] >> b) & 1u ? 1 : -1;
                out[8 * b] += s;
                out[8 * b + 1] += s * r;
                out[8 * b + 2] += s * d;
            }
}

int orc_msc_run(int Lx, int Ly, float Jx, float Jy, float h, double beta, uint64_t seed,
                uint32_t rid, uint64_t t0, int n_sweeps, int record_every, uint32_t *w32,
                int32_t *stats /* [n_rec][32][8] */)
{
    uint64_t T[18];
    uint32_t key[2], w[4];
    int i, c, y, x, b, rec = 0;
    if (!check_shape(Lx, Ly) || n_sweeps < 0 || record_every < 0)
        return ORC_EINVAL;
    if (orc_ising_table(Jx, Jy, h, beta, T) != ORC_OK)
        return ORC_EINVAL;
    seed_key(seed, key);
    for (i = 0; i < n_sweeps; i++) {
        uint64_t t = t0 + (uint64_t)i;
        for (c = 0; c < 2; c++) {
            uint32_t p = (uint32_t)(2 * t + (uint64_t)c);
            for (y = 0; y < Ly; y++)
                for (x = 0; x < Lx; x++) {
                    if (((x + y) & 1) != c)
                        continue;
                    uint32_t n = (uint32_t)(y * Lx + x), k = n >> 1;
                    draw(k >> 2, p, rid, TAG_MAIN, key, w);
                    uint64_t W = w[k & 3u];
                    uint32_t v = w32[n], flip = 0;
                    for (b = 0; b < 32; b++) {
                        int s = (v >> b) & 1u ? 1 : -1;
                        int l = (w32[y * Lx + wrap(x - 1, Lx)] >> b) & 1u ? 1 : -1;
                        int r = (w32[y * Lx + wrap(x + 1, Lx)] >> b) & 1u ? 1 : -1;
                        int u = (w32[wrap(y - 1, Ly) * Lx + x] >> b) & 1u ? 1 : -1;
                        int d = (w32[wrap(y + 1, Ly) * Lx + x] >> b) & 1u ? 1 : -1;
                        int idx = 9 * (s > 0) + 3 * ((l + r) / 2 + 1) + ((u + d) / 2 + 1);
                        if (W < T[idx])
                            flip |= 1u << b;
                    }
                    w32[n] = v ^ flip;
                }
        }
        if (record_every > 0 && ((i + 1) % record_every) == 0 && stats) {
            orc_msc_stats(Lx, Ly, w32, stats + 256 * rec);
            rec++;
        }
    }
    return rec;
}

/* ------------------------------------------------------------------------ */
/* Potts, Eq. (2), H = -J sum delta - h sum s.  For a proposal s -> s':
 * dn = #{nbrs == s'} - #{nbrs == s} in [-4,4], ds = s'-s;
 * dE = -(J dn + h ds); idx = (dn+4)(2q-1) + (ds + q - 1).                   */
int orc_potts_table(int q, float J, float h, double beta, uint64_t *T)
{
    int dn, ds;
    if (q < 2 || q > 255 || !(beta >= 0.0) || !isfinite(beta) || !isfinite(J) || !isfinite(h))
        return ORC_EINVAL;
    for (dn = -4; dn <= 4; dn++)
        for (ds = -(q - 1); ds <= q - 1; ds++) {
            double u = (double)J * (double)dn;
            u = u + (double)h * (double)ds;
            double dE = -u;
            T[(dn + 4) * (2 * q - 1) + (ds + q - 1)] = threshold_from_dE(dE, beta);
        }
    return ORC_OK;
}

void orc_potts_init(int Lx, int Ly, int q, uint64_t seed, uint32_t rid, uint8_t *s)
{
    uint32_t key[2], w[4];
    int y, x;
    seed_key(seed, key);
    for (y = 0; y < Ly; y++)
        for (x = 0; x < Lx; x++) {
            uint32_t n = (uint32_t)(y * Lx + x);
            draw(n >> 2, 0u, rid, TAG_INIT, key, w);
            s[n] = (uint8_t)(((uint64_t)w[n & 3] * (uint64_t)q) >> 32);
        }
}

/* Potts statistics: Nx, Ny = equal horizontal / vertical bonds, S = sum s,
 * nmax = size of the most populated state.                                 */
void orc_potts_stats(int Lx, int Ly, int q, const uint8_t *s, int32_t out[8])
{
    int32_t Nx = 0, Ny = 0, S = 0, nmax = 0;
    int32_t *hist = (int32_t *)calloc((size_t)q, sizeof(int32_t));
    int y, x, k;
    for (y = 0; y < Ly; y++)
        for (x = 0; x < Lx; x++) {
            int v = s[y * Lx + x];
            S += v;
            hist[v]++;
            Nx += (v == s[y * Lx + wrap(x + 1, Lx)]);
            Ny += (v == s[wrap(y + 1, Ly) * Lx + x]);
        }
    for (k = 0; k < q; k++)
        if (hist[k] > nmax)
            nmax = hist[k];
    free(hist);
    memset(out, 0, 8 * sizeof(int32_t));
    out[0] = Nx;
    out[1] = Ny;
    out[2] = S;
    out[3] = nmax;
}

/* Uniform offset in [0, m) for the Potts proposal: Lemire's multiply-shift
 * with rejection on 16 bits (exactly uniform when accepted); on the rare
 * rejection a 32-bit multiply-shift of a fallback word is used instead.     */
static uint32_t potts_offset(uint32_t rp, uint32_t fbword, uint32_t m)
{
    uint32_t prod = rp * m;
    uint32_t thr = 65536u % m;
    if ((prod & 0xFFFFu) < thr)
        return (uint32_t)(((uint64_t)fbword * (uint64_t)m) >> 32);
    return prod >> 16;
}

int orc_potts_run(int Lx, int Ly, int q, float J, float h, double beta, uint64_t seed,
                  uint32_t rid, uint64_t t0, int n_sweeps, int record_every, uint8_t *sg,
                  int32_t *stats)
{
    uint64_t *T;
    uint32_t key[2];
    int i, c, y, rec = 0;
    if (!check_shape(Lx, Ly) || n_sweeps < 0 || record_every < 0 || q < 2 || q > 255)
        return ORC_EINVAL;
    T = (uint64_t *)malloc(sizeof(uint64_t) * 9 * (size_t)(2 * q - 1));
    if (orc_potts_table(q, J, h, beta, T) != ORC_OK) {
        free(T);
        return ORC_EINVAL;
    }
    seed_key(seed, key);
    for (i = 0; i < n_sweeps; i++) {
        uint64_t t = t0 + (uint64_t)i;
        for (c = 0; c < 2; c++) {
            uint32_t p = (uint32_t)(2 * t + (uint64_t)c);
#pragma omp parallel for schedule(static) if (PASS_THREADS(Lx, Ly))
            for (y = 0; y < Ly; y++)
                for (int x = 0; x < Lx; x++) {
                    uint32_t w[4], f[4];
                    if (((x + y) & 1) != c)
                        continue;
                    uint32_t k = (uint32_t)(y * (Lx / 2) + (x >> 1));
                    draw(k >> 2, p, rid, TAG_MAIN, key, w);
                    uint32_t word = w[k & 3u];
                    uint32_t rp = word & 0xFFFFu, ra = word >> 16;
                    draw(k, p, rid, TAG_FALLBACK, key, f);
                    uint64_t W = ((uint64_t)ra << 16) | (uint64_t)(f[0] & 0xFFFFu);
                    int s = sg[y * Lx + x];
                    int s2 = (int)((s + 1 + (int)potts_offset(rp, f[1], (uint32_t)(q - 1))) % q);
                    int nb[4];
                    nb[0] = sg[y * Lx + wrap(x - 1, Lx)];
                    nb[1] = sg[y * Lx + wrap(x + 1, Lx)];
                    nb[2] = sg[wrap(y - 1, Ly) * Lx + x];
                    nb[3] = sg[wrap(y + 1, Ly) * Lx + x];
                    int dn = 0, j;
                    for (j = 0; j < 4; j++)
                        dn += (nb[j] == s2) - (nb[j] == s);
                    int idx = (dn + 4) * (2 * q - 1) + (s2 - s + q - 1);
                    if (W < T[idx])
                        sg[y * Lx + x] = (uint8_t)s2;
                }
        }
        if (record_every > 0 && ((i + 1) % record_every) == 0 && stats) {
            orc_potts_stats(Lx, Ly, q, sg, stats + 8 * rec);
            rec++;
        }
    }
    free(T);
    return rec;
}

/* ------------------------------------------------------------------------ */
/* Cellular Potts, Eq. (3).                                                   */

/* Smallest power-of-two scale S = 2^s, s <= 8, that makes every adhesion
 * J*S and lambda*S an integer of magnitude below 2^20.                      */
int orc_cpm_scale(int n_types, const float *J, float lambda, int32_t *S_out)
{
    int s, i;
    for (s = 0; s <= 8; s++) {
        double S = ldexp(1.0, s);
        int ok = 1;
        for (i = 0; i < n_types * n_types && ok; i++) {
            double v = (double)J[i] * S;
            if (!(fabs(v) < 1048576.0) || v != floor(v))
                ok = 0;
        }
        double l = (double)lambda * S;
        if (!(fabs(l) < 1048576.0) || l != floor(l))
            ok = 0;
        if (ok) {
            *S_out = (int32_t)S;
            return ORC_OK;
        }
    }
    return ORC_ENOTREP;
}

/* Threshold of a fixed-point energy change k >= 1. */
static uint64_t cpm_threshold(int64_t k, int32_t S, double temperature)
{
    return (uint64_t)ceil(ldexp(exp(-(double)k / ((double)S * temperature)), 32));
}

static int cpm_check(int Lx, int Ly, int n_cells, int n_types, const float *J,
                     const int8_t *type, float lambda, double temperature)
{
    int i, a, b;
    if (!check_shape(Lx, Ly) || n_cells < 1 || n_types < 1 || n_types > 4)
        return ORC_EINVAL;
    if (!(temperature > 0.0) || !isfinite(temperature) || !(lambda >= 0.0f))
        return ORC_EINVAL;
    if (type[0] != 0)
        return ORC_EINVAL;
    for (i = 0; i <= n_cells; i++)
        if (type[i] < 0 || type[i] >= n_types)
            return ORC_EINVAL;
    for (a = 0; a < n_types; a++)
        for (b = 0; b < n_types; b++)
            if (J[a * n_types + b] != J[b * n_types + a])
                return ORC_EINVAL;
    return ORC_OK;
}

/* Neighbourhood of range r (Chebyshev distance <= r, the Moore
 * neighbourhood for r = 1 and its second shell added for r = 2): the offsets
 * in row-major order of (dy, dx) without (0, 0); n = (2r+1)^2 - 1.          */
static int cpm_neighbours(int range, int *dy, int *dx)
{
    int n = 0, i, j;
    for (i = -range; i <= range; i++)
        for (j = -range; j <= range; j++)
            if (i != 0 || j != 0) {
                dy[n] = i;
                dx[n] = j;
                n++;
            }
    return n;
}

/* CPM statistics: von Neumann boundary bonds between different ids, by
 * unordered type pair (a<=b, index a*n_types - a(a-1)/2 + (b-a)), into
 * out[0..9]; fixed-point energy H*S as int64 into out[10] (lo), out[11] (hi).
 * Adhesion pairs within the neighbourhood of range 1 or 2 are counted once
 * each (the offsets that come later in row-major order).                     */
void orc_cpm_stats_r(int Lx, int Ly, int n_cells, int n_types, const float *J,
                     const int8_t *type, const int32_t *A, float lambda, const int32_t *ids,
                     int range, int32_t out[16])
{
    int32_t S = 1;
    int y, x, d, a, nn;
    int64_t H = 0;
    int32_t *area;
    int NDY[24], NDX[24];
    static const int FDY[2] = {0, 1};
    static const int FDX[2] = {1, 0};
    memset(out, 0, 16 * sizeof(int32_t));
    nn = cpm_neighbours(range, NDY, NDX);
    if (orc_cpm_scale(n_types, J, lambda, &S) != ORC_OK)
        return;
    area = (int32_t *)calloc((size_t)n_cells + 1, sizeof(int32_t));
    for (y = 0; y < Ly; y++)
        for (x = 0; x < Lx; x++) {
            int s = ids[y * Lx + x];
            area[s]++;
            for (d = 0; d < 2; d++) {
                int t = ids[wrap(y + FDY[d], Ly) * Lx + wrap(x + FDX[d], Lx)];
                if (t != s) {
                    int ta = type[s], tb = type[t];
                    if (ta > tb) {
                        int tmp = ta;
                        ta = tb;
                        tb = tmp;
                    }
                    out[ta * n_types - ta * (ta - 1) / 2 + (tb - ta)]++;
                }
            }
            for (d = nn / 2; d < nn; d++) {  /* the forward half of the offsets */
                int t = ids[wrap(y + NDY[d], Ly) * Lx + wrap(x + NDX[d], Lx)];
                if (t != s)
                    H += (int64_t)llround((double)J[type[s] * n_types + type[t]] * S);
            }
        }
    for (a = 1; a <= n_cells; a++) {
        int64_t dA = (int64_t)area[a] - (int64_t)A[a];
        H += (int64_t)llround((double)lambda * S) * dA * dA;
    }
    free(area);
    out[10] = (int32_t)(uint32_t)((uint64_t)H & 0xffffffffu);
    out[11] = (int32_t)(uint32_t)((uint64_t)H >> 32);
}

void orc_cpm_stats(int Lx, int Ly, int n_cells, int n_types, const float *J,
                   const int8_t *type, const int32_t *A, float lambda, const int32_t *ids,
                   int32_t out[16])
{
    orc_cpm_stats_r(Lx, Ly, n_cells, n_types, J, type, A, lambda, ids, 1, out);
}

/* One CPM run of n Monte Carlo steps from global step t0.  Range 1: the
 * 2x2 sublattice, 4 colour passes c = 2 (y & 1) + (x & 1), p = 4t + c,
 * within-colour index k = (y >> 1) Lx/2 + (x >> 1), neighbour = bits 0..2 of
 * the main word.  Range 2 (5x5 neighbourhood, Lx and Ly multiples of 6): the
 * 3x3 sublattice, 9 passes c = 3 (y % 3) + x % 3, p = 9t + c, k = (y / 3)
 * Lx/3 + x / 3, neighbour j of 24 by the multiply-shift j = (u 24) >> 16 of
 * the low 16 bits u, rejected when (u 24) mod 2^16 < 2^16 mod 24 = 16, in
 * which case j = (f1 24) >> 32 with f1 word 1 of the fallback block.
 * ids: Ly*Lx cell ids; area: [n_cells+1] in/out, recomputed from ids.      */
int orc_cpm_run_r(int Lx, int Ly, int n_cells, int n_types, const float *J, const int8_t *type,
                  const int32_t *A, float lambda, double temperature, uint64_t seed, uint32_t rid,
                  uint64_t t0, int n_mcs, int record_every, int range, int32_t *ids,
                  int32_t *area, int32_t *stats)
{
    int32_t S;
    int64_t *JS, LS;
    int32_t *snap;
    uint32_t key[2], w[4], f[4];
    int i, c, y, x, j, rec = 0, nn, nc;
    int NDY[24], NDX[24];
    if (range != 1 && range != 2)
        return ORC_EINVAL;
    if (range == 2 && (Lx % 6 != 0 || Ly % 6 != 0))
        return ORC_EINVAL;
    if (cpm_check(Lx, Ly, n_cells, n_types, J, type, lambda, temperature) != ORC_OK)
        return ORC_EINVAL;
    nn = cpm_neighbours(range, NDY, NDX);
    nc = range == 1 ? 4 : 9;
    if (n_mcs < 0 || record_every < 0)
        return ORC_EINVAL;
    for (i = 0; i < Lx * Ly; i++)
        if (ids[i] < 0 || ids[i] > n_cells)
            return ORC_EINVAL;
    if (orc_cpm_scale(n_types, J, lambda, &S) != ORC_OK)
        return ORC_ENOTREP;
    JS = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_types * n_types));
    for (i = 0; i < n_types * n_types; i++)
        JS[i] = (int64_t)llround((double)J[i] * S);
    LS = (int64_t)llround((double)lambda * S);
    memset(area, 0, sizeof(int32_t) * ((size_t)n_cells + 1));
    for (i = 0; i < Lx * Ly; i++)
        area[ids[i]]++;
    snap = (int32_t *)malloc(sizeof(int32_t) * ((size_t)n_cells + 1));
    seed_key(seed, key);
    for (i = 0; i < n_mcs; i++) {
        uint64_t t = t0 + (uint64_t)i;
        for (c = 0; c < nc; c++) {
            uint32_t p = (uint32_t)((uint64_t)nc * t + (uint64_t)c);
            memcpy(snap, area, sizeof(int32_t) * ((size_t)n_cells + 1));
            for (y = 0; y < Ly; y++)
                for (x = 0; x < Lx; x++) {
                    int col = range == 1 ? 2 * (y & 1) + (x & 1) : 3 * (y % 3) + x % 3;
                    if (col != c)
                        continue;
                    uint32_t k = range == 1 ? (uint32_t)((y >> 1) * (Lx / 2) + (x >> 1))
                                            : (uint32_t)((y / 3) * (Lx / 3) + x / 3);
                    draw(k >> 2, p, rid, TAG_MAIN, key, w);
                    uint32_t word = w[k & 3u];
                    int jn;
                    int have_f = 0;
                    if (range == 1) {
                        jn = (int)(word & 7u);
                    } else {
                        uint32_t l = (word & 0xFFFFu) * 24u;
                        jn = (int)(l >> 16);
                        if ((l & 0xFFFFu) < 16u) {
                            draw(k, p, rid, TAG_FALLBACK, key, f);
                            have_f = 1;
                            jn = (int)(((uint64_t)f[1] * 24u) >> 32);
                        }
                    }
                    uint32_t ra = word >> 16;
                    int s = ids[y * Lx + x];
                    int tgt = ids[wrap(y + NDY[jn], Ly) * Lx + wrap(x + NDX[jn], Lx)];
                    if (tgt == s)
                        continue;
                    if (!have_f)
                        draw(k, p, rid, TAG_FALLBACK, key, f);
                    uint64_t W = ((uint64_t)ra << 16) | (uint64_t)(f[0] & 0xFFFFu);
                    int64_t kk = 0;
                    for (j = 0; j < nn; j++) {
                        int m = ids[wrap(y + NDY[j], Ly) * Lx + wrap(x + NDX[j], Lx)];
                        if (tgt != m)
                            kk += JS[type[tgt] * n_types + type[m]];
                        if (s != m)
                            kk -= JS[type[s] * n_types + type[m]];
                    }
                    int64_t karea = 0;
                    if (tgt != 0)
                        karea += 2 * ((int64_t)snap[tgt] - (int64_t)A[tgt]) + 1;
                    if (s != 0)
                        karea += -2 * ((int64_t)snap[s] - (int64_t)A[s]) + 1;
                    kk += LS * karea;
                    int accept = (kk <= 0) || (W < cpm_threshold(kk, S, temperature));
                    if (accept) {
                        ids[y * Lx + x] = tgt;
                        area[tgt]++;
                        area[s]--;
                    }
                }
        }
        if (record_every > 0 && ((i + 1) % record_every) == 0 && stats) {
            orc_cpm_stats_r(Lx, Ly, n_cells, n_types, J, type, A, lambda, ids, range,
                            stats + 16 * rec);
            rec++;
        }
    }
    free(JS);
    free(snap);
    return rec;
}

int orc_cpm_run(int Lx, int Ly, int n_cells, int n_types, const float *J, const int8_t *type,
                const int32_t *A, float lambda, double temperature, uint64_t seed, uint32_t rid,
                uint64_t t0, int n_mcs, int record_every, int32_t *ids, int32_t *area,
                int32_t *stats)
{
    return orc_cpm_run_r(Lx, Ly, n_cells, n_types, J, type, A, lambda, temperature, seed, rid,
                         t0, n_mcs, record_every, 1, ids, area, stats);
}

/* ------------------------------------------------------------------------ */
/* Batches of independent chains (one replica per iteration, OpenMP over
 * replicas).  Lattices are concatenated; offsets are in elements.          */
int orc_ising_run_batch(int R, const int32_t *Lx, const int32_t *Ly, const float *Jx,
                        const float *Jy, const float *h, const double *beta, uint64_t seed,
                        const uint32_t *rid, uint64_t t0, int n_sweeps, int record_every,
                        int8_t *sg, const int64_t *off, int32_t *stats /* [R][n_rec][8] */)
{
    int r, bad = 0;
    int n_rec = record_every > 0 ? n_sweeps / record_every : 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (r = 0; r < R; r++) {
        int rc = orc_ising_run(Lx[r], Ly[r], Jx[r], Jy[r], h[r], beta[r], seed, rid[r], t0,
                               n_sweeps, record_every, sg + off[r],
                               stats ? stats + (size_t)r * n_rec * 8 : NULL);
        if (rc < 0)
            bad++;
    }
    return bad ? ORC_EINVAL : n_rec;
}

int orc_potts_run_batch(int R, const int32_t *Lx, const int32_t *Ly, const int32_t *q,
                        const float *J, const float *h, const double *beta, uint64_t seed,
                        const uint32_t *rid, uint64_t t0, int n_sweeps, int record_every,
                        uint8_t *sg, const int64_t *off, int32_t *stats)
{
    int r, bad = 0;
    int n_rec = record_every > 0 ? n_sweeps / record_every : 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (r = 0; r < R; r++) {
        int rc = orc_potts_run(Lx[r], Ly[r], q[r], J[r], h[r], beta[r], seed, rid[r], t0,
                               n_sweeps, record_every, sg + off[r],
                               stats ? stats + (size_t)r * n_rec * 8 : NULL);
        if (rc < 0)
            bad++;
    }
    return bad ? ORC_EINVAL : n_rec;
}

/* Philox outputs on a grid of counters: out[r][b][0..3] = Philox4x32-10 of
 * counter (b, c1, rids[r], c3) under key (k0, k1), b = 0..n_blocks-1.       */
void orc_philox_grid(int n_blocks, uint32_t c1, const uint32_t *rids, int n_rid, uint32_t c3,
                     uint32_t k0, uint32_t k1, uint32_t *out)
{
    int r, b;
    const uint32_t key[2] = {k0, k1};
    for (r = 0; r < n_rid; r++)
        for (b = 0; b < n_blocks; b++) {
            const uint32_t ctr[4] = {(uint32_t)b, c1, rids[r], c3};
            orc_philox4x32_10(ctr, key, out + ((size_t)r * n_blocks + b) * 4);
        }
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

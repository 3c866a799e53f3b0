// Shared definitions for the libqfs HIP kernels (gfx950).
//
// Monomial index: a homogeneous form of degree n in x1..x4 is a byte array in
// descending lexicographic order of (e1,e2,e3,e4).  The position of e is
//     rank(e) = C(e2+e3+e4+2, 3) + C(e3+e4+1, 2) + e4,
// which does not depend on n (it counts the tuples that precede e: those with
// a larger e1, then a larger e2, then a larger e3).
//
// Dehomogenised coordinates drop x4 (the homogeneous form is determined by
// its restriction x4 = 1 -- Section 5.1 of the paper uses the same fact for
// its Kronecker substitution), so a form of degree n lives on the simplex
// {x in Z^3 : x >= 0, x1+x2+x3 <= n}.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qfs {

__host__ __device__ constexpr int64_t num_mono(int deg)
{
    return deg < 0 ? 0 : (int64_t)(deg + 3) * (deg + 2) * (deg + 1) / 6;
}

// Ranks and degrees here stay far below the 32-bit limits ((m+2)(m+1)m < 2^32
// for m <= 1600; the largest degree used is 4p(p-1) = 440), so the arithmetic
// is done in 32 bits.
__host__ __device__ inline unsigned tet3(unsigned m) { return (m + 2) * (m + 1) * m / 6u; }  // C(m+2,3)
__host__ __device__ inline unsigned tri2(unsigned m) { return (m + 1) * m / 2u; }            // C(m+1,2)

__host__ __device__ inline int64_t cns_rank(int e2, int e3, int e4)
{
    const unsigned m1 = (unsigned)(e2 + e3 + e4), m2 = (unsigned)(e3 + e4);
    return (int64_t)(tet3(m1) + tri2(m2) + (unsigned)e4);
}

// Inverse of cns_rank for degree n: exponents (e1,e2,e3,e4) of position r.
__host__ __device__ inline void cns_unrank(int n, int64_t r64, int &e1, int &e2, int &e3, int &e4)
{
    const unsigned r = (unsigned)r64;
    // m1 = e2+e3+e4 is the largest m with C(m+2,3) <= r
    int m1 = (int)cbrtf((float)(6.0f * (float)r + 1.0f));
    if (m1 > n) m1 = n;
    while (m1 > 0 && tet3((unsigned)m1) > r) --m1;
    while (m1 < n && tet3((unsigned)m1 + 1u) <= r) ++m1;
    const unsigned r1 = r - tet3((unsigned)m1);
    // m2 = e3+e4 is the largest m <= m1 with C(m+1,2) <= r1
    int m2 = (int)sqrtf((float)(2u * r1 + 1u));
    if (m2 > m1) m2 = m1;
    while (m2 > 0 && tri2((unsigned)m2) > r1) --m2;
    while (m2 < m1 && tri2((unsigned)m2 + 1u) <= r1) ++m2;
    e4 = (int)(r1 - tri2((unsigned)m2));
    e3 = m2 - e4;
    e2 = m1 - m2;
    e1 = n - m1;
}

// The 35 exponent tuples of degree 4 in coefficient order, packed 8 bits each (e1..e4).
struct B4Table {
    uint32_t e[35];
};
__host__ __device__ constexpr B4Table make_b4()
{
    B4Table t{};
    int i = 0;
    for (int e1 = 4; e1 >= 0; --e1)
        for (int e2 = 4 - e1; e2 >= 0; --e2)
            for (int e3 = 4 - e1 - e2; e3 >= 0; --e3) {
                int e4 = 4 - e1 - e2 - e3;
                t.e[i++] = (uint32_t)e1 | ((uint32_t)e2 << 8) | ((uint32_t)e3 << 16) | ((uint32_t)e4 << 24);
            }
    return t;
}

// ---------------------------------------------------------------------------
// Per-prime sizes.
// ---------------------------------------------------------------------------
template <int P>
struct Prime {
    static constexpr int p = P;
    static constexpr int p2 = P * P;
    static constexpr int d = 4 * (P - 1);      // degree of g = f^(p-1)
    static constexpr int D = P * d;            // degree of Delta_1(g)
    static constexpr int len_g = (int)num_mono(d);
    static constexpr int64_t len_D = num_mono(D);
    // index of the monomial (x1 x2 x3 x4)^(p-1) in B_d
    static constexpr int e_index = (int)((3 * (P - 1) + 2) * (3 * (P - 1) + 1) * (int64_t)(3 * (P - 1)) / 6 +
                                         (2 * (P - 1) + 1) * (int64_t)(2 * (P - 1)) / 2 + (P - 1));
};

// Monomials of degree 4j (j = 1..P-1) whose four exponents are all <= P-1,
// packed 8 bits per exponent, grouped by degree.  The coefficient of
// (x1 x2 x3 x4)^(P-1) in f^(P-1) (Fedder's test) depends only on these
// coefficients of the powers f^j: a term f[t] f^j[m - t] with m <= P-1 in
// every exponent has m - t <= P-1 as well.
template <int P>
struct CapTable {
    static constexpr int count(int n)
    {
        int c = 0;
        for (int x1 = 0; x1 < P; ++x1)
            for (int x2 = 0; x2 < P; ++x2)
                for (int x3 = 0; x3 < P; ++x3) {
                    const int x4 = n - x1 - x2 - x3;
                    if (x4 >= 0 && x4 < P) ++c;
                }
        return c;
    }
    static constexpr int total()
    {
        int t = 0;
        for (int j = 1; j < P; ++j) t += count(4 * j);
        return t;
    }
    static constexpr int N = total();
    uint32_t m[N];
    int off[P], len[P];  // degree 4j: entries off[j] .. off[j] + len[j] - 1
};
template <int P>
constexpr CapTable<P> make_cap_table()
{
    CapTable<P> t{};
    int n = 0;
    for (int j = 1; j < P; ++j) {
        t.off[j] = n;
        for (int x1 = 0; x1 < P; ++x1)
            for (int x2 = 0; x2 < P; ++x2)
                for (int x3 = 0; x3 < P; ++x3) {
                    const int x4 = 4 * j - x1 - x2 - x3;
                    if (x4 >= 0 && x4 < P)
                        t.m[n++] = (uint32_t)x1 | ((uint32_t)x2 << 8) | ((uint32_t)x3 << 16) | ((uint32_t)x4 << 24);
                }
        t.len[j] = n - t.off[j];
    }
    return t;
}

// ---------------------------------------------------------------------------
// The deep chain.  Delta_1 needs g~^p mod p^2 (Algorithm 1).  Since
// g~ = f~^(p-1) + p h for some integral h, (g~ + p h)^p = g~^p mod p^2, so
// g~^p = f~^(p(p-1)) = m^NF mod p^2 for the multiplier m = f~^J mod p^2 with
// any J dividing p(p-1), NF = p(p-1)/J.  The chain A_1 = m,
// A_{k+1} = A_k * m (k = 1..NF-1) trades fewer, larger products (J = p-1,
// where m = g~ is used directly) against more, smaller ones (J = 1, m = f~).
// The values of J per prime are chosen by measurement.
// ---------------------------------------------------------------------------
#ifndef QFS_CHAIN_J3
#define QFS_CHAIN_J3 2
#endif
#ifndef QFS_CHAIN_J5
#define QFS_CHAIN_J5 2
#endif
#ifndef QFS_CHAIN_J7
#define QFS_CHAIN_J7 3
#endif
#ifndef QFS_CHAIN_J11
#define QFS_CHAIN_J11 2
#endif
template <int P>
constexpr int chain_j()
{
    return P == 3 ? QFS_CHAIN_J3 : P == 5 ? QFS_CHAIN_J5 : P == 7 ? QFS_CHAIN_J7 : QFS_CHAIN_J11;
}
// When J < p-1 divides p-1, A_{(p-1)/J} = f~^(p-1) mod p^2 is a link of the
// chain and g = f^(p-1) mod p is read off it (every coefficient of degree
// 4(p-1) <= p^2-1 is formed, also in the capped chain); otherwise g is
// computed beforehand.
template <int P>
constexpr bool g_from_chain()
{
    return chain_j<P>() < P - 1 && (P - 1) % chain_j<P>() == 0;
}

// ---------------------------------------------------------------------------
// Block-Toeplitz geometry for the matrix-core product C = A * m (m of degree
// dm = 4J).
//
// Dehomogenised positions are cut into tiles of T = (2,2,4) positions (16
// bytes, position s = s1*8 + s2*4 + s3 inside the tile).  With output tile q
// and input tile q - delta, the product restricted to one pair of tiles is a
// 16x16 matrix W_delta[s][s'] = m[T*delta + s - s'] applied to the 16 input
// bytes.  V is the set of offsets delta whose block can be nonzero for a
// form of degree dm: some T*delta + s - s' lies in {x >= 0, x1+x2+x3 <= dm}.
// ---------------------------------------------------------------------------
constexpr int T1 = 2, T2 = 2, T3 = 4, TILE = 16;

template <int P>
struct Geo {
    static constexpr int J = chain_j<P>();
    static_assert(J >= 1 && J <= P - 1 && (P * (P - 1)) % J == 0, "J must divide p(p-1)");
    static constexpr int dm = 4 * J;                // degree of the multiplier m
    static constexpr int NF = P * (P - 1) / J;      // factors of the chain
    static constexpr int D = 4 * P * (P - 1);       // degree of g~^p
    static constexpr bool valid(int a, int b, int c)
    {
        int s = 0;
        if (a >= 1) s += T1 * (a - 1) + 1;
        if (b >= 1) s += T2 * (b - 1) + 1;
        if (c >= 1) s += T3 * (c - 1) + 1;
        return s <= dm;
    }
    static constexpr int H1 = (dm - 1) / T1 + 1;   // largest delta coordinates
    static constexpr int H2 = (dm - 1) / T2 + 1;
    static constexpr int H3 = (dm - 1) / T3 + 1;
    static constexpr int count()
    {
        int n = 0;
        for (int a = 0; a <= H1; ++a)
            for (int b = 0; b <= H2; ++b)
                for (int c = 0; c <= H3; ++c)
                    if (valid(a, b, c)) ++n;
        return n;
    }
    static constexpr int NV = count();             // |V|
    static constexpr int NQ = (NV + 3) / 4;        // quads of 4 offsets per MFMA K=64
    static constexpr int NVP = NQ * 4;
    // coarse tile box for degree D, with a halo of H below zero in each axis
    static constexpr int C1 = D / T1 + 1, C2 = D / T2 + 1, C3 = D / T3 + 1;
    static constexpr int B1 = H1 + C1, B2 = H2 + C2, B3 = H3 + C3;
    static constexpr int64_t BOX_TILES = (int64_t)B1 * B2 * B3;
    static constexpr int64_t BOX_BYTES = BOX_TILES * TILE;
    static constexpr int64_t W_BYTES = (int64_t)NVP * 256;
};

// Tile coordinates (or offsets) packed as three 10-bit fields.
__host__ __device__ constexpr uint32_t pack3(int a, int b, int c)
{
    return (uint32_t)a | ((uint32_t)b << 10) | ((uint32_t)c << 20);
}
__host__ __device__ constexpr int unp0(uint32_t v) { return (int)(v & 1023u); }
__host__ __device__ constexpr int unp1(uint32_t v) { return (int)((v >> 10) & 1023u); }
__host__ __device__ constexpr int unp2(uint32_t v) { return (int)((v >> 20) & 1023u); }

// ---------------------------------------------------------------------------
// Super-tile form of the product used by the deep kernel.  Output tiles are
// grouped in 2x2 super-tiles in (c1, c2): a base tile q (c1, c2 even) and its
// shifts q + Delta_s, Delta in {0, e1, e2, e1+e2}.  For an input tile q - delta
// the four outputs q + Delta_s use the blocks W_{delta + Delta_s}, so one
// loaded input fragment feeds four matrix-core products.  The offsets delta
// run over VX = union over s of (V - Delta_s) (components >= -1 in c1, c2).
// ---------------------------------------------------------------------------
template <int P>
struct GeoX {
    using G = Geo<P>;
    static constexpr int dm = G::dm, D = G::D, NV = G::NV, NF = G::NF;
    static constexpr int H1 = G::H1, H2 = G::H2, H3 = G::H3;
    static constexpr bool inV(int a, int b, int c)
    {
        return a >= 0 && b >= 0 && c >= 0 && a <= H1 && b <= H2 && c <= H3 && G::valid(a, b, c);
    }
    static constexpr bool inVX(int a, int b, int c)
    {
        return inV(a, b, c) || inV(a + 1, b, c) || inV(a, b + 1, c) || inV(a + 1, b + 1, c);
    }
    static constexpr int count()
    {
        int n = 0;
        for (int a = -1; a <= H1; ++a)
            for (int b = -1; b <= H2; ++b)
                for (int c = 0; c <= H3; ++c)
                    if (inVX(a, b, c)) ++n;
        return n;
    }
    static constexpr int NVX = count();
    static constexpr int NQX = (NVX + 3) / 4;
    static constexpr int NVXP = NQX * 4;
    // coarse box: c in [-H, C] in c1, c2 and [-H3, C3) in c3
    static constexpr int C1 = D / T1 + 1, C2 = D / T2 + 1, C3 = D / T3 + 1;
    static constexpr int B1 = H1 + C1 + 1, B2 = H2 + C2 + 1, B3 = H3 + C3;
    static constexpr int64_t BOX_TILES = (int64_t)B1 * B2 * B3;
    static constexpr int64_t BOX_BYTES = BOX_TILES * TILE;
    static constexpr int64_t W_BYTES = (int64_t)(NV + 1) * 256;  // block NV is all zero
};

template <int P>
struct DeltaTableX {
    uint32_t vpacked[Geo<P>::NV];         // V, for building W
    uint32_t packed[GeoX<P>::NVXP];       // VX with +1 on c1, c2 (pack3(d1+1, d2+1, d3))
    int32_t toff[GeoX<P>::NVXP];          // tile-index offset of delta in the box
    uint32_t widx[GeoX<P>::NVXP][2];      // W block of delta + Delta_s, 16 bits per shift (NV = zero block)
    uint32_t qmin[GeoX<P>::NQX];          // per quad: min (offset packed), max, largest and smallest weight
    uint32_t qmax[GeoX<P>::NQX];
    int32_t qwmax[GeoX<P>::NQX];
    int32_t qwmin[GeoX<P>::NQX];
    uint32_t wnz[GeoX<P>::NQX];           // bit s: some block of the quad for shift s is nonzero
};

template <int P>
constexpr DeltaTableX<P> make_delta_table_x()
{
    using X = GeoX<P>;
    DeltaTableX<P> t{};
    int nv = 0;
    int vid[X::H1 + 2][X::H2 + 2][X::H3 + 1] = {};
    for (int a = 0; a <= X::H1; ++a)
        for (int b = 0; b <= X::H2; ++b)
            for (int c = 0; c <= X::H3; ++c) {
                vid[a][b][c] = -1;
                if (X::inV(a, b, c)) {
                    t.vpacked[nv] = pack3(a, b, c);
                    vid[a][b][c] = nv++;
                }
            }
    int n = 0;
    const int sh[4][2] = {{0, 0}, {1, 0}, {0, 1}, {1, 1}};
    for (int a = -1; a <= X::H1; ++a)
        for (int b = -1; b <= X::H2; ++b)
            for (int c = 0; c <= X::H3; ++c) {
                if (!X::inVX(a, b, c)) continue;
                t.packed[n] = pack3(a + 1, b + 1, c);
                t.toff[n] = (a * X::B2 + b) * X::B3 + c;
                uint32_t w[4];
                for (int s = 0; s < 4; ++s) {
                    const int aa = a + sh[s][0], bb = b + sh[s][1];
                    w[s] = X::inV(aa, bb, c) ? (uint32_t)vid[aa][bb][c] : (uint32_t)X::NV;
                }
                t.widx[n][0] = w[0] | (w[1] << 16);
                t.widx[n][1] = w[2] | (w[3] << 16);
                ++n;
            }
    for (; n < X::NVXP; ++n) {
        t.packed[n] = pack3(1, 1, 0);
        t.toff[n] = 0;
        t.widx[n][0] = (uint32_t)X::NV | ((uint32_t)X::NV << 16);
        t.widx[n][1] = t.widx[n][0];
    }
    for (int q = 0; q < X::NQX; ++q) {
        int lo[3] = {1 << 20, 1 << 20, 1 << 20}, hi[3] = {-(1 << 20), -(1 << 20), -(1 << 20)}, wmax = -(1 << 20),
            wmin = 1 << 20;
        uint32_t nz = 0;
        for (int i = 0; i < 4; ++i) {
            const uint32_t v = t.packed[4 * q + i];
            const int x[3] = {unp0(v) - 1, unp1(v) - 1, unp2(v)};
            for (int j = 0; j < 3; ++j) {
                if (x[j] < lo[j]) lo[j] = x[j];
                if (x[j] > hi[j]) hi[j] = x[j];
            }
            const int w = T1 * x[0] + T2 * x[1] + T3 * x[2];
            if (w > wmax) wmax = w;
            if (w < wmin) wmin = w;
            for (int s = 0; s < 4; ++s) {
                const uint32_t wi = (t.widx[4 * q + i][s >> 1] >> (16 * (s & 1))) & 0xFFFFu;
                if (wi != (uint32_t)X::NV) nz |= 1u << s;
            }
        }
        t.qmin[q] = pack3(lo[0] + 1, lo[1] + 1, lo[2]);
        t.qmax[q] = pack3(hi[0] + 1, hi[1] + 1, hi[2]);
        t.qwmax[q] = wmax;
        t.qwmin[q] = wmin;
        t.wnz[q] = nz;
    }
    return t;
}

// Number of output tiles with w(c) = 2 c1 + 2 c2 + 4 c3 <= n, c >= 0.
__host__ __device__ constexpr int64_t tiles_upto(int n)
{
    if (n < 0) return 0;
    int64_t cnt = 0;
    for (int a = 0; T1 * a <= n; ++a)
        for (int b = 0; T1 * a + T2 * b <= n; ++b)
            cnt += (n - T1 * a - T2 * b) / T3 + 1;
    return cnt;
}

}  // namespace qfs

namespace qfs {

// ---------------------------------------------------------------------------
// Cartier-split layout of Delta for the map theta(a)[r] = sum_c Delta[p r + e - c] a[c]
// (e = (p-1,...,p-1)).  Writing c = p c' + s with s = c mod p gives
// p r + e - c = p (r - c') + (e - s): the Delta coefficient sits in residue
// class sigma = e - s at "coarse" position y = r - c'.  Only pairs whose
// exponents add to e mod p survive u (Section 4, Corollary "unique match"),
// and for c of degree d = 4(p-1) the coarse part c' has degree j <= d/p < 4.
//
// Delta is stored per j (the degree of c'): region j is a row-major matrix
// with one row per y in B_{d-j} (CNS order) and one column per s in S_j =
// {s in [0,p)^4 : |s| = d - p j} (lexicographic s, row stride padded to 16).
// theta then reads, for each output r and each c' <= r, one contiguous row.
// ---------------------------------------------------------------------------
template <int P>
struct ThetaGeo {
    static constexpr int d = 4 * (P - 1);
    static constexpr int D = P * d;
    static constexpr int J = d / P + 1;  // j = 0..J-1
    static constexpr int ns(int j)
    {
        int n = 0, target = d - P * j;
        for (int a = 0; a < P; ++a)
            for (int b = 0; b < P; ++b)
                for (int c = 0; c < P; ++c) {
                    int e = target - a - b - c;
                    if (e >= 0 && e < P) ++n;
                }
        return n;
    }
    static constexpr int rs(int j) { return (ns(j) + 15) / 16 * 16; }
    static constexpr int64_t region_off(int j)
    {
        int64_t o = 0;
        for (int i = 0; i < j; ++i) o += num_mono(d - i) * rs(i);
        return o;
    }
    static constexpr int64_t BYTES = region_off(J);
    static constexpr int count_cp()
    {
        int n = 0;
        for (int j = 0; j < J; ++j) n += (int)num_mono(j);
        return n;
    }
    static constexpr int count_aperm()
    {
        int n = 0;
        for (int j = 0; j < J; ++j) n += (int)num_mono(j) * rs(j);
        return n;
    }
    static constexpr int NCP = count_cp();       // number of coarse parts c' (35 when J = 4)
    static constexpr int APERM = count_aperm();  // bytes of the permuted input vector
    static constexpr int NSIG = P * P * P * P;
    // first column of region j in the column table, first c' of degree j
    static constexpr int col_off(int j)
    {
        int o = 0;
        for (int i = 0; i < j; ++i) o += rs(i);
        return o;
    }
    static constexpr int NCOL = col_off(J);
    static constexpr int cp_off(int j)
    {
        int o = 0;
        for (int i = 0; i < j; ++i) o += (int)num_mono(i);
        return o;
    }
};

template <int P>
struct ThetaTable {
    int16_t sidx[ThetaGeo<P>::NSIG];        // sigma code -> column in its region, -1 if |sigma| != 0 mod p
    uint16_t aperm_src[ThetaGeo<P>::APERM]; // a_perm slot -> position in B_d, 0xFFFF = padding
    uint32_t cprime[ThetaGeo<P>::NCP];      // c' exponents packed 8 bits each
    int32_t cp_seg[ThetaGeo<P>::NCP];       // start of c''s segment in a_perm
    int32_t cp_j[ThetaGeo<P>::NCP];
    int32_t rs[4];
    int64_t roff[4];
    alignas(16) uint16_t sig[ThetaGeo<P>::NCOL]; // column of a region -> sigma, 4 bits per exponent; 0xFFFF = padding
};

template <int P>
constexpr ThetaTable<P> make_theta_table()
{
    using TG = ThetaGeo<P>;
    ThetaTable<P> t{};
    constexpr int d = TG::d;
    for (int i = 0; i < TG::NSIG; ++i) t.sidx[i] = -1;
    for (int j = 0; j < 4; ++j) {
        t.rs[j] = j < TG::J ? TG::rs(j) : 0;
        t.roff[j] = j < TG::J ? TG::region_off(j) : TG::BYTES;
    }
    int seg = 0, ncp = 0;
    for (int j = 0; j < TG::J; ++j) {
        // S_j in lexicographic order; sidx of sigma = e - s
        int s_list_n = 0;
        int target = d - P * j;
        for (int a = 0; a < P; ++a)
            for (int b = 0; b < P; ++b)
                for (int c = 0; c < P; ++c) {
                    int e = target - a - b - c;
                    if (e < 0 || e >= P) continue;
                    int sg = (((P - 1 - a) * P + (P - 1 - b)) * P + (P - 1 - c)) * P + (P - 1 - e);
                    t.sig[TG::col_off(j) + s_list_n] = (uint16_t)((P - 1 - a) | ((P - 1 - b) << 4) |
                                                                  ((P - 1 - c) << 8) | ((P - 1 - e) << 12));
                    t.sidx[sg] = (int16_t)s_list_n++;
                }
        for (int k = s_list_n; k < TG::rs(j); ++k) t.sig[TG::col_off(j) + k] = 0xFFFF;
        // c' in B_j (descending lex) and their a_perm segments
        for (int c1 = j; c1 >= 0; --c1)
            for (int c2 = j - c1; c2 >= 0; --c2)
                for (int c3 = j - c1 - c2; c3 >= 0; --c3) {
                    int c4 = j - c1 - c2 - c3;
                    t.cprime[ncp] = (uint32_t)c1 | ((uint32_t)c2 << 8) | ((uint32_t)c3 << 16) | ((uint32_t)c4 << 24);
                    t.cp_seg[ncp] = seg;
                    t.cp_j[ncp] = j;
                    int k = 0;
                    for (int a = 0; a < P; ++a)
                        for (int b = 0; b < P; ++b)
                            for (int c = 0; c < P; ++c) {
                                int e = target - a - b - c;
                                if (e < 0 || e >= P) continue;
                                int x2 = P * c2 + b, x3 = P * c3 + c, x4 = P * c4 + e;
                                int64_t m1 = x2 + x3 + x4, m2 = x3 + x4;
                                t.aperm_src[seg + k] =
                                    (uint16_t)((m1 + 2) * (m1 + 1) * m1 / 6 + (m2 + 1) * m2 / 2 + x4);
                                ++k;
                            }
                    for (; k < TG::rs(j); ++k) t.aperm_src[seg + k] = 0xFFFF;
                    seg += TG::rs(j);
                    ++ncp;
                }
    }
    return t;
}

}  // namespace qfs

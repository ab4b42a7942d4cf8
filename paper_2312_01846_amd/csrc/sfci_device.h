// Device-side building blocks of sigma = H v on gfx950.
//
// One 64-lane wavefront owns one source determinant at a time and walks its
// connected determinants (Sec. 3: single and double excitations, elements
// generated on the fly) in six classes: diagonal, alpha singles, beta singles,
// alpha-alpha doubles, beta-beta doubles, alpha-beta doubles.  Per-source
// tables (occupied/virtual lists, single-excitation ranks and phases, pair
// lists) live in a per-wave LDS slice; the alpha-beta class, which holds most
// of the terms, then costs two LDS reads, one integral gather and one rank add
// per term.  What happens to a term is decided by a Sink (dense FP64 atomics,
// counting, tuple emission for the sort path, or the backward gather).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;

#define SFCI_MAXN 32
#define SFCI_WAVES_PER_BLOCK 4
#define SFCI_BLOCK (64 * SFCI_WAVES_PER_BLOCK)
#define SFCI_MAX_SINGLES 256  // max k (n - k) for n <= 32
#define SFCI_MAX_PAIRS 496    // C(32, 2)

// Binomial table C(a, b), 0 <= a, b <= 32, row-major 33 x 33 (C(a,b) = 0 for b > a).
struct BinomLds {
    u64 c[33][33];
};

__device__ __forceinline__ void load_binom(BinomLds& B, const u64* __restrict__ gtab) {
    for (int t = threadIdx.x; t < 33 * 33; t += blockDim.x) (&B.c[0][0])[t] = gtab[t];
}

// Eq. 12 on a spin string: sum over occupied orbitals p (ascending, t-th
// electron) of C(p, t).
__device__ __forceinline__ u64 str_rank(u32 bits, const BinomLds& B) {
    u64 r = 0;
    int t = 0;
    while (bits) {
        int p = __builtin_ctz(bits);
        bits &= bits - 1u;
        ++t;
        r += B.c[p][t];
    }
    return r;
}

// Inverse of Eq. 12 for k electrons in n orbitals.  Never indexes outside the
// table: the search stops at c = t - 1 at the latest because C(t-1, t) = 0.
__device__ __forceinline__ u32 str_unrank(u64 r, int k, int n, const BinomLds& B) {
    u32 bits = 0;
    int c = n;
    for (int t = k; t >= 1; --t) {
        c = c - 1;
        while (B.c[c][t] > r) --c;
        bits |= 1u << c;
        r -= B.c[c][t];
    }
    return bits;
}

// The same, by a whole wavefront (every lane active, every lane gets the
// string): electron t's orbital is the highest c below the previous one with
// C(c, t) <= r, found by one ballot over lanes c instead of a downward scan.
__device__ __forceinline__ u32 str_unrank_wave(u64 r, int k, int n, const BinomLds& B) {
    const int lane = (int)(threadIdx.x & 63u);
    u32 bits = 0;
    int hi = n;
    for (int t = k; t >= 1; --t) {
        const bool ok = lane < hi && B.c[lane][t] <= r;
        const int c = 63 - __clzll((long long)__ballot(ok));  // C(c, t) = 0 <= r for c < t: never empty
        bits |= 1u << c;
        r -= B.c[c][t];
        hi = c;
    }
    return bits;
}

// Parity of the occupied orbitals strictly between i and a (i != a).
__device__ __forceinline__ int between_parity(u32 S, int i, int a) {
    int lo = i < a ? i : a, hi = i < a ? a : i;
    u32 m = ((1u << hi) - 1u) & ~((2u << lo) - 1u);
    return __popc(S & m) & 1;
}

struct Ints {
    const double* __restrict__ h;  // n*n
    const double* __restrict__ g;  // n^4, (pq|rs) at ((p*n+q)*n+r)*n+s
    int n;
    // h and g live in device global memory: read them as such (not through flat addressing)
    __device__ __forceinline__ double H(int p, int q) const {
        return ((const __attribute__((address_space(1))) double*)h)[p * n + q];
    }
    __device__ __forceinline__ double G(int p, int q, int r, int s) const {
        return ((const __attribute__((address_space(1))) double*)g)[((p * n + q) * n + r) * n + s];
    }
};

// Diagonal element.  The addition order is fixed so that every mode, and the
// CPU reference, produce the same bits: alpha h_pp, beta h_pp, alpha pairs
// p<q [(pp|qq) - (pq|qp)], beta pairs, then alpha-beta (pp|qq).
__device__ inline double diag_element(const Ints& I, u32 A, u32 Bs) {
    double e = 0.0;
    for (u32 m = A; m; m &= m - 1u) { int p = __builtin_ctz(m); e += I.H(p, p); }
    for (u32 m = Bs; m; m &= m - 1u) { int p = __builtin_ctz(m); e += I.H(p, p); }
    for (u32 m = A; m; m &= m - 1u) {
        int p = __builtin_ctz(m);
        for (u32 m2 = (m & (m - 1u)); m2; m2 &= m2 - 1u) {
            int q = __builtin_ctz(m2);
            e += (I.G(p, p, q, q) - I.G(p, q, q, p));
        }
    }
    for (u32 m = Bs; m; m &= m - 1u) {
        int p = __builtin_ctz(m);
        for (u32 m2 = (m & (m - 1u)); m2; m2 &= m2 - 1u) {
            int q = __builtin_ctz(m2);
            e += (I.G(p, p, q, q) - I.G(p, q, q, p));
        }
    }
    for (u32 m = A; m; m &= m - 1u) {
        int p = __builtin_ctz(m);
        for (u32 m2 = Bs; m2; m2 &= m2 - 1u) {
            int q = __builtin_ctz(m2);
            e += I.G(p, p, q, q);
        }
    }
    return e;
}

// Single excitation i -> a in string Ss (other spin So), without the phase:
// h_ia + sum_{k in Ss, k != i} [(ia|kk) - (ik|ka)] + sum_{k in So} (ia|kk).
__device__ inline double single_element_nophase(const Ints& I, u32 Ss, u32 So, int i, int a) {
    double e = I.H(i, a);
    for (u32 m = Ss & ~(1u << i); m; m &= m - 1u) {
        int k = __builtin_ctz(m);
        e += (I.G(i, a, k, k) - I.G(i, k, k, a));
    }
    for (u32 m = So; m; m &= m - 1u) {
        int k = __builtin_ctz(m);
        e += I.G(i, a, k, k);
    }
    return e;
}

// Per-wave LDS slice holding the tables of the current source.
struct WaveLds {
    u64 aRankNb[SFCI_MAX_SINGLES];  // alpha single: rank(alpha') * N_beta
    u32 aInfo[SFCI_MAX_SINGLES];    // i | a << 8 | phase bit << 16
    u32 bRank[SFCI_MAX_SINGLES];    // beta single: rank(beta') (< 2^32 for n <= 32)
    u32 bInfo[SFCI_MAX_SINGLES];
    uint16_t pairOA[SFCI_MAX_PAIRS], pairVA[SFCI_MAX_PAIRS];  // (x | y << 8), x < y
    uint16_t pairOB[SFCI_MAX_PAIRS], pairVB[SFCI_MAX_PAIRS];
    uint8_t occA[32], virA[32], occB[32], virB[32];
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Pair index -> (x, y), 0 <= x < y < k, in lexicographic order.
__device__ __forceinline__ uint16_t decode_pair(int idx, int k) {
    int x = 0;
    while (idx >= k - 1 - x) { idx -= k - 1 - x; ++x; }
    return (uint16_t)(x | ((x + 1 + idx) << 8));
}

struct SpaceDev {
    int n, na, nb;
    u64 Na, Nb;
};

// Range filter on the target alpha rank (used by the sort path's passes).
struct AlphaRange {
    u64 lo, hi;  // keep targets with lo <= rank(alpha') < hi
    __device__ __forceinline__ bool in(u64 ra) const { return ra >= lo && ra < hi; }
};

// What a sink is told about each term besides target and element: the class
// (0 diagonal, 1 alpha single, 2 beta single, 3 alpha-alpha double, 4
// beta-beta double, 5 alpha-beta double), the orbitals (i->a, j->b; for a beta
// single the orbitals are in i, a), the phase parity and the source strings.
struct Term {
    int cls, i, a, j, b, par;  // cls: 0 diagonal, 1/2 alpha/beta single, 3/4/5 alpha-alpha/beta-beta/alpha-beta double
    u32 A, Bs;
};

// Excitation screen (the heat-bath idea named for future work in Sec. 4): a
// double excitation's term value t = H_ki v_i is dropped when |t| < eps_x
// (the element of a double depends only on its four orbitals).  eps_x = 0
// keeps everything.
__device__ __forceinline__ bool xscreened(double t, double eps_x) { return fabs(t) < eps_x; }

// Number of (source, excitation) pairs visited per source.
__host__ __device__ inline u64 terms_per_source(int n, int na, int nb) {
    u64 sa = (u64)na * (n - na), sb = (u64)nb * (n - nb);
    u64 pa = (u64)na * (na - 1) / 2, qa = (u64)(n - na) * (n - na - 1) / 2;
    u64 pb = (u64)nb * (nb - 1) / 2, qb = (u64)(n - nb) * (n - nb - 1) / 2;
    return 1 + sa + sb + pa * qa + pb * qb + sa * sb;
}

// Walk every connected determinant of the source (R, c).  All 64 lanes of the
// wave must call this together with the same arguments.  sink(ok, target, e,
// c, term) is called wave-uniformly; ok is false for padding lanes and, unless
// ALL is set, for elements that are exactly zero.
template <bool FILTER, class Sink, bool ALL = false>
__device__ void enumerate_source(const SpaceDev& sp, const Ints& I, const BinomLds& B, WaveLds& W, u64 R,
                                 double c, const AlphaRange& rng, Sink& sink) {
    const int lane = lane_id();
    const int n = sp.n, na = sp.na, nb = sp.nb;
    const int nva = n - na, nvb = n - nb;
    const u64 Nb = sp.Nb;
    const u64 rA = R / Nb;
    const u64 rB = R - rA * Nb;
    const u32 A = str_unrank(rA, na, n, B);
    const u32 Bs = str_unrank(rB, nb, n, B);
    const u64 baseA = rA * Nb;

    wave_sync();  // previous source's tables are no longer read
    if (lane < n) {
        u32 below = (1u << lane) - 1u;
        if ((A >> lane) & 1u) W.occA[__popc(A & below)] = (uint8_t)lane;
        else W.virA[lane - __popc(A & below)] = (uint8_t)lane;
        if ((Bs >> lane) & 1u) W.occB[__popc(Bs & below)] = (uint8_t)lane;
        else W.virB[lane - __popc(Bs & below)] = (uint8_t)lane;
    }
    const int sA = na * nva, sB = nb * nvb;
    const int PA = na * (na - 1) / 2, QA = nva * (nva - 1) / 2;
    const int PB = nb * (nb - 1) / 2, QB = nvb * (nvb - 1) / 2;
    for (int t = lane; t < PA; t += 64) W.pairOA[t] = decode_pair(t, na);
    for (int t = lane; t < QA; t += 64) W.pairVA[t] = decode_pair(t, nva);
    for (int t = lane; t < PB; t += 64) W.pairOB[t] = decode_pair(t, nb);
    for (int t = lane; t < QB; t += 64) W.pairVB[t] = decode_pair(t, nvb);
    wave_sync();
    for (int t = lane; t < sA; t += 64) {
        int i = W.occA[t / nva], a = W.virA[t % nva];
        u32 A2 = A ^ (1u << i) ^ (1u << a);
        W.aRankNb[t] = str_rank(A2, B) * Nb;
        W.aInfo[t] = (u32)i | ((u32)a << 8) | ((u32)between_parity(A, i, a) << 16);
    }
    for (int t = lane; t < sB; t += 64) {
        int j = W.occB[t / nvb], b = W.virB[t % nvb];
        u32 B2 = Bs ^ (1u << j) ^ (1u << b);
        W.bRank[t] = (u32)str_rank(B2, B);
        W.bInfo[t] = (u32)j | ((u32)b << 8) | ((u32)between_parity(Bs, j, b) << 16);
    }
    wave_sync();

    const bool keepA = !FILTER || rng.in(rA);

    // (a) diagonal
    {
        bool ok = false;
        double e = 0.0;
        if (lane == 0 && keepA) {
            e = diag_element(I, A, Bs);
            ok = ALL || (e != 0.0);
        }
        sink(ok, R, e, c, Term{0, 0, 0, 0, 0, 0, A, Bs});
    }
    // (b) alpha singles, beta unchanged
    for (int t0 = 0; t0 < sA; t0 += 64) {
        int t = t0 + lane;
        bool ok = false;
        double e = 0.0;
        u64 tgt = 0;
        Term tm{1, 0, 0, 0, 0, 0, A, Bs};
        if (t < sA) {
            u64 rnb = W.aRankNb[t];
            u32 info = W.aInfo[t];
            if (!FILTER || rng.in(rnb / Nb)) {
                int i = info & 255, a = (info >> 8) & 255;
                e = single_element_nophase(I, A, Bs, i, a);
                tm.i = i; tm.a = a; tm.par = (info >> 16) & 1;
                if (tm.par) e = -e;
                tgt = rnb + rB;
                ok = ALL || (e != 0.0);
            }
        }
        sink(ok, tgt, e, c, tm);
    }
    // (c) beta singles, alpha unchanged
    for (int t0 = 0; t0 < sB; t0 += 64) {
        int t = t0 + lane;
        bool ok = false;
        double e = 0.0;
        u64 tgt = 0;
        Term tm{2, 0, 0, 0, 0, 0, A, Bs};
        if (t < sB && keepA) {
            u32 info = W.bInfo[t];
            int j = info & 255, b = (info >> 8) & 255;
            e = single_element_nophase(I, Bs, A, j, b);
            tm.i = j; tm.a = b; tm.par = (info >> 16) & 1;
            if (tm.par) e = -e;
            tgt = baseA + W.bRank[t];
            ok = ALL || (e != 0.0);
        }
        sink(ok, tgt, e, c, tm);
    }
    // (d) alpha-alpha doubles: (i<j) x (a<b), pairing i->a, j->b
    {
        const int tot = PA * QA;
        int q = (QA > 0) ? lane / QA : 0, r = (QA > 0) ? lane % QA : 0;
        const int dq = (QA > 0) ? 64 / QA : 0, dr = (QA > 0) ? 64 % QA : 0;
        for (int t0 = 0; t0 < tot; t0 += 64) {
            int t = t0 + lane;
            bool ok = false;
            double e = 0.0;
            u64 tgt = 0;
            Term tm{3, 0, 0, 0, 0, 0, A, Bs};
            if (t < tot) {
                u32 po = W.pairOA[q], pv = W.pairVA[r];
                int i = W.occA[po & 255], j = W.occA[po >> 8];
                int a = W.virA[pv & 255], b = W.virA[pv >> 8];
                u32 mid = A ^ (1u << i) ^ (1u << a);
                u32 A2 = mid ^ (1u << j) ^ (1u << b);
                u64 ra = str_rank(A2, B);
                if (!FILTER || rng.in(ra)) {
                    int par = between_parity(A, i, a) ^ between_parity(mid, j, b);
                    e = (I.G(i, a, j, b) - I.G(i, b, j, a));
                    if (par) e = -e;
                    tgt = ra * Nb + rB;
                    ok = ALL || (e != 0.0);
                    tm = Term{3, i, a, j, b, par, A, Bs};
                }
            }
            sink(ok, tgt, e, c, tm);
            r += dr; q += dq;
            if (r >= QA) { r -= QA; q += 1; }
        }
    }
    // (e) beta-beta doubles
    {
        const int tot = PB * QB;
        int q = (QB > 0) ? lane / QB : 0, r = (QB > 0) ? lane % QB : 0;
        const int dq = (QB > 0) ? 64 / QB : 0, dr = (QB > 0) ? 64 % QB : 0;
        for (int t0 = 0; t0 < tot; t0 += 64) {
            int t = t0 + lane;
            bool ok = false;
            double e = 0.0;
            u64 tgt = 0;
            Term tm{4, 0, 0, 0, 0, 0, A, Bs};
            if (t < tot && keepA) {
                u32 po = W.pairOB[q], pv = W.pairVB[r];
                int i = W.occB[po & 255], j = W.occB[po >> 8];
                int a = W.virB[pv & 255], b = W.virB[pv >> 8];
                u32 mid = Bs ^ (1u << i) ^ (1u << a);
                u32 B2 = mid ^ (1u << j) ^ (1u << b);
                int par = between_parity(Bs, i, a) ^ between_parity(mid, j, b);
                e = (I.G(i, a, j, b) - I.G(i, b, j, a));
                if (par) e = -e;
                tgt = baseA + str_rank(B2, B);
                ok = ALL || (e != 0.0);
                tm = Term{4, i, a, j, b, par, A, Bs};
            }
            sink(ok, tgt, e, c, tm);
            r += dr; q += dq;
            if (r >= QB) { r -= QB; q += 1; }
        }
    }
    // (f) alpha-beta doubles: (i->a in alpha) x (j->b in beta), element (ia|jb)
    {
        const int tot = sA * sB;
        int q = (sB > 0) ? lane / sB : 0, r = (sB > 0) ? lane % sB : 0;
        const int dq = (sB > 0) ? 64 / sB : 0, dr = (sB > 0) ? 64 % sB : 0;
        for (int t0 = 0; t0 < tot; t0 += 64) {
            int t = t0 + lane;
            bool ok = false;
            double e = 0.0;
            u64 tgt = 0;
            Term tm{5, 0, 0, 0, 0, 0, A, Bs};
            if (t < tot) {
                u64 rnb = W.aRankNb[q];
                if (!FILTER || rng.in(rnb / Nb)) {
                    u32 ai = W.aInfo[q], bi = W.bInfo[r];
                    int i = ai & 255, a = (ai >> 8) & 255;
                    int j = bi & 255, b = (bi >> 8) & 255;
                    e = I.G(i, a, j, b);
                    int par = ((ai ^ bi) >> 16) & 1u;
                    if (par) e = -e;
                    tgt = rnb + W.bRank[r];
                    ok = ALL || (e != 0.0);
                    tm.i = i; tm.a = a; tm.j = j; tm.b = b; tm.par = par;
                }
            }
            sink(ok, tgt, e, c, tm);
            r += dr; q += dq;
            if (r >= sB) { r -= sB; q += 1; }
        }
    }
}

// Sparse-FCI CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, obviously-correct CPU reference for the sigma = H v hot path
// of sparse full configuration interaction (Wang, arXiv 2312.01846).  Only the
// test suite, the smoke check and the CPU-baseline leg of the benchmark may
// load it; the product path never does.  It shares no code with the HIP
// library.  Everything is FP64, compiled with -ffp-contract=off.
//
// Conventions (readings of points the paper leaves open):
//  * A spin string is an n-bit mask; bit p set means spatial orbital p is
//    occupied.  The paper writes strings left to right starting at orbital 1,
//    so the leftmost character is bit 0 (Sec. 2.2, Table 1).
//  * String rank (Sec. 2.2, Eq. 12): h = sum_{i=1..k} C(chi_i - 1, i) over the
//    ascending 1-based occupied orbitals chi_i, with C(a, b) = 0 for a < b.
//  * Determinant rank: R = r_alpha * N_beta + r_beta (alpha-major), so alpha
//    rank ranges are contiguous rank ranges (Sec. 3 buckets on spin-up only).
//  * Spin orbitals are ordered all-alpha then all-beta, orbital ascending;
//    |D> = product of creators in that order acting on |0> (Jordan-Wigner).
//  * H = sum_pq h_pq sum_s a+_ps a_qs
//      + 1/2 sum_pqrs (pq|rs) sum_st a+_ps a+_rt a_st a_qs   (real orbitals).
//
// Functions whose results have a plain definition compute that definition:
//  * orc_sigma_explicit applies H term by term in second quantization.
//  * orc_sigma_entry computes one entry sigma_k = sum_i H_ki v_i (ascending i).
// The remaining functions follow the paper's algorithm steps:
//  * orc_sigma: generate intermediate elements from each input entry, then
//    merge equal determinants by a stable sort and a linear scan (Sec. 2.2).
//  * orc_topm / orc_lanczos: the truncated Lanczos basis, the generalized
//    eigenproblem T x = lambda S x and the restart (Sec. 2.1, Eqs. 10-11).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <parallel/algorithm>
#include <vector>

typedef uint64_t u64;
typedef int64_t i64;

// ---------------------------------------------------------------------------
// Binomial coefficients C(a, b) for 0 <= a <= 64, by Pascal's rule.
// C(64, 32) < 2^64, so every entry fits in u64.
static u64 g_binom[65][65];
static bool g_binom_ready = false;

static void binom_init() {
    if (g_binom_ready) return;
    for (int a = 0; a <= 64; ++a) {
        for (int b = 0; b <= 64; ++b) {
            if (b == 0) g_binom[a][b] = 1;
            else if (a == 0) g_binom[a][b] = 0;
            else g_binom[a][b] = g_binom[a - 1][b - 1] + g_binom[a - 1][b];
        }
    }
    g_binom_ready = true;
}

extern "C" u64 orc_binom(int a, int b) {
    binom_init();
    if (a < 0 || b < 0 || a > 64 || b > 64 || a < b) return 0;
    return g_binom[a][b];
}

static int popc(u64 x) { return __builtin_popcountll(x); }

// ---------------------------------------------------------------------------
// Eq. 12: h(D) = sum_{i=1}^{k} C(chi_i - 1, i), chi_i the 1-based orbital of
// the i-th electron, electrons in ascending orbital order.
extern "C" u64 orc_str_rank(u64 bits) {
    binom_init();
    u64 h = 0;
    int i = 0;  // electron counter, 1-based after increment
    while (bits) {
        int p = __builtin_ctzll(bits);  // next occupied orbital, ascending
        bits &= bits - 1ull;
        ++i;
        int chi = p + 1;
        h += g_binom[chi - 1][i];  // chi - 1 >= i - 1; the table holds 0 for chi - 1 < i
    }
    return h;
}

// Inverse of Eq. 12 for strings with k electrons: the k-th electron sits at
// the largest orbital c with C(c, k) <= r, and so on downwards.
extern "C" u64 orc_str_unrank(u64 r, int k) {
    binom_init();
    u64 bits = 0;
    int c = 64;
    for (int i = k; i >= 1; --i) {
        c = c - 1;
        while (c >= 0 && orc_binom(c, i) > r) --c;
        // c >= i - 1 always holds because C(i-1, i) = 0 <= r.
        bits |= 1ull << c;
        r -= orc_binom(c, i);
    }
    return bits;
}

// The successor function g of Sec. 2.2: scanning from the left (orbital 1 =
// bit 0), find the first 1-bit whose right neighbour is a 0-bit; move every
// 1-bit to its left to the far left, and swap the pair.  Returns 0 when the
// input is the final string 00..011..1 (no successor).
extern "C" int orc_gchain_next(u64 bits, int n, u64* out) {
    for (int p = 0; p + 1 < n; ++p) {
        bool one = (bits >> p) & 1ull;
        bool right_zero = !((bits >> (p + 1)) & 1ull);
        if (one && right_zero) {
            int left_ones = popc(bits & ((1ull << p) - 1ull));
            u64 nb = bits & ~((1ull << (p + 2)) - 1ull);  // keep bits right of the pair
            nb |= (1ull << left_ones) - 1ull;               // flushed left
            nb |= 1ull << (p + 1);                          // swapped pair
            *out = nb;
            return 1;
        }
    }
    return 0;
}

extern "C" u64 orc_space_size(int n, int na, int nb) {
    binom_init();
    if (n < 1 || n > 32 || na < 0 || nb < 0 || na > n || nb > n) return 0;
    unsigned __int128 p = (unsigned __int128)orc_binom(n, na) * orc_binom(n, nb);
    if (p >> 64) return 0;
    return (u64)p;
}

extern "C" void orc_det_rank(int n, int na, int nb, const u64* a, const u64* b, i64 cnt, u64* out) {
    u64 Nb = orc_binom(n, nb);
    (void)na;
    for (i64 t = 0; t < cnt; ++t) out[t] = orc_str_rank(a[t]) * Nb + orc_str_rank(b[t]);
}

extern "C" void orc_det_unrank(int n, int na, int nb, const u64* r, i64 cnt, u64* a, u64* b) {
    u64 Nb = orc_binom(n, nb);
    for (i64 t = 0; t < cnt; ++t) {
        a[t] = orc_str_unrank(r[t] / Nb, na);
        b[t] = orc_str_unrank(r[t] % Nb, nb);
    }
}

// ---------------------------------------------------------------------------
// Second quantization on a 2n-bit spin-orbital occupation (alpha 0..n-1, beta
// n..2n-1).  Each returns false when the operator annihilates the state.
static bool op_annihilate(u64& D, int q, int& sign) {
    if (!((D >> q) & 1ull)) return false;
    if (popc(D & ((1ull << q) - 1ull)) & 1) sign = -sign;
    D ^= 1ull << q;
    return true;
}

static bool op_create(u64& D, int p, int& sign) {
    if ((D >> p) & 1ull) return false;
    if (popc(D & ((1ull << p) - 1ull)) & 1) sign = -sign;
    D |= 1ull << p;
    return true;
}

struct Space {
    int n, na, nb;
    u64 Na, Nb, Ndet;
    const double* h;
    const double* g;
    double H(int p, int q) const { return h[p * n + q]; }
    double G(int p, int q, int r, int s) const { return g[((size_t)(p * n + q) * n + r) * n + s]; }
    u64 rank_so(u64 D) const {  // spin-orbital bits -> determinant rank
        u64 a = D & ((1ull << n) - 1ull);
        u64 b = D >> n;
        return orc_str_rank(a) * Nb + orc_str_rank(b);
    }
    u64 so_of_rank(u64 R) const {
        u64 a = orc_str_unrank(R / Nb, na);
        u64 b = orc_str_unrank(R % Nb, nb);
        return a | (b << n);
    }
};

static Space make_space(int n, int na, int nb, const double* h, const double* g) {
    binom_init();
    Space S;
    S.n = n; S.na = na; S.nb = nb;
    S.Na = orc_binom(n, na); S.Nb = orc_binom(n, nb); S.Ndet = S.Na * S.Nb;
    S.h = h; S.g = g;
    return S;
}

// Enumerate H|D> term by term: for every operator string with a nonzero
// integral, call f(target spin-orbital bits, coefficient).  The coefficient
// is integral * fermionic sign (one-body) or 1/2 * integral * sign (two-body).
template <class F>
static void apply_H_explicit(const Space& S, u64 D0, F&& f) {
    const int n = S.n;
    for (int sg = 0; sg < 2; ++sg) {
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) {
                double hpq = S.H(p, q);
                if (hpq == 0.0) continue;
                u64 D = D0; int sign = 1;
                if (!op_annihilate(D, q + sg * n, sign)) continue;
                if (!op_create(D, p + sg * n, sign)) continue;
                f(D, hpq * (double)sign);
            }
    }
    for (int sg = 0; sg < 2; ++sg)
        for (int tg = 0; tg < 2; ++tg)
            for (int p = 0; p < n; ++p)
                for (int q = 0; q < n; ++q)
                    for (int r = 0; r < n; ++r)
                        for (int s = 0; s < n; ++s) {
                            double v = S.G(p, q, r, s);
                            if (v == 0.0) continue;
                            u64 D = D0; int sign = 1;
                            if (!op_annihilate(D, q + sg * n, sign)) continue;
                            if (!op_annihilate(D, s + tg * n, sign)) continue;
                            if (!op_create(D, r + tg * n, sign)) continue;
                            if (!op_create(D, p + sg * n, sign)) continue;
                            f(D, 0.5 * v * (double)sign);
                        }
}

// Plain definition of sigma = H v on a tiny space, by explicit operator
// application.  out_dense has N_det entries and is overwritten.
extern "C" int orc_sigma_explicit(int n, int na, int nb, const double* h, const double* g, i64 nnz,
                                  const u64* rank, const double* amp, double* out_dense) {
    Space S = make_space(n, na, nb, h, g);
    for (u64 k = 0; k < S.Ndet; ++k) out_dense[k] = 0.0;
    for (i64 t = 0; t < nnz; ++t) {
        if (rank[t] >= S.Ndet) return -2;
        u64 D0 = S.so_of_rank(rank[t]);
        double vi = amp[t];
        apply_H_explicit(S, D0, [&](u64 D, double c) { out_dense[S.rank_so(D)] += c * vi; });
    }
    return 0;
}

// Dense H matrix of a tiny space by explicit operator application.  The
// determinants are enumerated along the g-chain (Sec. 2.2): the alpha and beta
// strings are each walked from 11..100..0 by successive applications of g.
extern "C" int orc_dense_H(int n, int na, int nb, const double* h, const double* g, double* Hout) {
    Space S = make_space(n, na, nb, h, g);
    if (S.Ndet > 20000) return -1;
    std::vector<u64> astr, bstr;
    u64 x = (1ull << na) - 1ull, y;
    astr.push_back(x);
    while (orc_gchain_next(x, n, &y)) { astr.push_back(y); x = y; }
    x = (1ull << nb) - 1ull;
    bstr.push_back(x);
    while (orc_gchain_next(x, n, &y)) { bstr.push_back(y); x = y; }
    if (astr.size() != S.Na || bstr.size() != S.Nb) return -3;
    // Chain position -> determinant index (alpha-major); the explicit H uses
    // a std::vector lookup keyed by the spin-orbital pattern through a sort.
    std::vector<std::pair<u64, u64>> key;  // (spin-orbital bits, chain index)
    for (u64 ia = 0; ia < S.Na; ++ia)
        for (u64 ib = 0; ib < S.Nb; ++ib) key.push_back({astr[ia] | (bstr[ib] << n), ia * S.Nb + ib});
    std::sort(key.begin(), key.end());
    auto index_of = [&](u64 D) -> u64 {
        auto it = std::lower_bound(key.begin(), key.end(), std::make_pair(D, (u64)0));
        return it->second;
    };
    u64 N = S.Ndet;
    for (u64 t = 0; t < N * N; ++t) Hout[t] = 0.0;
    for (u64 col = 0; col < N; ++col) {
        u64 D0 = astr[col / S.Nb] | (bstr[col % S.Nb] << n);
        apply_H_explicit(S, D0, [&](u64 D, double c) { Hout[index_of(D) * N + col] += c; });
    }
    return 0;
}

// ---------------------------------------------------------------------------
// Slater-Condon generation of the connected determinants of one source
// (Sec. 3: "up to double excitations"; generation on the fly, Sec. 2.2).
//
// Phase of moving an electron i -> a inside one spin string S: (-1) to the
// number of occupied orbitals strictly between i and a.
static int single_sign(u64 S, int i, int a) {
    int lo = i < a ? i : a, hi = i < a ? a : i;
    u64 between = ((1ull << hi) - 1ull) & ~((1ull << (lo + 1)) - 1ull);
    return (popc(S & between) & 1) ? -1 : 1;
}

static void occ_virt(u64 S, int n, std::vector<int>& occ, std::vector<int>& vir) {
    occ.clear(); vir.clear();
    occ.reserve(32); vir.reserve(32);
    for (int p = 0; p < n; ++p) ((S >> p) & 1ull) ? occ.push_back(p) : vir.push_back(p);
}

// Diagonal element <D|H|D>.  Addition order is fixed: alpha one-body, beta
// one-body, alpha pairs p<q, beta pairs p<q, then alpha-beta pairs.
static double diag_element(const Space& S, const std::vector<int>& oa, const std::vector<int>& ob) {
    double e = 0.0;
    for (int p : oa) e += S.H(p, p);
    for (int p : ob) e += S.H(p, p);
    for (size_t x = 0; x < oa.size(); ++x)
        for (size_t y = x + 1; y < oa.size(); ++y) {
            int p = oa[x], q = oa[y];
            e += (S.G(p, p, q, q) - S.G(p, q, q, p));
        }
    for (size_t x = 0; x < ob.size(); ++x)
        for (size_t y = x + 1; y < ob.size(); ++y) {
            int p = ob[x], q = ob[y];
            e += (S.G(p, p, q, q) - S.G(p, q, q, p));
        }
    for (int p : oa)
        for (int q : ob) e += S.G(p, p, q, q);
    return e;
}

// Single excitation i -> a in spin string "same" (occupied list os), with the
// other spin's occupied list oo.  Returns sign * element.
static double single_element(const Space& S, u64 same, const std::vector<int>& os,
                             const std::vector<int>& oo, int i, int a) {
    double e = S.H(i, a);
    for (int k : os) {
        if (k == i) continue;
        e += (S.G(i, a, k, k) - S.G(i, k, k, a));
    }
    for (int k : oo) e += S.G(i, a, k, k);
    return (double)single_sign(same, i, a) * e;
}

// Enumerate all (target alpha, target beta, element) of one source in the
// canonical order: diagonal; alpha singles; beta singles; alpha-alpha doubles
// (i<j, a<b lexicographic); beta-beta doubles; alpha-beta doubles (i,a,j,b).
// Elements that are exactly 0.0 are not reported.  f(A', B', element, kind)
// with kind 0 = diagonal, 1 = single, 2 = double excitation.
enum { TERM_DIAG = 0, TERM_SINGLE = 1, TERM_DOUBLE = 2 };

template <class F>
static void sc_terms_kind(const Space& S, u64 A, u64 B, F&& f) {
    const int n = S.n;
    static thread_local std::vector<int> oa, va, ob, vb;
    occ_virt(A, n, oa, va);
    occ_virt(B, n, ob, vb);
    double e = diag_element(S, oa, ob);
    if (e != 0.0) f(A, B, e, TERM_DIAG);
    for (int i : oa)
        for (int a : va) {
            double x = single_element(S, A, oa, ob, i, a);
            if (x != 0.0) f(A ^ (1ull << i) ^ (1ull << a), B, x, TERM_SINGLE);
        }
    for (int i : ob)
        for (int a : vb) {
            double x = single_element(S, B, ob, oa, i, a);
            if (x != 0.0) f(A, B ^ (1ull << i) ^ (1ull << a), x, TERM_SINGLE);
        }
    for (int spin = 0; spin < 2; ++spin) {
        u64 Str = spin == 0 ? A : B;
        const std::vector<int>& oc = spin == 0 ? oa : ob;
        const std::vector<int>& vi = spin == 0 ? va : vb;
        for (size_t x = 0; x < oc.size(); ++x)
            for (size_t y = x + 1; y < oc.size(); ++y)
                for (size_t u = 0; u < vi.size(); ++u)
                    for (size_t w = u + 1; w < vi.size(); ++w) {
                        int i = oc[x], j = oc[y], a = vi[u], b = vi[w];
                        u64 mid = Str ^ (1ull << i) ^ (1ull << a);
                        int sg = single_sign(Str, i, a) * single_sign(mid, j, b);
                        double v = (double)sg * (S.G(i, a, j, b) - S.G(i, b, j, a));
                        if (v == 0.0) continue;
                        u64 T = mid ^ (1ull << j) ^ (1ull << b);
                        if (spin == 0) f(T, B, v, TERM_DOUBLE); else f(A, T, v, TERM_DOUBLE);
                    }
    }
    for (int i : oa)
        for (int a : va) {
            int sa = single_sign(A, i, a);
            u64 A2 = A ^ (1ull << i) ^ (1ull << a);
            for (int j : ob)
                for (int b : vb) {
                    int sb = single_sign(B, j, b);
                    double v = (double)(sa * sb) * S.G(i, a, j, b);
                    if (v == 0.0) continue;
                    f(A2, B ^ (1ull << j) ^ (1ull << b), v, TERM_DOUBLE);
                }
        }
}

template <class F>
static void sc_terms(const Space& S, u64 A, u64 B, F&& f) {
    sc_terms_kind(S, A, B, [&](u64 A2, u64 B2, double e, int) { f(A2, B2, e); });
}

// Matrix element <target|H|source> by Slater-Condon generation from the
// source (0.0 when the two are not connected).
extern "C" double orc_element(int n, int na, int nb, const double* h, const double* g, u64 src_rank,
                              u64 tgt_rank) {
    Space S = make_space(n, na, nb, h, g);
    u64 A = orc_str_unrank(src_rank / S.Nb, na), B = orc_str_unrank(src_rank % S.Nb, nb);
    double out = 0.0;
    sc_terms(S, A, B, [&](u64 A2, u64 B2, double e) {
        if (orc_str_rank(A2) * S.Nb + orc_str_rank(B2) == tgt_rank) out = e;
    });
    return out;
}

// Per-source term dump in canonical order (ranks and elements), for tests.
extern "C" i64 orc_source_terms(int n, int na, int nb, const double* h, const double* g, u64 src_rank,
                                u64* tgt, double* elem, i64 cap) {
    Space S = make_space(n, na, nb, h, g);
    u64 A = orc_str_unrank(src_rank / S.Nb, na), B = orc_str_unrank(src_rank % S.Nb, nb);
    i64 cnt = 0;
    sc_terms(S, A, B, [&](u64 A2, u64 B2, double e) {
        if (cnt < cap) { tgt[cnt] = orc_str_rank(A2) * S.Nb + orc_str_rank(B2); elem[cnt] = e; }
        ++cnt;
    });
    return cnt;
}

// ---------------------------------------------------------------------------
// sigma = H v by the paper's two steps (Sec. 2.2): generate the intermediate
// elements (target, H_ki v_i) from every input entry, sources in ascending
// rank; then merge equal targets: stable sort by target, scan and add.  Every
// target therefore receives its contributions in ascending source order.
// Output: entries whose merged value is not 0.0, ascending rank, together
// with sum_i |H_ki v_i| per entry (the scale for amplitude tolerances).
// Returns the number of output entries, or -(needed) when cap is too small
// (the output arrays may then be NULL), or -1 on bad input.
struct Acc { u64 r; double v, a; };
typedef std::pair<u64, double> Tup;

static void stable_sort_by_target(std::vector<Tup>& tup) {
    std::stable_sort(tup.begin(), tup.end(), [](const Tup& x, const Tup& y) { return x.first < y.first; });
}

// Merge a chunk of intermediate elements, sorted by target (equal targets in
// source order), into the running merged list: one addition at a time.
static void merge_chunk(std::vector<Acc>& run, const std::vector<Tup>& tup) {
    std::vector<Acc> next;
    next.reserve(run.size() + tup.size());
    size_t x = 0, y = 0;
    while (x < run.size() || y < tup.size()) {
        if (y == tup.size() || (x < run.size() && run[x].r < tup[y].first)) {
            next.push_back(run[x++]);
            continue;
        }
        Acc cur;
        if (x < run.size() && run[x].r == tup[y].first) cur = run[x++];
        else { cur.r = tup[y].first; cur.v = 0.0; cur.a = 0.0; }
        while (y < tup.size() && tup[y].first == cur.r) {
            cur.v += tup[y].second;
            cur.a += std::fabs(tup[y].second);
            ++y;
        }
        next.push_back(cur);
    }
    run.swap(next);
}

// eps_x > 0: the excitation screen -- a double excitation's term H_ki v_i is
// not generated when |H_ki v_i| < eps_x (the element of a double depends only
// on its four orbitals: the heat-bath idea named for future work in Sec. 4).
// Singles and the diagonal are always generated.
static inline bool screened(int kind, double t, double eps_x) {
    return kind == TERM_DOUBLE && std::fabs(t) < eps_x;
}

static std::vector<Acc> sigma_merged_seq(const Space& S, i64 nnz, const u64* rank, const double* amp,
                                         double eps_x) {
    const int na = S.na, nb = S.nb;
    std::vector<Acc> run;       // merged so far, ascending rank
    std::vector<Tup> tup;
    const size_t chunk_cap = (size_t)1 << 25;
    i64 t = 0;
    while (t < nnz) {
        tup.clear();
        // Generate intermediate elements for a run of sources.
        while (t < nnz && tup.size() < chunk_cap) {
            u64 A = orc_str_unrank(rank[t] / S.Nb, na), B = orc_str_unrank(rank[t] % S.Nb, nb);
            double vi = amp[t];
            sc_terms_kind(S, A, B, [&](u64 A2, u64 B2, double e, int kind) {
                const double tv = e * vi;
                if (screened(kind, tv, eps_x)) return;
                tup.push_back({orc_str_rank(A2) * S.Nb + orc_str_rank(B2), tv});
            });
            ++t;
        }
        stable_sort_by_target(tup);
        merge_chunk(run, tup);
    }
    return run;
}

// The same two steps in the paper's shared-memory parallel form (Sec. 2.2):
// each of T threads generates the intermediate elements of its own segment
// of the input into thread-local buckets (bucket = an equal range of the
// determinant rank, the hash-range split); then every bucket is merged on its
// own by one thread, its threads' parts taken in thread order.  The paper
// sorts a bucket with introsort; here the sort is stable, so that every target
// still receives its contributions in ascending source order and the result
// has the bits of the sequential form above (tested).
static int g_threads = 1;

extern "C" void orc_set_threads(int t) { g_threads = t < 1 ? 1 : t; }
extern "C" int orc_get_threads(void) { return g_threads; }

static std::vector<Acc> sigma_merged_buckets(const Space& S, i64 nnz, const u64* rank, const double* amp, int T,
                                             double eps_x) {
    const int na = S.na, nb = S.nb, n = S.n;
    const int NB = 16 * T;
    const u64 width = S.Ndet / (u64)NB + 1;
    const i64 sa = (i64)na * (n - na), sb = (i64)nb * (n - nb);
    const i64 per_src = 1 + sa + sb + sa * sb + (i64)(na * (na - 1) / 2) * ((n - na) * (n - na - 1) / 2) +
                        (i64)(nb * (nb - 1) / 2) * ((n - nb) * (n - nb - 1) / 2);
    const i64 chunk_src = std::max<i64>(1, ((i64)1 << 24) * T / per_src);
    std::vector<std::vector<Acc>> run(NB);
    std::vector<std::vector<std::vector<Tup>>> loc(T, std::vector<std::vector<Tup>>(NB));
    for (i64 t0 = 0; t0 < nnz; t0 += chunk_src) {
        const i64 t1 = std::min(nnz, t0 + chunk_src);
#pragma omp parallel for num_threads(T) schedule(static, 1)
        for (int k = 0; k < T; ++k) {
            for (auto& b : loc[k]) b.clear();
            const i64 lo = t0 + (t1 - t0) * k / T, hi = t0 + (t1 - t0) * (k + 1) / T;
            for (i64 t = lo; t < hi; ++t) {
                u64 A = orc_str_unrank(rank[t] / S.Nb, na), B = orc_str_unrank(rank[t] % S.Nb, nb);
                double vi = amp[t];
                sc_terms_kind(S, A, B, [&](u64 A2, u64 B2, double e, int kind) {
                    const double tv = e * vi;
                    if (screened(kind, tv, eps_x)) return;
                    const u64 R = orc_str_rank(A2) * S.Nb + orc_str_rank(B2);
                    loc[k][R / width].push_back({R, tv});
                });
            }
        }
#pragma omp parallel for num_threads(T) schedule(dynamic, 1)
        for (int b = 0; b < NB; ++b) {
            std::vector<Tup> tup;
            for (int k = 0; k < T; ++k) tup.insert(tup.end(), loc[k][b].begin(), loc[k][b].end());
            stable_sort_by_target(tup);
            merge_chunk(run[b], tup);
        }
    }
    std::vector<Acc> out;
    size_t tot = 0;
    for (auto& r : run) tot += r.size();
    out.reserve(tot);
    for (auto& r : run) out.insert(out.end(), r.begin(), r.end());
    return out;
}

static std::vector<Acc> sigma_merged(const Space& S, i64 nnz, const u64* rank, const double* amp,
                                     double eps_x = 0.0) {
    if (g_threads > 1) return sigma_merged_buckets(S, nnz, rank, amp, g_threads, eps_x);
    return sigma_merged_seq(S, nnz, rank, amp, eps_x);
}

extern "C" i64 orc_sigma_x(int n, int na, int nb, const double* h, const double* g, i64 nnz,
                           const u64* rank, const double* amp, u64* out_rank, double* out_amp,
                           double* out_abs, i64 cap, double eps_x) {
    Space S = make_space(n, na, nb, h, g);
    for (i64 t = 0; t < nnz; ++t) {
        if (rank[t] >= S.Ndet) return -1;
        if (t > 0 && rank[t] <= rank[t - 1]) return -1;
    }
    std::vector<Acc> run = sigma_merged(S, nnz, rank, amp, eps_x);
    i64 cnt = 0;
    for (const Acc& e : run)
        if (e.v != 0.0) ++cnt;
    if (cnt > cap) return -cnt;
    i64 o = 0;
    for (const Acc& e : run) {
        if (e.v == 0.0) continue;
        out_rank[o] = e.r; out_amp[o] = e.v;
        if (out_abs) out_abs[o] = e.a;
        ++o;
    }
    return cnt;
}

extern "C" i64 orc_sigma(int n, int na, int nb, const double* h, const double* g, i64 nnz,
                         const u64* rank, const double* amp, u64* out_rank, double* out_amp,
                         double* out_abs, i64 cap) {
    return orc_sigma_x(n, na, nb, h, g, nnz, rank, amp, out_rank, out_amp, out_abs, cap, 0.0);
}

// One output entry by its plain definition: sigma_k = sum_i H_ki v_i with the
// sum over the connected input entries i in ascending rank.  The elements come
// from the Slater-Condon generation of the target k (H is real symmetric and,
// for exactly symmetric integrals, the generated elements are bitwise
// Hermitian, which the tests check).  abs_out = sum_i |H_ki v_i|.
extern "C" double orc_sigma_entry(int n, int na, int nb, const double* h, const double* g, i64 nnz,
                                  const u64* rank, const double* amp, u64 target, double* abs_out) {
    Space S = make_space(n, na, nb, h, g);
    u64 A = orc_str_unrank(target / S.Nb, na), B = orc_str_unrank(target % S.Nb, nb);
    std::vector<std::pair<u64, double>> conn;
    sc_terms(S, A, B, [&](u64 A2, u64 B2, double e) {
        conn.push_back({orc_str_rank(A2) * S.Nb + orc_str_rank(B2), e});
    });
    std::sort(conn.begin(), conn.end());
    double s = 0.0, sa = 0.0;
    for (const auto& c : conn) {
        const u64* it = std::lower_bound(rank, rank + nnz, c.first);
        if (it == rank + nnz || *it != c.first) continue;
        double p = c.second * amp[it - rank];
        s += p;
        sa += std::fabs(p);
    }
    if (abs_out) *abs_out = sa;
    return s;
}

// ---------------------------------------------------------------------------
// Truncation (Sec. 2.1, Eqs. 10-11): each basis vector keeps at most N_d = M
// entries, the largest in magnitude.  The nonzero entries are ordered by |c|
// descending; the paper leaves exact ties open, and they go to the lower rank.
// The first min(M, nnz) are kept and returned by ascending rank.  M < 0 keeps
// all.  In/out may alias.  Returns the kept count.
//
// band != 0 switches on an extension that is not the paper's rule: after the
// first M, every further entry whose |c| is at least (1 - 2^-36) times the
// M-th |c| is kept as well (so partners that are equal in exact arithmetic are
// never split by a rounding difference), unless that adds more than
// ORC_TIE_SLACK entries, in which case exactly M are kept.
static const i64 ORC_TIE_SLACK = 256;

extern "C" i64 orc_topm_band(i64 nnz, const u64* rank, const double* amp, i64 M, u64* out_rank, double* out_amp,
                             int band) {
    std::vector<std::pair<u64, double>> e;
    for (i64 t = 0; t < nnz; ++t)
        if (amp[t] != 0.0) e.push_back({rank[t], amp[t]});
    if (M >= 0 && (i64)e.size() > M) {
        // a total order (ranks are unique), so any correct sort gives the same sequence
        auto by_mag = [](const std::pair<u64, double>& x, const std::pair<u64, double>& y) {
            double ax = std::fabs(x.second), ay = std::fabs(y.second);
            if (ax != ay) return ax > ay;
            return x.first < y.first;
        };
        if (g_threads > 1) __gnu_parallel::sort(e.begin(), e.end(), by_mag);
        else std::sort(e.begin(), e.end(), by_mag);
        i64 keep = M;
        if (band && M > 0) {
            const double thr = std::fabs(e[(size_t)M - 1].second) * (1.0 - 1.0 / 68719476736.0);  // 1 - 2^-36
            i64 k = M;
            while (k < (i64)e.size() && std::fabs(e[(size_t)k].second) >= thr) ++k;
            if (k - M <= ORC_TIE_SLACK) keep = k;
        }
        e.resize((size_t)keep);
    }
    std::sort(e.begin(), e.end());
    for (size_t t = 0; t < e.size(); ++t) { out_rank[t] = e[t].first; out_amp[t] = e[t].second; }
    return (i64)e.size();
}

extern "C" i64 orc_topm(i64 nnz, const u64* rank, const double* amp, i64 M, u64* out_rank, double* out_amp) {
    return orc_topm_band(nnz, rank, amp, M, out_rank, out_amp, 0);
}

// Eq. 11: divide by the 2-norm; the sum of squares runs in ascending rank.
extern "C" double orc_normalize(i64 nnz, double* amp) {
    double s = 0.0;
    for (i64 t = 0; t < nnz; ++t) s += amp[t] * amp[t];
    double nrm = std::sqrt(s);
    if (nrm > 0.0)
        for (i64 t = 0; t < nnz; ++t) amp[t] = amp[t] / nrm;
    return nrm;
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi eigen-decomposition of a symmetric m x m matrix (row-major,
// destroyed).  V receives the eigenvectors as columns, w the eigenvalues.
// One rotation per off-diagonal pair (p<q, row by row) per sweep, with the
// classical stable choice of the rotation angle; sweeps stop when the sum of
// squared off-diagonal elements is at most 1e-30 times the squared Frobenius
// norm of the diagonal, or after 64 sweeps.
extern "C" void orc_jacobi(int m, double* A, double* V, double* w) {
    for (int p = 0; p < m; ++p)
        for (int q = 0; q < m; ++q) V[p * m + q] = (p == q) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, dg = 0.0;
        for (int p = 0; p < m; ++p) {
            dg += A[p * m + p] * A[p * m + p];
            for (int q = p + 1; q < m; ++q) off += A[p * m + q] * A[p * m + q];
        }
        if (off <= 1e-30 * dg) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                double apq = A[p * m + q];
                if (apq == 0.0) continue;
                // Angle that zeroes A[p][q]: tan(phi) = t, the smaller root of
                // t^2 + 2 theta t - 1 = 0 with theta = (A_qq - A_pp) / (2 A_pq).
                double theta = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
                double t = 1.0 / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                if (theta < 0.0) t = -t;
                double c = 1.0 / std::sqrt(t * t + 1.0);
                double s = t * c;
                double tau = s / (1.0 + c);
                A[p * m + p] = A[p * m + p] - t * apq;
                A[q * m + q] = A[q * m + q] + t * apq;
                A[p * m + q] = 0.0;
                A[q * m + p] = 0.0;
                for (int r = 0; r < m; ++r) {
                    if (r == p || r == q) continue;
                    double arp = A[r * m + p], arq = A[r * m + q];
                    double nrp = arp - s * (arq + tau * arp);
                    double nrq = arq + s * (arp - tau * arq);
                    A[r * m + p] = nrp; A[p * m + r] = nrp;
                    A[r * m + q] = nrq; A[q * m + r] = nrq;
                }
                for (int r = 0; r < m; ++r) {
                    double vrp = V[r * m + p], vrq = V[r * m + q];
                    V[r * m + p] = vrp - s * (vrq + tau * vrp);
                    V[r * m + q] = vrq + s * (vrp - tau * vrq);
                }
            }
    }
    for (int p = 0; p < m; ++p) w[p] = A[p * m + p];
}

// Generalized problem T x = lambda S x (Sec. 2.1) for the lowest lambda, by
// canonical orthogonalisation: S = U s U^T; keep s_k > 1e-10 max(s);
// X = U_k s_k^(-1/2); diagonalise X^T T X; x = X y.  The sign of x is fixed
// so that its largest-magnitude component (lowest index on ties) is positive.
// Returns the number of kept directions (0 means failure).
extern "C" int orc_geneig(int m, const double* T, const double* Sm, double* lambda, double* x) {
    std::vector<double> A(Sm, Sm + m * m), U(m * m), s(m);
    orc_jacobi(m, A.data(), U.data(), s.data());
    double smax = 0.0;
    for (int k = 0; k < m; ++k) if (s[k] > smax) smax = s[k];
    std::vector<int> keep;
    for (int k = 0; k < m; ++k) if (s[k] > 1e-10 * smax) keep.push_back(k);
    int r = (int)keep.size();
    if (r == 0) return 0;
    std::vector<double> X(m * r);
    for (int i = 0; i < m; ++i)
        for (int c = 0; c < r; ++c) X[i * r + c] = U[i * m + keep[c]] / std::sqrt(s[keep[c]]);
    // Tp = X^T T X, formed as X^T (T X) with sums in ascending index order.
    std::vector<double> TX(m * r), Tp(r * r);
    for (int i = 0; i < m; ++i)
        for (int c = 0; c < r; ++c) {
            double acc = 0.0;
            for (int k = 0; k < m; ++k) acc += T[i * m + k] * X[k * r + c];
            TX[i * r + c] = acc;
        }
    for (int a = 0; a < r; ++a)
        for (int c = 0; c < r; ++c) {
            double acc = 0.0;
            for (int k = 0; k < m; ++k) acc += X[k * r + a] * TX[k * r + c];
            Tp[a * r + c] = acc;
        }
    // Symmetrise exactly before the eigensolve.
    for (int a = 0; a < r; ++a)
        for (int c = a + 1; c < r; ++c) {
            double v = 0.5 * (Tp[a * r + c] + Tp[c * r + a]);
            Tp[a * r + c] = v; Tp[c * r + a] = v;
        }
    std::vector<double> Y(r * r), lam(r);
    orc_jacobi(r, Tp.data(), Y.data(), lam.data());
    int best = 0;
    for (int k = 1; k < r; ++k) if (lam[k] < lam[best]) best = k;
    *lambda = lam[best];
    for (int i = 0; i < m; ++i) {
        double acc = 0.0;
        for (int c = 0; c < r; ++c) acc += X[i * r + c] * Y[c * r + best];
        x[i] = acc;
    }
    int imax = 0;
    for (int i = 1; i < m; ++i) if (std::fabs(x[i]) > std::fabs(x[imax])) imax = i;
    if (x[imax] < 0.0)
        for (int i = 0; i < m; ++i) x[i] = -x[i];
    return r;
}

// ---------------------------------------------------------------------------
// Sparse vectors as (ascending ranks, amplitudes).
struct SVec { std::vector<u64> r; std::vector<double> a; };

// <x|y> summed over supp(x) in ascending rank.
static double sdot(const SVec& x, const SVec& y) {
    double s = 0.0;
    size_t j = 0;
    for (size_t i = 0; i < x.r.size(); ++i) {
        while (j < y.r.size() && y.r[j] < x.r[i]) ++j;
        if (j < y.r.size() && y.r[j] == x.r[i]) s += x.a[i] * y.a[j];
    }
    return s;
}

static SVec sigma_full(const Space& S, const SVec& v, double eps_x = 0.0) {
    std::vector<Acc> run = sigma_merged(S, (i64)v.r.size(), v.r.data(), v.a.data(), eps_x);
    SVec y;
    for (const Acc& e : run)
        if (e.v != 0.0) { y.r.push_back(e.r); y.a.push_back(e.v); }
    return y;
}

static SVec topm_normalize(const SVec& u, i64 M, int band) {
    SVec w;
    w.r.resize(u.r.size()); w.a.resize(u.r.size());
    i64 k = orc_topm_band((i64)u.r.size(), u.r.data(), u.a.data(), M, w.r.data(), w.a.data(), band);
    w.r.resize(k); w.a.resize(k);
    orc_normalize(k, w.a.data());
    return w;
}

// u = (y - a x) - b z, entrywise over the union of supports (missing = 0),
// ranks ascending: a merge of the three rank-sorted lists.
static SVec lanczos_update(const SVec& y, double a, const SVec& x, double b, const SVec* z) {
    const u64 END = ~0ull;
    size_t iy = 0, ix = 0, iz = 0;
    const size_t nz = z ? z->r.size() : 0;
    SVec u;
    u.r.reserve(y.r.size() + x.r.size() + nz);
    u.a.reserve(y.r.size() + x.r.size() + nz);
    while (true) {
        const u64 ky = iy < y.r.size() ? y.r[iy] : END;
        const u64 kx = ix < x.r.size() ? x.r[ix] : END;
        const u64 kz = iz < nz ? z->r[iz] : END;
        const u64 k = std::min(ky, std::min(kx, kz));
        if (k == END) break;
        const double gy = (ky == k) ? y.a[iy++] : 0.0;
        const double gx = (kx == k) ? x.a[ix++] : 0.0;
        double val = gy - a * gx;
        if (z) {
            const double gz = (kz == k) ? z->a[iz++] : 0.0;
            val = val - b * gz;
        }
        if (val != 0.0) { u.r.push_back(k); u.a.push_back(val); }
    }
    return u;
}

// The SFCI iteration (Sec. 2.1).  A block holds N_L vectors w_0..w_{N_L-1}:
//   y = H w_j;  T_lj = T_jl = <w_l|y>,  S_lj = S_jl = <w_l|w_j>  for l <= j;
//   if j < N_L-1:  u = (y - T_jj w_j) - T_{j-1,j} w_{j-1}  (Eq. 10),
//                  w_{j+1} = truncate to M and normalise (Eq. 11);
// then solve T x = lambda S x, form Psi = sum_j x_j w_j (j ascending),
// truncate and normalise it into the next block's w_0 (restart).
// n_iter sigma applications are run (n_iter / N_L blocks).  energies[b]
// receives each block's lambda.  The final Psi (before truncation) is
// written to psi_* when psi_cap suffices; returns its size, or -1.
// y <- y - c x entrywise over the union of supports (missing = 0), each entry
// rounded as y_k - (c * x_k).
static SVec axpy_union(const SVec& y, double c, const SVec& x) {
    SVec out;
    size_t i = 0, j = 0;
    while (i < y.r.size() || j < x.r.size()) {
        if (j == x.r.size() || (i < y.r.size() && y.r[i] < x.r[j])) {
            out.r.push_back(y.r[i]); out.a.push_back(y.a[i]); ++i;
        } else if (i == y.r.size() || x.r[j] < y.r[i]) {
            const double prod = c * x.a[j];
            out.r.push_back(x.r[j]); out.a.push_back(0.0 - prod); ++j;
        } else {
            const double prod = c * x.a[j];
            out.r.push_back(y.r[i]); out.a.push_back(y.a[i] - prod); ++i; ++j;
        }
    }
    return out;
}

// Projection onto the complement of the previously found eigenvectors
// (Sec. 4: excited states by projecting the found eigenvectors out of the
// effective Hamiltonian): P y = y - sum_i Psi_i <Psi_i|y> / <Psi_i|Psi_i>,
// the roots taken in order.
struct Roots {
    std::vector<SVec> v;    // Psi_i
    std::vector<SVec> hv;   // H Psi_i
    std::vector<double> q;  // <Psi_i|Psi_i>
};

static SVec project(const Roots& R, SVec y) {
    for (size_t i = 0; i < R.v.size(); ++i) {
        const double d = sdot(R.v[i], y) / R.q[i];
        y = axpy_union(y, d, R.v[i]);
    }
    return y;
}

// eps > 0: the screening of Sec. 3 -- entries of the merged H w_j with
// amplitude below eps are not taken into v, so T, the Eq. 10 update and the
// candidates all see the screened vector.
// n_roots > 0: the iteration runs on P H P (P as above) from the projected,
// truncated start vector, for the next excited state: every sigma becomes
//   y = screen(H w) - sum_i c_i H Psi_i  (c_i = <Psi_i|w>/<Psi_i|Psi_i>),  then y = P y,
// and the block-end Psi is projected before its truncation.  Root i is
// (root_r, root_a)[root_off[i] .. root_off[i+1]), ranks ascending.
// band: the truncation extension of orc_topm_band (0 = the paper's rule).
// conv_eps > 0: the halting test of Sec. 2.1 -- after block n >= 1 the run
// stops when E(n-1) - E(n) < conv_eps (the signed difference, as the paper
// writes it); *blocks_run (may be NULL) receives the number of blocks run and
// energies[] beyond it are left untouched.  basis_nnz (may be NULL, n_iter
// entries) receives the entry count of every basis vector w_j, block after
// block.  eps_x > 0: every H w_j with the excitation screen of sigma_merged
// (the roots' H Psi_i are not screened).
extern "C" i64 orc_lanczos_ex(int n, int na, int nb, const double* h, const double* g, i64 nnz0, const u64* r0,
                              const double* a0, i64 M, int nL, int n_iter, double* energies, double* Tout,
                              double* Sout, u64* psi_rank, double* psi_amp, i64 psi_cap, double eps,
                              int n_roots, const i64* root_off, const u64* root_r, const double* root_a, int band,
                              double conv_eps, int* blocks_run, i64* basis_nnz, double eps_x) {
    Space S = make_space(n, na, nb, h, g);
    Roots R;
    for (int i = 0; i < n_roots; ++i) {
        SVec x;
        x.r.assign(root_r + root_off[i], root_r + root_off[i + 1]);
        x.a.assign(root_a + root_off[i], root_a + root_off[i + 1]);
        double q = 0.0;
        for (double v : x.a) q += v * v;
        R.hv.push_back(sigma_full(S, x));
        R.q.push_back(q);
        R.v.push_back(x);
    }
    SVec w0;
    w0.r.assign(r0, r0 + nnz0);
    w0.a.assign(a0, a0 + nnz0);
    if (n_roots > 0) w0 = topm_normalize(project(R, w0), M, band);
    else orc_normalize((i64)w0.a.size(), w0.a.data());
    int nblocks = n_iter / nL;
    SVec psi;
    if (blocks_run) *blocks_run = 0;
    for (int blk = 0; blk < nblocks; ++blk) {
        std::vector<SVec> w(nL);
        w[0] = w0;
        std::vector<double> T(nL * nL, 0.0), Sm(nL * nL, 0.0);
        for (int j = 0; j < nL; ++j) {
            if (basis_nnz) basis_nnz[(size_t)blk * nL + j] = (i64)w[j].r.size();
            SVec y = sigma_full(S, w[j], eps_x);
            if (eps > 0.0) {
                SVec ys;
                for (size_t t = 0; t < y.r.size(); ++t)
                    if (!(std::fabs(y.a[t]) < eps)) { ys.r.push_back(y.r[t]); ys.a.push_back(y.a[t]); }
                y = ys;
            }
            if (n_roots > 0) {
                // H P w = H w - sum_i c_i H Psi_i, then P
                for (int i = 0; i < n_roots; ++i) {
                    const double c = sdot(R.v[i], w[j]) / R.q[i];
                    y = axpy_union(y, c, R.hv[i]);
                }
                y = project(R, y);
            }
            for (int l = 0; l <= j; ++l) {
                double t = sdot(w[l], y);
                T[l * nL + j] = t; T[j * nL + l] = t;
                double s = sdot(w[l], w[j]);
                Sm[l * nL + j] = s; Sm[j * nL + l] = s;
            }
            if (j + 1 < nL) {
                SVec u = lanczos_update(y, T[j * nL + j], w[j], j >= 1 ? T[(j - 1) * nL + j] : 0.0,
                                        j >= 1 ? &w[j - 1] : nullptr);
                w[j + 1] = topm_normalize(u, M, band);
            }
        }
        if (Tout) std::memcpy(Tout + (size_t)blk * nL * nL, T.data(), sizeof(double) * nL * nL);
        if (Sout) std::memcpy(Sout + (size_t)blk * nL * nL, Sm.data(), sizeof(double) * nL * nL);
        double lam;
        std::vector<double> x(nL);
        if (orc_geneig(nL, T.data(), Sm.data(), &lam, x.data()) == 0) return -1;
        energies[blk] = lam;
        // Psi = sum_j x_j w_j, added in j order on the union of supports.
        std::vector<u64> all;
        for (int j = 0; j < nL; ++j) all.insert(all.end(), w[j].r.begin(), w[j].r.end());
        std::sort(all.begin(), all.end());
        all.erase(std::unique(all.begin(), all.end()), all.end());
        std::vector<double> acc(all.size(), 0.0);
        for (int j = 0; j < nL; ++j)
            for (size_t t = 0; t < w[j].r.size(); ++t) {
                size_t pos = std::lower_bound(all.begin(), all.end(), w[j].r[t]) - all.begin();
                acc[pos] = acc[pos] + x[j] * w[j].a[t];
            }
        psi.r.clear(); psi.a.clear();
        for (size_t t = 0; t < all.size(); ++t)
            if (acc[t] != 0.0) { psi.r.push_back(all[t]); psi.a.push_back(acc[t]); }
        if (n_roots > 0) {
            SVec pp = project(R, psi), nz;
            for (size_t t = 0; t < pp.r.size(); ++t)
                if (pp.a[t] != 0.0) { nz.r.push_back(pp.r[t]); nz.a.push_back(pp.a[t]); }
            psi = nz;
        }
        w0 = topm_normalize(psi, M, band);
        if (blocks_run) *blocks_run = blk + 1;
        if (conv_eps > 0.0 && blk >= 1 && energies[blk - 1] - energies[blk] < conv_eps) break;
    }
    if ((i64)psi.r.size() <= psi_cap && psi_rank && psi_amp) {
        std::copy(psi.r.begin(), psi.r.end(), psi_rank);
        std::copy(psi.a.begin(), psi.a.end(), psi_amp);
    }
    return (i64)psi.r.size();
}

extern "C" i64 orc_lanczos_roots(int n, int na, int nb, const double* h, const double* g, i64 nnz0, const u64* r0,
                                 const double* a0, i64 M, int nL, int n_iter, double* energies, double* Tout,
                                 double* Sout, u64* psi_rank, double* psi_amp, i64 psi_cap, double eps,
                                 int n_roots, const i64* root_off, const u64* root_r, const double* root_a) {
    return orc_lanczos_ex(n, na, nb, h, g, nnz0, r0, a0, M, nL, n_iter, energies, Tout, Sout, psi_rank, psi_amp,
                          psi_cap, eps, n_roots, root_off, root_r, root_a, 0, 0.0, nullptr, nullptr, 0.0);
}

extern "C" i64 orc_lanczos(int n, int na, int nb, const double* h, const double* g, i64 nnz0, const u64* r0,
                           const double* a0, i64 M, int nL, int n_iter, double* energies, double* Tout,
                           double* Sout, u64* psi_rank, double* psi_amp, i64 psi_cap, double eps) {
    return orc_lanczos_ex(n, na, nb, h, g, nnz0, r0, a0, M, nL, n_iter, energies, Tout, Sout, psi_rank, psi_amp,
                          psi_cap, eps, 0, nullptr, nullptr, nullptr, 0, 0.0, nullptr, nullptr, 0.0);
}

// ---------------------------------------------------------------------------
// Backward of sigma = H(h, g) v for a cotangent sbar (an extension,
// not in the paper).  With L = sbar^T H v:
//   vbar_i = sum_k H_ki sbar_k                 for i in supp(v)
//   gamma_pq = sum_ki sbar_k v_i <k| sum_s a+_ps a_qs |i>
//   Gamma_pqrs = sum_ki sbar_k v_i <k| sum_st a+_ps a+_rt a_st a_qs |i>
// dh = (gamma + gamma^T) / 2 and dg = the average of Gamma/2 over the eight
// index permutations of (pq|rs): the gradients along symmetric perturbations.
// All by explicit operator application (independent of Slater-Condon).
static double lookup(i64 nnz, const u64* r, const double* a, u64 k) {
    const u64* it = std::lower_bound(r, r + nnz, k);
    return (it != r + nnz && *it == k) ? a[it - r] : 0.0;
}

static void sym8(int n, const double* G, double* out) {
    auto I = [n](int p, int q, int r, int s) { return ((size_t)(p * n + q) * n + r) * n + s; };
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            for (int r = 0; r < n; ++r)
                for (int s = 0; s < n; ++s) {
                    double v = G[I(p, q, r, s)] + G[I(q, p, r, s)] + G[I(p, q, s, r)] + G[I(q, p, s, r)] +
                               G[I(r, s, p, q)] + G[I(s, r, p, q)] + G[I(r, s, q, p)] + G[I(s, r, q, p)];
                    out[I(p, q, r, s)] = v / 8.0;
                }
}

// Second-order Epstein-Nesbet correction of a variational vector Psi, the
// perturbative correction the paper names for future work (its comparison
// with ASCI in the results).  Standard partitioning, H0 = diagonal of H:
//   E0 = <Psi|H|Psi> / <Psi|Psi>,
//   E2 = [ sum over k outside supp(Psi) of (H Psi)_k^2 / (E0 - H_kk) ] / <Psi|Psi>.
// H Psi comes from the merge of orc_sigma; every sum runs over ascending rank
// (E0's numerator over the entries of H Psi inside supp(Psi)); H_kk is the
// diagonal element above.  *n_ext = number of external determinants with
// (H Psi)_k != 0.  Returns 0, or -1 on bad input.
extern "C" int orc_pt2(int n, int na, int nb, const double* h, const double* g, i64 nnz, const u64* rank,
                       const double* amp, double* e0, double* e2, u64* n_ext) {
    Space S = make_space(n, na, nb, h, g);
    for (i64 t = 0; t < nnz; ++t) {
        if (rank[t] >= S.Ndet) return -1;
        if (t > 0 && rank[t] <= rank[t - 1]) return -1;
    }
    std::vector<Acc> y = sigma_merged(S, nnz, rank, amp);
    double num = 0.0, den = 0.0;
    for (i64 t = 0; t < nnz; ++t) den += amp[t] * amp[t];
    // <Psi|H Psi>: walk both rank-sorted lists together
    i64 t = 0;
    for (const Acc& e : y) {
        while (t < nnz && rank[t] < e.r) ++t;
        if (t < nnz && rank[t] == e.r) num += amp[t] * e.v;
    }
    const double E0 = num / den;
    std::vector<int> oa, va, ob, vb;
    double s = 0.0;
    u64 cnt = 0;
    t = 0;
    for (const Acc& e : y) {
        while (t < nnz && rank[t] < e.r) ++t;
        if ((t < nnz && rank[t] == e.r) || e.v == 0.0) continue;
        occ_virt(orc_str_unrank(e.r / S.Nb, na), n, oa, va);
        occ_virt(orc_str_unrank(e.r % S.Nb, nb), n, ob, vb);
        const double hkk = diag_element(S, oa, ob);
        s += (e.v * e.v) / (E0 - hkk);
        ++cnt;
    }
    *e0 = E0;
    *e2 = s / den;
    *n_ext = cnt;
    return 0;
}

extern "C" int orc_backward_explicit(int n, int na, int nb, const double* h, const double* g, i64 nnz_v,
                                     const u64* rv, const double* av, i64 nnz_s, const u64* rs, const double* as,
                                     double* vbar, double* dh, double* dg) {
    Space S = make_space(n, na, nb, h, g);
    std::vector<double> gam(n * n, 0.0), Gam((size_t)n * n * n * n, 0.0);
    for (i64 t = 0; t < nnz_v; ++t) {
        u64 D0 = S.so_of_rank(rv[t]);
        double vi = av[t];
        if (vbar) {
            double acc = 0.0;
            apply_H_explicit(S, D0, [&](u64 D, double c) { acc += c * lookup(nnz_s, rs, as, S.rank_so(D)); });
            vbar[t] = acc;
        }
        for (int sg = 0; sg < 2; ++sg)
            for (int p = 0; p < n; ++p)
                for (int q = 0; q < n; ++q) {
                    u64 D = D0; int sign = 1;
                    if (!op_annihilate(D, q + sg * n, sign)) continue;
                    if (!op_create(D, p + sg * n, sign)) continue;
                    double sk = lookup(nnz_s, rs, as, S.rank_so(D));
                    if (sk != 0.0) gam[p * n + q] += sk * vi * (double)sign;
                }
        for (int sg = 0; sg < 2; ++sg)
            for (int tg = 0; tg < 2; ++tg)
                for (int p = 0; p < n; ++p)
                    for (int q = 0; q < n; ++q)
                        for (int r = 0; r < n; ++r)
                            for (int s = 0; s < n; ++s) {
                                u64 D = D0; int sign = 1;
                                if (!op_annihilate(D, q + sg * n, sign)) continue;
                                if (!op_annihilate(D, s + tg * n, sign)) continue;
                                if (!op_create(D, r + tg * n, sign)) continue;
                                if (!op_create(D, p + sg * n, sign)) continue;
                                double sk = lookup(nnz_s, rs, as, S.rank_so(D));
                                if (sk != 0.0)
                                    Gam[((size_t)(p * n + q) * n + r) * n + s] += sk * vi * (double)sign;
                            }
    }
    if (dh)
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) dh[p * n + q] = 0.5 * (gam[p * n + q] + gam[q * n + p]);
    if (dg) {
        std::vector<double> half(Gam.size());
        for (size_t t = 0; t < Gam.size(); ++t) half[t] = 0.5 * Gam[t];
        sym8(n, half.data(), dg);
    }
    return 0;
}

// The same backward from the Slater-Condon generation (faster; checked
// against orc_backward_explicit on tiny spaces).  Each generated term adds
// sbar_k v_i times the coefficient of every integral in its element formula
// to a raw gradient, which is then symmetrised as above.
extern "C" int orc_backward_sc(int n, int na, int nb, const double* h, const double* g, i64 nnz_v, const u64* rv,
                               const double* av, i64 nnz_s, const u64* rs, const double* as, double* vbar,
                               double* dh, double* dg) {
    Space S = make_space(n, na, nb, h, g);
    std::vector<double> Rh(n * n, 0.0), Rg((size_t)n * n * n * n, 0.0);
    auto G = [n](int p, int q, int r, int s) { return ((size_t)(p * n + q) * n + r) * n + s; };
    for (i64 t = 0; t < nnz_v; ++t) {
        u64 A = orc_str_unrank(rv[t] / S.Nb, na), B = orc_str_unrank(rv[t] % S.Nb, nb);
        double vi = av[t];
        std::vector<int> oa, va, ob, vb;
        occ_virt(A, n, oa, va);
        occ_virt(B, n, ob, vb);
        if (vbar) {
            double acc = 0.0;
            sc_terms(S, A, B, [&](u64 A2, u64 B2, double e) {
                acc += e * lookup(nnz_s, rs, as, orc_str_rank(A2) * S.Nb + orc_str_rank(B2));
            });
            vbar[t] = acc;
        }
        // diagonal
        double w = lookup(nnz_s, rs, as, rv[t]) * vi;
        if (w != 0.0) {
            for (int p : oa) Rh[p * n + p] += w;
            for (int p : ob) Rh[p * n + p] += w;
            for (int sp = 0; sp < 2; ++sp) {
                const std::vector<int>& o = sp == 0 ? oa : ob;
                for (size_t x = 0; x < o.size(); ++x)
                    for (size_t y = x + 1; y < o.size(); ++y) {
                        Rg[G(o[x], o[x], o[y], o[y])] += w;
                        Rg[G(o[x], o[y], o[y], o[x])] -= w;
                    }
            }
            for (int p : oa)
                for (int q : ob) Rg[G(p, p, q, q)] += w;
        }
        // singles
        for (int sp = 0; sp < 2; ++sp) {
            u64 Str = sp == 0 ? A : B;
            const std::vector<int>& os = sp == 0 ? oa : ob;
            const std::vector<int>& vs = sp == 0 ? va : vb;
            const std::vector<int>& oo = sp == 0 ? ob : oa;
            for (int i : os)
                for (int a : vs) {
                    u64 T = Str ^ (1ull << i) ^ (1ull << a);
                    u64 tr = sp == 0 ? orc_str_rank(T) * S.Nb + orc_str_rank(B) : orc_str_rank(A) * S.Nb + orc_str_rank(T);
                    double ws = lookup(nnz_s, rs, as, tr) * vi * (double)single_sign(Str, i, a);
                    if (ws == 0.0) continue;
                    Rh[i * n + a] += ws;
                    for (int k : os) {
                        if (k == i) continue;
                        Rg[G(i, a, k, k)] += ws;
                        Rg[G(i, k, k, a)] -= ws;
                    }
                    for (int k : oo) Rg[G(i, a, k, k)] += ws;
                }
        }
        // same-spin doubles
        for (int sp = 0; sp < 2; ++sp) {
            u64 Str = sp == 0 ? A : B;
            const std::vector<int>& oc = sp == 0 ? oa : ob;
            const std::vector<int>& vi_ = sp == 0 ? va : vb;
            for (size_t x = 0; x < oc.size(); ++x)
                for (size_t y = x + 1; y < oc.size(); ++y)
                    for (size_t u = 0; u < vi_.size(); ++u)
                        for (size_t z = u + 1; z < vi_.size(); ++z) {
                            int i = oc[x], j = oc[y], a = vi_[u], b = vi_[z];
                            u64 mid = Str ^ (1ull << i) ^ (1ull << a);
                            u64 T = mid ^ (1ull << j) ^ (1ull << b);
                            u64 tr = sp == 0 ? orc_str_rank(T) * S.Nb + orc_str_rank(B)
                                             : orc_str_rank(A) * S.Nb + orc_str_rank(T);
                            double wd = lookup(nnz_s, rs, as, tr) * vi *
                                        (double)(single_sign(Str, i, a) * single_sign(mid, j, b));
                            if (wd == 0.0) continue;
                            Rg[G(i, a, j, b)] += wd;
                            Rg[G(i, b, j, a)] -= wd;
                        }
        }
        // alpha-beta doubles
        for (int i : oa)
            for (int a : va) {
                u64 A2 = A ^ (1ull << i) ^ (1ull << a);
                u64 ra = orc_str_rank(A2) * S.Nb;
                int sa = single_sign(A, i, a);
                for (int j : ob)
                    for (int b : vb) {
                        u64 B2 = B ^ (1ull << j) ^ (1ull << b);
                        double wd = lookup(nnz_s, rs, as, ra + orc_str_rank(B2)) * vi *
                                    (double)(sa * single_sign(B, j, b));
                        if (wd != 0.0) Rg[G(i, a, j, b)] += wd;
                    }
            }
    }
    if (dh)
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) dh[p * n + q] = 0.5 * (Rh[p * n + q] + Rh[q * n + p]);
    if (dg) sym8(n, Rg.data(), dg);
    return 0;
}

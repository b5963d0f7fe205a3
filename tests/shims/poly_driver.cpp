// poly_driver.cpp -- the jump-ahead planner's GF(2)[x] routines
// (mtgp_poly.cpp) against bit-by-bit schoolbook arithmetic, as a standalone
// program that the CPU tests build with the address and undefined-behaviour
// sanitizers.  Exit status 0 when every check holds.
#include <cstdio>
#include <random>
#include <vector>

#include "mtgp_poly.hpp"

using mtgp::poly::Poly;
using Bits = std::vector<uint8_t>;  // one coefficient per byte, index = power

static int g_fail = 0;
#define CHECK(cond, what)                                                     \
    do {                                                                      \
        if (!(cond)) {                                                        \
            std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, what); \
            ++g_fail;                                                         \
        }                                                                     \
    } while (0)

static Bits bits_of(const Poly &a) {
    Bits b(a.size() * 64, 0);
    for (size_t i = 0; i < b.size(); ++i) b[i] = (uint8_t)((a[i / 64] >> (i % 64)) & 1u);
    while (!b.empty() && !b.back()) b.pop_back();
    return b;
}
static Poly poly_of(const Bits &b) {
    Poly a((b.size() + 63) / 64, 0);
    for (size_t i = 0; i < b.size(); ++i)
        if (b[i]) a[i / 64] |= 1ull << (i % 64);
    mtgp::poly::trim(a);
    return a;
}
static void norm(Bits &b) {
    while (!b.empty() && !b.back()) b.pop_back();
}
static Bits nmul(const Bits &a, const Bits &b) {
    if (a.empty() || b.empty()) return {};
    Bits r(a.size() + b.size() - 1, 0);
    for (size_t i = 0; i < a.size(); ++i)
        if (a[i])
            for (size_t j = 0; j < b.size(); ++j) r[i + j] ^= b[j];
    norm(r);
    return r;
}
// remainder and quotient by long division, highest power first
static Bits ndivmod(Bits a, const Bits &p, Bits *q) {
    norm(a);
    const size_t dp = p.size() - 1;
    if (q) q->assign(a.size() >= p.size() ? a.size() - dp : 0, 0);
    for (size_t k = a.size(); k-- > dp;) {
        if (!a[k]) continue;
        if (q) (*q)[k - dp] = 1;
        for (size_t j = 0; j <= dp; ++j) a[k - dp + j] ^= p[j];
    }
    norm(a);
    if (q) norm(*q);
    return a;
}
static Bits rand_bits(std::mt19937_64 &rng, size_t n, bool top) {
    Bits b(n, 0);
    for (auto &x : b) x = (uint8_t)(rng() & 1u);
    if (top && n) b[n - 1] = 1;
    norm(b);
    return b;
}
static bool same(const Poly &a, const Bits &b) { return bits_of(a) == b; }

static void arithmetic(int d, std::mt19937_64 &rng) {
    namespace P = mtgp::poly;
    Bits p = rand_bits(rng, (size_t)d + 1, true);
    p[0] = 1;
    const Poly pp = poly_of(p);
    CHECK(P::degree(pp) == d, "degree");
    const P::Modulus m(pp);
    for (int trial = 0; trial < 3; ++trial) {
        const Bits a = rand_bits(rng, (size_t)(2 * d + 7), false);
        const Bits b = rand_bits(rng, (size_t)(d + 3), false);
        const Poly A = poly_of(a), B = poly_of(b);
        CHECK(same(P::mul(A, B), nmul(a, b)), "mul");
        CHECK(same(P::square(A), nmul(a, a)), "square");
        Bits x77(78, 0);
        x77[77] = 1;
        CHECK(same(P::shl(A, 77), nmul(a, x77)), "shl");
        Bits q;
        const Bits r = ndivmod(a, p, &q);
        CHECK(same(P::mod(A, pp), r), "mod");
        CHECK(same(P::divq(A, pp), q), "divq");
        CHECK(same(m.reduce(A), r), "Barrett reduce below 2d");
        const Bits big = rand_bits(rng, (size_t)(3 * d + 5), false);  // beyond Barrett's range
        CHECK(same(m.reduce(poly_of(big)), ndivmod(big, p, nullptr)), "reduce above 2d");
        const Bits ra = ndivmod(a, p, nullptr), rb = ndivmod(b, p, nullptr);
        CHECK(same(m.mulmod(poly_of(ra), poly_of(rb)), ndivmod(nmul(ra, rb), p, nullptr)),
              "mulmod");
        CHECK(same(m.sqrmod(poly_of(ra)), ndivmod(nmul(ra, ra), p, nullptr)), "sqrmod");
    }
    // x^e mod p by schoolbook square-and-multiply, most significant bit first
    const uint64_t du = (uint64_t)d;
    const std::vector<uint64_t> exps = {0, 1, du - 1, du, du + 1, 2 * du + 3, 12345,
                                        (1ull << 20) - 1, 1ull << 33};
    for (uint64_t e : exps) {
        Bits r{1};
        const Bits x{0, 1};
        for (int k = 63; k >= 0; --k) {
            r = ndivmod(nmul(r, r), p, nullptr);
            if ((e >> k) & 1u) r = ndivmod(nmul(r, x), p, nullptr);
        }
        CHECK(same(m.powx(e), r), "powx");
    }
}

static void gcd_lcm(std::mt19937_64 &rng) {
    namespace P = mtgp::poly;
    for (int trial = 0; trial < 20; ++trial) {
        const Bits f = rand_bits(rng, 1 + rng() % 90, true), g = rand_bits(rng, 1 + rng() % 90, true),
                   h = rand_bits(rng, 1 + rng() % 90, true);
        const Bits a = nmul(f, g), b = nmul(g, h);
        const Poly A = poly_of(a), B = poly_of(b);
        const Poly G = P::gcd(A, B), L = P::lcm(A, B);
        const Bits gb = bits_of(G), lb = bits_of(L);
        CHECK(!gb.empty() && gb.back() == 1, "gcd nonzero");
        CHECK(ndivmod(a, gb, nullptr).empty() && ndivmod(b, gb, nullptr).empty(),
              "gcd divides both");
        CHECK(ndivmod(gb, g, nullptr).empty(), "the common factor divides the gcd");
        CHECK(ndivmod(lb, a, nullptr).empty() && ndivmod(lb, b, nullptr).empty(),
              "both divide the lcm");
        CHECK(nmul(gb, lb) == nmul(a, b), "gcd * lcm = a * b");
    }
}

static void massey(std::mt19937_64 &rng) {
    namespace P = mtgp::poly;
    // a sequence of the trinomial recurrence s_t = s_{t-89} ^ s_{t-38}
    // (x^89 + x^38 + 1 is primitive): linear complexity 89 from a random start
    for (int n : {200, 1000, 5000}) {
        std::vector<uint8_t> s;
        for (int i = 0; i < 89; ++i) s.push_back((uint8_t)(rng() & 1u));
        while ((int)s.size() < n) s.push_back(s[s.size() - 89] ^ s[s.size() - 38]);
        Poly ann;
        const int L = P::berlekamp_massey(s.data(), n, &ann);
        CHECK(L == 89, "trinomial sequence complexity");
        const Bits a = bits_of(ann);
        Bits expect(90, 0);
        expect[0] = expect[51] = expect[89] = 1;  // x^89 + x^51 + 1 reads s forwards
        // n >= 2L: the shortest recurrence is unique
        CHECK(a == expect, "annihilator of the trinomial sequence");
        for (int t = 0; t + L < n; ++t) {
            uint8_t acc = 0;
            for (int j = 0; j <= L; ++j)
                if (j < (int)a.size() && a[j]) acc ^= s[(size_t)(t + j)];
            if (acc) {
                CHECK(false, "annihilator fails on the sequence");
                break;
            }
        }
    }
    // random bits: the complexity is about n/2, and the result annihilates them
    for (int n : {1, 2, 64, 333, 2000}) {
        std::vector<uint8_t> s((size_t)n);
        for (auto &x : s) x = (uint8_t)(rng() & 1u);
        Poly ann;
        const int L = P::berlekamp_massey(s.data(), n, &ann);
        const Bits a = bits_of(ann);
        CHECK(L >= 0 && L <= n && (int)a.size() <= L + 1, "complexity range");
        for (int t = 0; t + L < n; ++t) {
            uint8_t acc = 0;
            for (int j = 0; j < (int)a.size(); ++j)
                if (a[j]) acc ^= s[(size_t)(t + j)];
            if (acc) {
                CHECK(false, "annihilator fails on random bits");
                break;
            }
        }
    }
    // the all-zero sequence has complexity 0
    std::vector<uint8_t> z(50, 0);
    Poly ann;
    CHECK(P::berlekamp_massey(z.data(), 50, &ann) == 0, "zero sequence");
}

int main() {
    std::mt19937_64 rng(20150130);
    for (int d : {1, 2, 5, 63, 64, 65, 127, 200, 1000, 3217}) arithmetic(d, rng);
    gcd_lcm(rng);
    massey(rng);
    std::printf("poly checks: %d failed\n", g_fail);
    return g_fail == 0 ? 0 : 1;
}

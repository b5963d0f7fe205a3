// mtgp_poly.cpp -- GF(2)[x] arithmetic for jump-ahead planning (host).
// Compiled by the host compiler with the carry-less multiply extension.
#include "mtgp_poly.hpp"

#include <emmintrin.h>
#include <wmmintrin.h>

#include <algorithm>
#include <cstring>

namespace mtgp {
namespace poly {

static inline void clmul(uint64_t a, uint64_t b, uint64_t &lo, uint64_t &hi) {
    const __m128i r = _mm_clmulepi64_si128(_mm_cvtsi64_si128((long long)a),
                                           _mm_cvtsi64_si128((long long)b), 0x00);
    lo = (uint64_t)_mm_cvtsi128_si64(r);
    hi = (uint64_t)_mm_cvtsi128_si64(_mm_unpackhi_epi64(r, r));
}

int degree(const Poly &a) {
    for (size_t w = a.size(); w-- > 0;)
        if (a[w]) return (int)(w * 64 + 63 - __builtin_clzll(a[w]));
    return -1;
}

void trim(Poly &a) {
    while (!a.empty() && a.back() == 0) a.pop_back();
}

static inline bool bit(const Poly &a, int i) {
    const size_t w = (size_t)i >> 6;
    return w < a.size() && ((a[w] >> (i & 63)) & 1u);
}

// r[0 .. 2n) ^= a[0 .. n) * b[0 .. n), schoolbook.
static void mul_base(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n) {
    for (size_t i = 0; i < n; ++i) {
        if (!a[i]) continue;
        for (size_t j = 0; j < n; ++j) {
            uint64_t lo, hi;
            clmul(a[i], b[j], lo, hi);
            r[i + j] ^= lo;
            r[i + j + 1] ^= hi;
        }
    }
}

// r[0 .. 2n) = a * b for n-word operands (n = base * 2^k, base < 32),
// Karatsuba: a = a0 + x^h a1, b likewise,
// a b = a0 b0 + x^h ((a0 + a1)(b0 + b1) + a0 b0 + a1 b1) + x^2h a1 b1.
// tmp holds 4n words of scratch.
static void mul_kara(uint64_t *r, const uint64_t *a, const uint64_t *b, size_t n, uint64_t *tmp) {
    if (n < 32) {
        std::memset(r, 0, 2 * n * 8);
        mul_base(r, a, b, n);
        return;
    }
    const size_t h = n / 2;
    uint64_t *sa = tmp, *sb = tmp + h, *mid = tmp + 2 * h, *rest = tmp + 4 * h;
    mul_kara(r, a, b, h, rest);               // a0 b0 -> r[0, n)
    mul_kara(r + n, a + h, b + h, h, rest);   // a1 b1 -> r[n, 2n)
    for (size_t i = 0; i < h; ++i) {
        sa[i] = a[i] ^ a[h + i];
        sb[i] = b[i] ^ b[h + i];
    }
    mul_kara(mid, sa, sb, h, rest);           // (a0+a1)(b0+b1) -> mid[0, n)
    for (size_t i = 0; i < n; ++i) mid[i] ^= r[i] ^ r[n + i];
    for (size_t i = 0; i < n; ++i) r[h + i] ^= mid[i];
}

Poly mul(const Poly &a, const Poly &b) {
    if (a.empty() || b.empty()) return {};
    const size_t m = std::max(a.size(), b.size());
    if (m < 32 || std::min(a.size(), b.size()) * 2 < m) {
        Poly r(a.size() + b.size(), 0);
        for (size_t i = 0; i < a.size(); ++i) {
            if (!a[i]) continue;
            for (size_t j = 0; j < b.size(); ++j) {
                uint64_t lo, hi;
                clmul(a[i], b[j], lo, hi);
                r[i + j] ^= lo;
                r[i + j + 1] ^= hi;
            }
        }
        trim(r);
        return r;
    }
    int k = 0;
    while (((m + ((size_t)1 << k) - 1) >> k) >= 32) ++k;
    const size_t n = ((m + ((size_t)1 << k) - 1) >> k) << k;  // base * 2^k >= m
    std::vector<uint64_t> A(n, 0), B(n, 0), R(2 * n, 0), tmp(8 * n, 0);
    std::memcpy(A.data(), a.data(), a.size() * 8);
    std::memcpy(B.data(), b.data(), b.size() * 8);
    mul_kara(R.data(), A.data(), B.data(), n, tmp.data());
    R.resize(a.size() + b.size());
    trim(R);
    return R;
}

Poly square(const Poly &a) {
    Poly r(a.size() * 2, 0);
    for (size_t i = 0; i < a.size(); ++i) clmul(a[i], a[i], r[2 * i], r[2 * i + 1]);
    trim(r);
    return r;
}

Poly shl(const Poly &a, int n) {
    if (a.empty()) return {};
    const int q = n >> 6, s = n & 63;
    Poly r(a.size() + (size_t)q + 1, 0);
    for (size_t i = 0; i < a.size(); ++i) {
        r[i + q] ^= a[i] << s;
        if (s) r[i + q + 1] ^= a[i] >> (64 - s);
    }
    trim(r);
    return r;
}

// r ^= p * x^sh, with p of n words
static void xor_shifted(uint64_t *r, size_t rn, const uint64_t *p, size_t pn, int sh) {
    const size_t q = (size_t)sh >> 6;
    const int s = sh & 63;
    for (size_t i = 0; i < pn; ++i) {
        if (i + q < rn) r[i + q] ^= p[i] << s;
        if (s && i + q + 1 < rn) r[i + q + 1] ^= p[i] >> (64 - s);
    }
}

static Poly divmod(const Poly &a, const Poly &p, Poly *quot) {
    const int dp = degree(p);
    Poly r = a;
    int dr = degree(r);
    if (quot) quot->assign(dr >= dp ? (size_t)((dr - dp) / 64 + 1) : 0, 0);
    while (dr >= dp) {
        const int sh = dr - dp;
        xor_shifted(r.data(), r.size(), p.data(), p.size(), sh);
        if (quot) (*quot)[(size_t)sh >> 6] |= 1ull << (sh & 63);
        dr = degree(r);
    }
    trim(r);
    if (quot) trim(*quot);
    return r;
}

Poly mod(const Poly &a, const Poly &p) { return divmod(a, p, nullptr); }

Poly divq(const Poly &a, const Poly &p) {
    Poly q;
    divmod(a, p, &q);
    return q;
}

Poly gcd(Poly a, Poly b) {
    trim(a);
    trim(b);
    while (!b.empty()) {
        Poly r = mod(a, b);
        a = std::move(b);
        b = std::move(r);
    }
    return a;
}

Poly lcm(const Poly &a, const Poly &b) {
    Poly g = gcd(a, b);
    return mul(a, divq(b, g));
}

Modulus::Modulus(const Poly &p_) : p(p_) {
    trim(p);
    d = degree(p);
    Poly x2d((size_t)(2 * d) / 64 + 1, 0);
    x2d[(size_t)(2 * d) >> 6] = 1ull << ((2 * d) & 63);
    mu = divq(x2d, p);
}

static Poly shr(const Poly &a, int n) {
    const size_t q = (size_t)n >> 6;
    const int s = n & 63;
    if (q >= a.size()) return {};
    Poly r(a.size() - q, 0);
    for (size_t i = 0; i < r.size(); ++i) {
        r[i] = a[i + q] >> s;
        if (s && i + q + 1 < a.size()) r[i] |= a[i + q + 1] << (64 - s);
    }
    trim(r);
    return r;
}

Poly Modulus::reduce(const Poly &a) const {
    const int da = degree(a);
    if (da < d) {
        Poly r = a;
        trim(r);
        return r;
    }
    if (da >= 2 * d) return mod(a, p);  // Barrett below is exact for deg < 2d
    const Poly q = shr(mul(shr(a, d), mu), d);
    Poly r = a;
    const Poly qp = mul(q, p);
    if (r.size() < qp.size()) r.resize(qp.size(), 0);
    for (size_t i = 0; i < qp.size(); ++i) r[i] ^= qp[i];
    trim(r);
    return r;
}

Poly Modulus::mulmod(const Poly &a, const Poly &b) const { return reduce(mul(a, b)); }
Poly Modulus::sqrmod(const Poly &a) const { return reduce(square(a)); }

Poly Modulus::powx(uint64_t e) const {
    Poly r{1};
    if (e == 0) return d > 0 ? r : Poly{};
    int top = 63 - __builtin_clzll(e);
    for (int b = top; b >= 0; --b) {
        r = sqrmod(r);
        if ((e >> b) & 1u) {
            r = shl(r, 1);
            if (degree(r) == d) {
                if (r.size() < p.size()) r.resize(p.size(), 0);
                for (size_t i = 0; i < p.size(); ++i) r[i] ^= p[i];
                trim(r);
            }
        }
    }
    return r;
}

int berlekamp_massey(const uint8_t *bits, int n, Poly *annihilator) {
    // C: connection polynomial, B: previous C; bit i = coefficient of x^i.
    const size_t nw = (size_t)n / 64 + 2;
    Poly C(nw, 0), B(nw, 0), T;
    C[0] = B[0] = 1;
    // window[i] = s_{k-i}: kept as a reversed packed copy of the prefix
    Poly rev((size_t)n / 64 + 2, 0);  // rev bit (n-1-t) = s_t
    for (int t = 0; t < n; ++t)
        if (bits[t] & 1) rev[(size_t)(n - 1 - t) >> 6] |= 1ull << ((n - 1 - t) & 63);
    int L = 0, m = 1;
    for (int k = 0; k < n; ++k) {
        // d = sum_{i=0..L} C_i s_{k-i};  s_{k-i} = rev bit (n-1-k+i)
        const int base = n - 1 - k;
        uint64_t acc = 0;
        const int words = L / 64 + 1;
        for (int w = 0; w < words; ++w) {
            const int pos = base + 64 * w;
            const size_t q = (size_t)pos >> 6;
            const int s = pos & 63;
            uint64_t win = rev[q] >> s;
            if (s && q + 1 < rev.size()) win |= rev[q + 1] << (64 - s);
            if (w == words - 1 && ((L + 1) & 63)) win &= (1ull << ((L + 1) & 63)) - 1;
            acc ^= C[w] & win;
        }
        if (!__builtin_parityll(acc)) {
            ++m;
            continue;
        }
        if (2 * L <= k) {
            T = C;
            xor_shifted(C.data(), C.size(), B.data(), B.size(), m);
            L = k + 1 - L;
            B = std::move(T);
            m = 1;
        } else {
            xor_shifted(C.data(), C.size(), B.data(), B.size(), m);
            ++m;
        }
    }
    if (annihilator) {
        Poly P((size_t)L / 64 + 1, 0);
        for (int j = 0; j <= L; ++j)
            if (bit(C, L - j)) P[(size_t)j >> 6] |= 1ull << (j & 63);
        trim(P);
        *annihilator = std::move(P);
    }
    return L;
}

}  // namespace poly
}  // namespace mtgp

// mtgp_poly.hpp -- GF(2)[x] polynomial arithmetic for jump-ahead planning.
//
// A polynomial is a bit vector in 64-bit words, bit i = coefficient of x^i.
// Host code only.  Multiplication uses the x86 carry-less multiply
// instruction; reduction modulo p uses Barrett's method with a precomputed
// quotient of x^(2d) by p (exact over GF(2)).
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

namespace mtgp {
namespace poly {

using Poly = std::vector<uint64_t>;

int degree(const Poly &a);                 // -1 for the zero polynomial
void trim(Poly &a);
Poly mul(const Poly &a, const Poly &b);    // carry-less product
Poly square(const Poly &a);
Poly shl(const Poly &a, int n);            // a * x^n
Poly mod(const Poly &a, const Poly &p);    // schoolbook remainder
Poly divq(const Poly &a, const Poly &p);   // schoolbook quotient
Poly gcd(Poly a, Poly b);
Poly lcm(const Poly &a, const Poly &b);

// Reducer for one modulus p of degree d >= 1.
struct Modulus {
    Poly p;
    int d = 0;
    Poly mu;  // floor(x^(2d) / p)
    explicit Modulus(const Poly &p_);
    Poly reduce(const Poly &a) const;  // a mod p (Barrett when deg(a) < 2d)
    Poly mulmod(const Poly &a, const Poly &b) const;
    Poly sqrmod(const Poly &a) const;
    Poly powx(uint64_t e) const;        // x^e mod p
};

// Berlekamp-Massey on n bits (one per byte).  Returns L and the
// annihilating polynomial P(x) = x^L C(1/x) of the sequence, i.e.
// sum_i P_i s_{t+i} = 0 for all t with t+L < n.
int berlekamp_massey(const uint8_t *bits, int n, Poly *annihilator);

}  // namespace poly
}  // namespace mtgp

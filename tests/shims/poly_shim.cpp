// Test shim: exposes the library's host GF(2)[x] routines with a C ABI so
// the CPU tests can check them against Python big-integer arithmetic.
#include <cstring>

#include "mtgp_poly.hpp"

using mtgp::poly::Poly;

static Poly in(const unsigned long long *w, int n) { return Poly(w, w + n); }
static int out(const Poly &p, unsigned long long *o, int cap) {
    int n = (int)p.size();
    if (n > cap) return -1;
    std::memcpy(o, p.data(), sizeof(unsigned long long) * (size_t)n);
    return n;
}

extern "C" {
int shim_mulmod(const unsigned long long *a, int na, const unsigned long long *b, int nb,
                const unsigned long long *p, int np, unsigned long long *o, int cap) {
    mtgp::poly::Modulus m(in(p, np));
    return out(m.mulmod(m.reduce(in(a, na)), m.reduce(in(b, nb))), o, cap);
}
int shim_powx(unsigned long long e, const unsigned long long *p, int np, unsigned long long *o,
              int cap) {
    mtgp::poly::Modulus m(in(p, np));
    return out(m.powx(e), o, cap);
}
int shim_lcm(const unsigned long long *a, int na, const unsigned long long *b, int nb,
             unsigned long long *o, int cap) {
    return out(mtgp::poly::lcm(in(a, na), in(b, nb)), o, cap);
}
int shim_bm(const unsigned char *bits, int n, unsigned long long *o, int cap, int *L) {
    Poly ann;
    *L = mtgp::poly::berlekamp_massey(bits, n, &ann);
    return out(ann, o, cap);
}
}

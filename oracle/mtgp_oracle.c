/*
 * mtgp_oracle.c -- plain CPU oracle for MTGP32 bulk generation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg load this library.  The GPU library shares
 * no code, header, table or helper with it, and neither side includes the
 * other.
 *
 * What it computes (Passerat-Palmbach et al., ESM 2010):
 *   - a generator is a seed status plus a parameterised status (Sec. 3.1);
 *   - each generator is one independent stream, owned by one thread block on
 *     the GPU, with the same numbers produced on the CPU (Sec. 2, Sec. 3.2);
 *   - the generator is a GF(2)-linear Mersenne-Twister-family recurrence
 *     (Sec. 3.1), whose word-level form the paper leaves to Saito's MTGP.
 *     The form used here is the published MTGP32 one: two adjacent words
 *     mixed under the period mask, a left-shift self-XOR, the right-shifted
 *     pos-tap, and a 16-entry table indexed by the low four bits; the output
 *     is tempered by a 16-entry table indexed by a byte-folded helper word.
 *
 * Everything is written in the order of that definition, one word at a time,
 * over a full history array.  No blocking, no vectorisation, no reordering.
 * Floating point: the only fp operation is the final single-precision
 * subtraction of 1.0, which is exact for every input (the operand lies in
 * [1, 2) and the result is a multiple of 2^-23).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint32_t mexp, pos, sh1, sh2, mask;
    uint32_t rec[16];  /* recursion table, indexed by the low 4 bits of Y   */
    uint32_t tmp[16];  /* tempering table for uint32 output                 */
    uint32_t flt[16];  /* tempering table for float output (exponent 0x7F)  */
} oracle_params;

/* State length in 32-bit words for a Mersenne exponent: the smallest N with
 * 32N > mexp, i.e. floor(mexp/32)+1.  The oracle accepts any mexp >= 65 that
 * is not a multiple of 32 (so at least one bit of the oldest word is kept). */
int oracle_state_words(uint32_t mexp)
{
    if (mexp < 65 || mexp % 32 == 0) return -1;
    return (int)(mexp / 32 + 1);
}

/* Period mask: the upper 32 - r bits of the oldest word, r = 32N - mexp. */
uint32_t oracle_mask(uint32_t mexp)
{
    int n = oracle_state_words(mexp);
    if (n < 0) return 0;
    uint32_t r = 32u * (uint32_t)n - mexp;
    return 0xFFFFFFFFu << r;
}

/* 0 if the parameter set is usable, otherwise a negative code naming the
 * first bad field: -1 mexp, -2 mask, -3 pos, -4 sh1, -5 sh2, -6 float table. */
int oracle_check_params(const oracle_params *p)
{
    int n = oracle_state_words(p->mexp);
    if (n < 0) return -1;
    if (p->mask != oracle_mask(p->mexp)) return -2;
    if (p->pos < 1 || p->pos > (uint32_t)n - 2) return -3;
    if (p->sh1 > 31) return -4;
    if (p->sh2 > 31) return -5;
    for (int i = 0; i < 16; i++)
        if ((p->flt[i] >> 23) != 0x7Fu) return -6;
    return 0;
}

/* Seed status -> initial state, the Mersenne Twister initialisation:
 *   x_0 = seed,  x_i = 1812433253 * (x_{i-1} XOR (x_{i-1} >> 30)) + i  (mod 2^32).
 * The paper fixes the seed status to 0 in its experiments (Sec. 5.1). */
void oracle_seed(uint32_t seed, int n_words, uint32_t *x)
{
    x[0] = seed;
    for (int i = 1; i < n_words; i++)
        x[i] = 1812433253u * (x[i - 1] ^ (x[i - 1] >> 30)) + (uint32_t)i;
}

/* One new word from the three taps of the recurrence. */
static uint32_t recursion(const oracle_params *p, uint32_t oldest,
                          uint32_t next, uint32_t tap)
{
    uint32_t X = (oldest & p->mask) ^ next;
    X ^= X << p->sh1;
    uint32_t Y = X ^ (tap >> p->sh2);
    return Y ^ p->rec[Y & 0xFu];
}

/* Index into the tempering tables from the helper word. */
static uint32_t temper_index(uint32_t helper)
{
    uint32_t H = helper;
    H ^= H >> 16;
    H ^= H >> 8;
    return H & 0xFu;
}

/* Advance one stream by `count` outputs.
 *   state  : N words in sequence order (x_j .. x_{j+N-1}); updated in place
 *            to the state after the call, so that calls continue the stream.
 *   as_float == 0 : out[j] = x_{N+j} XOR tmp[t_j]                (uint32)
 *   as_float != 0 : out[j] = bits of  float((x_{N+j} >> 9) XOR flt[t_j]) - 1.0f
 * where t_j is the tempering index of the helper word x_{j+pos-1}.
 * Returns 0, or -1 on bad parameters / allocation failure. */
int oracle_generate(const oracle_params *p, uint32_t *state, uint64_t count,
                    int as_float, uint32_t *out)
{
    if (oracle_check_params(p) != 0) return -1;
    const uint64_t N = (uint64_t)oracle_state_words(p->mexp);
    const uint64_t pos = p->pos;
    uint32_t *x = (uint32_t *)malloc((size_t)(N + count) * sizeof(uint32_t));
    if (!x) return -1;
    memcpy(x, state, (size_t)N * sizeof(uint32_t));

    for (uint64_t j = 0; j < count; j++) {
        uint64_t n = N + j;
        x[n] = recursion(p, x[j], x[j + 1], x[j + pos]);
        uint32_t t = temper_index(x[j + pos - 1]);
        if (!as_float) {
            out[j] = x[n] ^ p->tmp[t];
        } else {
            uint32_t bits = (x[n] >> 9) ^ p->flt[t];
            float f;
            memcpy(&f, &bits, sizeof f);
            f = f - 1.0f;
            memcpy(&out[j], &f, sizeof f);
        }
    }
    memcpy(state, x + count, (size_t)N * sizeof(uint32_t));
    free(x);
    return 0;
}

/* Berlekamp-Massey over GF(2) (Massey 1969), bit-packed into 64-bit words.
 * s: n bits, one per byte (0/1).  Returns the linear complexity L and, if
 * conn != NULL, writes the connection polynomial C(x) = 1 + c_1 x + ... + c_L x^L
 * as conn[0..L] (one coefficient per byte); conn must hold n+1 bytes.
 * The sequence then satisfies s_k = XOR_{i=1..L} c_i s_{k-i} for L <= k < n. */
int oracle_berlekamp_massey(const uint8_t *s, int n, uint8_t *conn)
{
    if (n <= 0) { if (conn) conn[0] = 1; return 0; }
    const int nw = (n + 1 + 63) / 64 + 1;
    /* rs = s reversed: bit k of rs is s[n-1-k]; then s[m-i] is bit n-1-m+i. */
    uint64_t *rs = (uint64_t *)calloc((size_t)(2 * nw + 4), 8);
    uint64_t *C = (uint64_t *)calloc((size_t)nw, 8);
    uint64_t *B = (uint64_t *)calloc((size_t)nw, 8);
    uint64_t *T = (uint64_t *)calloc((size_t)nw, 8);
    if (!rs || !C || !B || !T) { free(rs); free(C); free(B); free(T); return -1; }
    for (int k = 0; k < n; k++)
        if (s[n - 1 - k] & 1) rs[k >> 6] |= 1ull << (k & 63);
    C[0] = 1; B[0] = 1;
    int L = 0, m = 1;
    for (int k = 0; k < n; k++) {
        /* discrepancy d = sum_{i=0..L} c_i s_{k-i} = parity(C & (rs >> (n-1-k))) */
        int off = n - 1 - k;
        int q = off >> 6, r = off & 63;
        uint64_t acc = 0;
        int words = (L + 1 + 63) / 64;
        for (int w = 0; w < words; w++) {
            uint64_t lo = rs[q + w] >> r;
            uint64_t hi = r ? rs[q + w + 1] << (64 - r) : 0;
            uint64_t win = lo | hi;
            if (w == words - 1) {
                int keep = (L + 1) - 64 * w;
                if (keep < 64) win &= (1ull << keep) - 1;
            }
            acc ^= C[w] & win;
        }
        int d = __builtin_parityll(acc);
        if (d == 0) { m++; continue; }
        int qm = m >> 6, rm = m & 63;
        if (2 * L <= k) {
            memcpy(T, C, (size_t)nw * 8);
            for (int w = nw - 1; w >= 0; w--) {  /* C ^= B << m */
                uint64_t v = 0;
                if (w - qm >= 0) v = B[w - qm] << rm;
                if (rm && w - qm - 1 >= 0) v |= B[w - qm - 1] >> (64 - rm);
                C[w] ^= v;
            }
            L = k + 1 - L;
            memcpy(B, T, (size_t)nw * 8);
            m = 1;
        } else {
            for (int w = nw - 1; w >= 0; w--) {
                uint64_t v = 0;
                if (w - qm >= 0) v = B[w - qm] << rm;
                if (rm && w - qm - 1 >= 0) v |= B[w - qm - 1] >> (64 - rm);
                C[w] ^= v;
            }
            m++;
        }
    }
    if (conn)
        for (int i = 0; i <= n; i++)
            conn[i] = (i <= L) ? (uint8_t)((C[i >> 6] >> (i & 63)) & 1) : 0;
    free(rs); free(C); free(B); free(T);
    return L;
}

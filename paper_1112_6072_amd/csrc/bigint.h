// Small fixed-width unsigned integers and residue helpers for exact recombination on the host.
#pragma once
#include <stdint.h>

#include <cmath>
#include <vector>

namespace hp {

typedef unsigned __int128 u128;
typedef __int128 i128;

// 512-bit unsigned integer, little-endian 64-bit limbs.
struct U512 {
    uint64_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    void add(const U512 &o) {
        u128 c = 0;
        for (int k = 0; k < 8; ++k) {
            c += (u128)w[k] + o.w[k];
            w[k] = (uint64_t)c;
            c >>= 64;
        }
    }
    void add_u128(u128 v) {
        U512 t;
        t.w[0] = (uint64_t)v;
        t.w[1] = (uint64_t)(v >> 64);
        add(t);
    }
    void mul_u64(uint64_t m) {
        u128 c = 0;
        for (int k = 0; k < 8; ++k) {
            c += (u128)w[k] * m;
            w[k] = (uint64_t)c;
            c >>= 64;
        }
    }
    int nlimb() const {
        int n = 8;
        while (n > 0 && w[n - 1] == 0) --n;
        return n;
    }
    int bits() const {
        const int n = nlimb();
        if (n == 0) return 0;
        return 64 * (n - 1) + (64 - __builtin_clzll(w[n - 1]));
    }
};

// Compare magnitudes: -1, 0, 1.
inline int cmp(const U512 &a, const U512 &b) {
    for (int k = 7; k >= 0; --k)
        if (a.w[k] != b.w[k]) return a.w[k] < b.w[k] ? -1 : 1;
    return 0;
}

// a - b for a >= b.
inline U512 sub(const U512 &a, const U512 &b) {
    U512 r;
    uint64_t borrow = 0;
    for (int k = 0; k < 8; ++k) {
        const u128 t = (u128)a.w[k] - b.w[k] - borrow;
        r.w[k] = (uint64_t)t;
        borrow = (uint64_t)(t >> 64) ? 1 : 0;
    }
    return r;
}

// Signed 512-bit integer in sign-magnitude form (the exact interpolation of the permanental
// polynomial). Operations report overflow of the 512-bit magnitude by returning false.
struct S512 {
    U512 mag;
    bool neg = false;
    bool is_zero() const { return mag.nlimb() == 0; }
    S512 operator-() const {
        S512 r = *this;
        if (!r.is_zero()) r.neg = !r.neg;
        return r;
    }
};

inline S512 add(const S512 &a, const S512 &b) {
    S512 r;
    if (a.neg == b.neg) {
        r.mag = a.mag;
        r.mag.add(b.mag);
        r.neg = a.neg;
    } else if (cmp(a.mag, b.mag) >= 0) {
        r.mag = sub(a.mag, b.mag);
        r.neg = a.neg;
    } else {
        r.mag = sub(b.mag, a.mag);
        r.neg = b.neg;
    }
    if (r.is_zero()) r.neg = false;
    return r;
}

inline S512 sub(const S512 &a, const S512 &b) { return add(a, -b); }

// a * m; false when the magnitude leaves 512 bits.
inline bool mul_u64(S512 &a, uint64_t m) {
    u128 c = 0;
    for (int k = 0; k < 8; ++k) {
        c += (u128)a.mag.w[k] * m;
        a.mag.w[k] = (uint64_t)c;
        c >>= 64;
    }
    if (a.is_zero()) a.neg = false;
    return c == 0;
}

// a / m when m divides a exactly; false otherwise.
inline bool divexact_u64(S512 &a, uint64_t m) {
    u128 rem = 0;
    for (int k = 7; k >= 0; --k) {
        const u128 cur = (rem << 64) | a.mag.w[k];
        a.mag.w[k] = (uint64_t)(cur / m);
        rem = cur % m;
    }
    return rem == 0;
}

inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)((u128)a * b % p); }

inline uint64_t powmod(uint64_t a, uint64_t e, uint64_t p) {
    uint64_t r = 1 % p;
    a %= p;
    while (e) {
        if (e & 1) r = mulmod(r, a, p);
        a = mulmod(a, a, p);
        e >>= 1;
    }
    return r;
}

// Inverse modulo a prime p (Fermat).
inline uint64_t invmod(uint64_t a, uint64_t p) { return powmod(a, p - 2, p); }

// Whether v is prime (trial division).
inline bool is_prime_u32(uint32_t v) {
    if (v < 2) return false;
    for (uint32_t d = 2; (uint64_t)d * d <= v; ++d)
        if (v % d == 0) return false;
    return true;
}

// Odd primes below `below`, largest first, until their product exceeds 2^(bits + 1), then one
// more (a check prime). Empty when the primes below `below` run out first.
inline std::vector<uint32_t> residue_primes(uint32_t below, double bits) {
    std::vector<uint32_t> p;
    double cover = 0.0;
    uint32_t q = below > 3 ? below - 1 : 0;
    if (!(q & 1)) --q;
    bool done = false;
    for (; q >= 3; q -= 2)
        if (is_prime_u32(q)) {
            if (done) {
                p.push_back(q);
                return p;
            }
            p.push_back(q);
            cover += std::log2((double)q);
            done = cover > bits + 1.0;
        }
    return {};
}

// The value in [0, p_0 ... p_(K-1)) with residues r[k] modulo the distinct primes p[k] < 2^32
// (Garner's mixed-radix form: x = v_0 + p_0 (v_1 + p_1 (v_2 + ...))). The product must stay
// below 2^512.
inline U512 crt_garner(const std::vector<uint32_t> &p, const uint64_t *r) {
    const size_t K = p.size();
    std::vector<uint64_t> v(K);
    for (size_t k = 0; k < K; ++k) {
        uint64_t t = 0, prod = 1;   // the mixed-radix value so far, and p_0 .. p_(k-1), modulo p_k
        for (size_t j = k; j-- > 0;) t = (t * p[j] + v[j]) % p[k];
        for (size_t j = 0; j < k; ++j) prod = prod * p[j] % p[k];
        v[k] = (r[k] % p[k] + p[k] - t) % p[k] * invmod(prod, p[k]) % p[k];
    }
    U512 x;
    for (size_t k = K; k-- > 0;) {
        x.mul_u64(p[k]);
        U512 a;
        a.w[0] = v[k];
        x.add(a);
    }
    return x;
}

// x modulo m (m < 2^63).
inline uint64_t mod_u512(const U512 &x, uint64_t m) {
    u128 r = 0;
    for (int w = 7; w >= 0; --w) r = ((r << 64) | x.w[w]) % m;
    return (uint64_t)r;
}

}  // namespace hp

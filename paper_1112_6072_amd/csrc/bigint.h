// Small fixed-width unsigned integers and residue helpers for exact recombination on the host.
#pragma once
#include <stdint.h>

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

}  // namespace hp

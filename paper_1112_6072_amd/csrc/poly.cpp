// The permanental polynomial per(xI - A) of a non-negative integer matrix (the paper's
// application section, where it is evaluated at complex points in floating point). Here it
// is exact: per(xI + A) = sum_k a_k x^k, where a_k is the sum of the permanents of the
// principal sub-matrices of A of order n - k (every term of the permanent takes, for each row,
// either the x of the diagonal or an entry of A), so a_k >= 0 and
// per(xI - A) = sum_k (-1)^(n-k) a_k x^k. The matrices xI + A for x = 0..n have non-negative
// entries: they are n + 1 problems of one batched device pass (steps 1-6 of the hot path),
// and the n + 1 values determine the degree-n polynomial. The coefficients come from exact
// integer interpolation: forward differences give the Newton coefficients e_k =
// Delta^k p(0) / k! (integers, as p has integer coefficients), and p(x) = sum_k e_k x(x-1)..(x-k+1)
// is expanded by Horner's rule in that basis, p = e_0 + x(e_1 + (x-1)(e_2 + ...)).
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/hperm.h"
#include "bigint.h"
#include "expand.h"

using hp::S512;
using hp::U512;

namespace {

// The CSR arrays of xI + A (entries of A on the diagonal are increased by x).
void add_diagonal(int32_t n, const int32_t *rp, const int32_t *ci, const uint32_t *va, uint32_t x,
                  std::vector<int32_t> &orp, std::vector<int32_t> &oci, std::vector<uint32_t> &ova) {
    const size_t base = oci.size();
    for (int32_t i = 0; i < n; ++i) {
        orp.push_back((int32_t)(oci.size() - base));
        bool placed = false;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (!placed && ci[e] >= i) {
                if (ci[e] == i) {
                    oci.push_back(i);
                    ova.push_back(va[e] + x);
                    placed = true;
                    continue;
                }
                if (x) {
                    oci.push_back(i);
                    ova.push_back(x);
                }
                placed = true;
            }
            oci.push_back(ci[e]);
            ova.push_back(va[e]);
        }
        if (!placed && x) {
            oci.push_back(i);
            ova.push_back(x);
        }
    }
    orp.push_back((int32_t)(oci.size() - base));
}

// The coefficients of the degree-n polynomial through (x, y_x), x = 0..n, modulo the prime
// p > n: forward differences, Newton coefficients Delta^k p(0) / k!, and Horner's rule in the
// falling-factorial basis, as in the exact interpolation.
std::vector<uint64_t> interpolate_mod(const std::vector<uint64_t> &y, uint64_t p) {
    const size_t np = y.size();
    std::vector<uint64_t> d(y);
    for (size_t k = 1; k < np; ++k)
        for (size_t i = np - 1; i >= k; --i) d[i] = (d[i] + p - d[i - 1]) % p;
    uint64_t fact = 1;
    for (size_t k = 2; k < np; ++k) {
        fact = fact * k % p;
        d[k] = d[k] * hp::invmod(fact, p) % p;
    }
    std::vector<uint64_t> poly(np, 0);
    poly[0] = d[np - 1];
    for (size_t k = np - 1; k-- > 0;) {
        const size_t deg = np - 2 - k;   // degree of poly before this step
        for (size_t j = deg + 1; j-- > 0;) {
            poly[j + 1] = (poly[j + 1] + poly[j]) % p;
            poly[j] = (p - poly[j] * (k % p) % p) % p;
        }
        poly[0] = (poly[0] + d[k]) % p;
    }
    return poly;
}

S512 from_limbs(const uint64_t *limb) {
    S512 v;
    for (int k = 0; k < 8; ++k) v.mag.w[k] = limb[k];
    return v;
}

}  // namespace

hperm_status hperm_polynomial_interpolate(int32_t n, const uint64_t *values, int32_t alternate,
                                          hperm_coeff *coeffs) {
    if (n < 0 || n > 128 || !values || !coeffs) return HPERM_E_INVALID;
    const int np = n + 1;
    // forward differences d[k] = Delta^k p(0)
    std::vector<S512> d((size_t)np);
    for (int x = 0; x < np; ++x) d[(size_t)x] = from_limbs(values + 8 * (size_t)x);
    for (int k = 1; k < np; ++k)
        for (int i = n; i >= k; --i) d[(size_t)i] = hp::sub(d[(size_t)i], d[(size_t)i - 1]);
    // Newton coefficients e_k = d[k] / k!
    for (int k = 2; k < np; ++k)
        for (int j = 2; j <= k; ++j)
            if (!hp::divexact_u64(d[(size_t)k], (uint64_t)j)) return HPERM_E_INVALID;
    // Horner in the falling-factorial basis: poly = e_k + (x - k) poly, k = n-1 .. 0
    std::vector<S512> poly((size_t)np);
    poly[0] = d[(size_t)n];
    for (int k = n - 1; k >= 0; --k) {
        const int deg = n - 1 - k;   // degree of poly before this step
        std::vector<S512> next((size_t)deg + 2);
        for (int j = deg; j >= 0; --j) {
            next[(size_t)j + 1] = hp::add(next[(size_t)j + 1], poly[(size_t)j]);
            S512 t = poly[(size_t)j];
            if (!hp::mul_u64(t, (uint64_t)k)) return HPERM_E_RANGE;
            next[(size_t)j] = hp::sub(next[(size_t)j], t);
        }
        next[0] = hp::add(next[0], d[(size_t)k]);
        for (int j = 0; j <= deg + 1; ++j) {
            poly[(size_t)j] = next[(size_t)j];
            if (poly[(size_t)j].mag.bits() > 500) return HPERM_E_RANGE;
        }
    }
    // exactness: the polynomial reproduces every value
    for (int x = 0; x < np; ++x) {
        S512 v = poly[(size_t)n];
        for (int j = n - 1; j >= 0; --j) {
            if (!hp::mul_u64(v, (uint64_t)x)) return HPERM_E_RANGE;
            v = hp::add(v, poly[(size_t)j]);
        }
        const S512 want = from_limbs(values + 8 * (size_t)x);
        if (v.neg || hp::cmp(v.mag, want.mag) != 0) return HPERM_E_INVALID;
    }
    for (int j = 0; j < np; ++j) {
        memset(&coeffs[j], 0, sizeof(hperm_coeff));
        for (int k = 0; k < 8; ++k) coeffs[j].limb[k] = poly[(size_t)j].mag.w[k];
        coeffs[j].nlimb = poly[(size_t)j].mag.nlimb();
        bool neg = poly[(size_t)j].neg;
        if (alternate && ((n - j) & 1)) neg = !neg;
        coeffs[j].negative = (neg && coeffs[j].nlimb) ? 1 : 0;
    }
    return HPERM_OK;
}

namespace {

// per(xI - A) for orders 23..64 beyond the exact rings. The coefficients of per(xI + A) are
// a_k = sum over the principal sub-matrices A_S of order n - k of per(A_S), and
// per(A_S) <= prod_{i in S} g_i with g_i the row sum of A (or, for a 0-1 matrix, Bregman's
// (r_i!)^(1/r_i)), so a_k <= e_{n-k}(g), the elementary symmetric function. per(xI + A) is
// evaluated at x = 0..n modulo K + 1 primes below 2^18 (the device path's modular mode), the
// polynomial interpolated modulo each prime, and each coefficient rebuilt by the Chinese
// remainder theorem over the K primes whose product exceeds the bound, then checked against
// the last prime. The values reach the bound of the largest evaluation, the coefficients far
// less (C60: values about 2^355, coefficients below 2^50, bound 2^86.4: 6 primes, not 22).
hperm_status modular_polynomial(hperm_ctx *ctx, int32_t n, const int32_t *row_ptr, const uint32_t *val,
                                const std::vector<int32_t> &sizes, const std::vector<int64_t> &rp_off,
                                const std::vector<int64_t> &nz_off, const std::vector<int32_t> &rp,
                                const std::vector<int32_t> &ci, const std::vector<uint32_t> &va,
                                hperm_coeff *coeffs) {
    const int np = n + 1;
    bool zero_one = true;
    std::vector<long double> g((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        uint64_t rs = 0;
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            rs += val[e];
            zero_one = zero_one && val[e] <= 1;
        }
        g[(size_t)i] = (long double)rs;
    }
    if (zero_one)
        for (int32_t i = 0; i < n; ++i) {   // Bregman: (r!)^(1/r)
            const long double r = g[(size_t)i];
            g[(size_t)i] = r > 0 ? std::exp(std::lgamma(r + 1.0L) / r) : 0.0L;
        }
    std::vector<long double> e((size_t)np, 0.0L);   // e_j(g), j = 0..n
    e[0] = 1.0L;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j >= 1; --j) e[(size_t)j] += e[(size_t)j - 1] * g[(size_t)i];
    long double emax = 1.0L;
    for (int j = 0; j < np; ++j) emax = std::max(emax, e[(size_t)j]);
    const double bound = (double)std::log2(emax) * (1.0 + 1e-9) + 1.0;   // rounding of the sums
    // (residue_primes adds one more bit)
    const std::vector<uint32_t> primes = hp::residue_primes(1u << 18, bound);
    if (primes.empty()) return HPERM_E_RANGE;
    double cover = 0.0;
    for (uint32_t q : primes) cover += std::log2((double)q);
    if (cover > 500.0) return HPERM_E_RANGE;   // beyond the 512-bit coefficients
    std::vector<uint64_t> y((size_t)np * primes.size());   // prime x point
    for (size_t j = 0; j < primes.size(); ++j) {
        const hperm_status s = hperm_permanent_mod_batch_csr(ctx, np, sizes.data(), rp_off.data(), nz_off.data(),
                                                             rp.data(), ci.data(), va.data(), primes[j],
                                                             y.data() + j * (size_t)np);
        if (s) return s;
    }
    const hperm_status s = hperm_polynomial_from_residues(n, (int32_t)primes.size(), primes.data(), y.data(), 1, coeffs);
    if (s == HPERM_E_INVALID) return HPERM_E_INTERNAL;   // residues that disagree
    if (s) return s;
    if (!(coeffs[n].nlimb == 1 && coeffs[n].limb[0] == 1)) return HPERM_E_INTERNAL;   // monic
    return HPERM_OK;
}

}  // namespace

hperm_status hperm_polynomial_from_residues(int32_t n, int32_t nprimes, const uint32_t *primes,
                                            const uint64_t *residues, int32_t alternate, hperm_coeff *coeffs) {
    if (n < 0 || n > 128 || nprimes < 2 || !primes || !residues || !coeffs) return HPERM_E_INVALID;
    const int np = n + 1;
    std::vector<uint32_t> pr(primes, primes + nprimes);
    double cover = 0.0;
    for (int j = 0; j < nprimes; ++j) {
        if (pr[(size_t)j] <= (uint32_t)n || !hp::is_prime_u32(pr[(size_t)j])) return HPERM_E_INVALID;
        for (int i = 0; i < j; ++i)
            if (pr[(size_t)i] == pr[(size_t)j]) return HPERM_E_INVALID;
        if (j + 1 < nprimes) cover += std::log2((double)pr[(size_t)j]);
    }
    if (cover > 511.0) return HPERM_E_RANGE;   // the product of the CRT primes must fit 512 bits
    const size_t P = pr.size(), K = P - 1;
    std::vector<uint64_t> cr((size_t)np * P);   // coefficient x prime
    for (size_t j = 0; j < P; ++j) {
        std::vector<uint64_t> y(residues + j * (size_t)np, residues + (j + 1) * (size_t)np);
        for (uint64_t &v : y) v %= pr[j];
        const std::vector<uint64_t> c = interpolate_mod(y, pr[j]);
        for (int k = 0; k < np; ++k) cr[(size_t)k * P + j] = c[(size_t)k];
    }
    const std::vector<uint32_t> base(pr.begin(), pr.begin() + (long)K);
    for (int k = 0; k < np; ++k) {
        const uint64_t *rk = cr.data() + (size_t)k * P;
        const U512 a = hp::crt_garner(base, rk);
        if (hp::mod_u512(a, pr[K]) != rk[K]) return HPERM_E_INVALID;   // the check prime disagrees
        memset(&coeffs[k], 0, sizeof(hperm_coeff));
        for (int w = 0; w < 8; ++w) coeffs[k].limb[w] = a.w[w];
        coeffs[k].nlimb = a.nlimb();
        coeffs[k].negative = (alternate && coeffs[k].nlimb && ((n - k) & 1)) ? 1 : 0;
    }
    return HPERM_OK;
}

hperm_status hperm_permanental_polynomial(hperm_ctx *ctx, int32_t n, const int32_t *row_ptr,
                                          const int32_t *col_idx, const uint32_t *val,
                                          hperm_coeff *coeffs) {
    if (!ctx || !coeffs || n < 0 || n > 128) return HPERM_E_INVALID;
    if (n > 0 && (!row_ptr || !col_idx || !val)) return HPERM_E_INVALID;
    if (n > 0 && !hp::validate_csr(hp::CsrView{n, row_ptr, col_idx, val}).empty()) return HPERM_E_INVALID;
    for (int32_t i = 0; n > 0 && i < n; ++i)
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            if (col_idx[e] == i && val[e] > UINT32_MAX - (uint32_t)n) return HPERM_E_RANGE;
    const int np = n + 1;
    // the n + 1 problems xI + A, concatenated
    std::vector<int32_t> rp, ci, sizes((size_t)np, n);
    std::vector<uint32_t> va;
    std::vector<int64_t> rp_off((size_t)np), nz_off((size_t)np);
    for (int x = 0; x < np; ++x) {
        rp_off[(size_t)x] = (int64_t)rp.size();
        nz_off[(size_t)x] = (int64_t)ci.size();
        add_diagonal(n, row_ptr, col_idx, val, (uint32_t)x, rp, ci, va);
    }
    ci.push_back(0);   // non-empty arrays for the empty matrix
    va.push_back(0);
    std::vector<hperm_result> res((size_t)np);
    // up to order 40 every xI + A is a single job (m_cut = n): no expansion merges, which would
    // multiply the diagonal's large entries together
    hperm_opts saved, o;
    hperm_status s = hperm_ctx_get_opts(ctx, &saved);
    if (s) return s;
    o = saved;
    o.device_expand = 0;   // the host expansion keeps the single-job rule below (and its bounds)
    if (n <= 40) {
        o.m_cut = std::max(o.m_cut, n);
        o.m_cap = std::max(o.m_cap, o.m_cut);
    }
    s = hperm_ctx_set_opts(ctx, &o);
    if (s) return s;
    // the bound grows with x: check the last problem (x = n) on the host before any device work
    hperm_jobs *probe = nullptr;
    s = hperm_expand_batch_csr(ctx, 1, sizes.data() + n, rp_off.data() + n, nz_off.data() + n, rp.data(),
                               ci.data(), va.data(), &probe);
    if (probe) hperm_jobs_free(probe);
    const bool modular = s == HPERM_E_RANGE && n > 22 && n <= 64;
    if (!s)
        s = hperm_permanent_batch_csr(ctx, np, sizes.data(), rp_off.data(), nz_off.data(), rp.data(),
                                      ci.data(), va.data(), res.data());
    {
        const hperm_status r = hperm_ctx_set_opts(ctx, &saved);
        if (!s) s = r;
    }
    if (modular) return modular_polynomial(ctx, n, row_ptr, val, sizes, rp_off, nz_off, rp, ci, va, coeffs);
    if (s) return s;
    std::vector<uint64_t> values((size_t)np * 8);
    for (int x = 0; x < np; ++x)
        for (int k = 0; k < 8; ++k) values[(size_t)x * 8 + k] = res[(size_t)x].limb[k];
    // p(x) = per(xI + A); c_k = (-1)^(n-k) a_k
    const hperm_status si = hperm_polynomial_interpolate(n, values.data(), 1, coeffs);
    if (si == HPERM_E_INVALID) return HPERM_E_INTERNAL;   // values from the device that no
                                                          // integer polynomial of degree n fits
    if (si) return si;
    for (int j = 0; j < np; ++j)   // a_k >= 0: the sign must be exactly the alternation
        if (coeffs[j].nlimb && coeffs[j].negative != ((n - j) & 1)) return HPERM_E_INTERNAL;
    return HPERM_OK;
}

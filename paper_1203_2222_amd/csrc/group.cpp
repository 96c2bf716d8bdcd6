// SU(2) group tables on the host: 6j symbols by Racah's closed formula and
// the recoupling coefficients F of eq:sixj.  Spins are doubled integers
// throughout.  The alternating sum of Racah's formula is taken exactly: every
// term, multiplied by one common denominator, is an integer, and the terms
// are added as unsigned big integers (positive and negative parts apart), so
// no cancellation can lose digits.  Only the last steps round: the integer
// sum and the denominator go to long double (64-bit mantissa) and the
// triangle prefactor is a square root of a ratio of factorials, all positive
// products, so the result carries a relative error of a few 1e-19 before the
// final rounding to FP64, for every spin up to 60.
#include <cmath>
#include <cstdint>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace sym {
namespace {

// Doubled spins up to 120 (j = 60): every factorial is at most 241! (about
// 10^471) and the products below at most eight of them, inside long double's
// range (about 10^4932).
constexpr int kMaxSpin = 120;
constexpr int kMaxFact = 2 * kMaxSpin + 1;

long double fact(int n) {
    static std::vector<long double> table;
    static std::once_flag once;
    std::call_once(once, [] {
        table.resize(kMaxFact + 1);
        table[0] = 1.0L;
        for (int i = 1; i <= kMaxFact; ++i) table[static_cast<size_t>(i)] = table[static_cast<size_t>(i - 1)] * i;
    });
    if (n < 0 || n > kMaxFact) throw Error(SYM_E_UNSUPPORTED, "spin too large for the 6j table");
    return table[static_cast<size_t>(n)];
}

// Square of the triangle coefficient Delta(a,b,c), doubled spins.
long double delta2(int a, int b, int c) {
    return fact((a + b - c) / 2) * fact((a - b + c) / 2) * fact((-a + b + c) / 2) / fact((a + b + c) / 2 + 1);
}

// Unsigned big integer, 32-bit limbs, least significant first.
struct Big {
    std::vector<uint32_t> d;
    explicit Big(uint32_t v = 0) { if (v) d.push_back(v); }
    void mul(uint32_t m) {
        uint64_t carry = 0;
        for (uint32_t& x : d) {
            const uint64_t y = static_cast<uint64_t>(x) * m + carry;
            x = static_cast<uint32_t>(y);
            carry = y >> 32;
        }
        if (carry) d.push_back(static_cast<uint32_t>(carry));
        if (m == 0) d.clear();
    }
    void add(const Big& o) {
        uint64_t carry = 0;
        if (d.size() < o.d.size()) d.resize(o.d.size(), 0);
        for (size_t i = 0; i < d.size(); ++i) {
            const uint64_t y = static_cast<uint64_t>(d[i]) + (i < o.d.size() ? o.d[i] : 0u) + carry;
            d[i] = static_cast<uint32_t>(y);
            carry = y >> 32;
        }
        if (carry) d.push_back(static_cast<uint32_t>(carry));
    }
    bool less(const Big& o) const {
        if (d.size() != o.d.size()) return d.size() < o.d.size();
        for (size_t i = d.size(); i-- > 0;)
            if (d[i] != o.d[i]) return d[i] < o.d[i];
        return false;
    }
    // *this -= o, requires o <= *this
    void sub(const Big& o) {
        int64_t borrow = 0;
        for (size_t i = 0; i < d.size(); ++i) {
            int64_t y = static_cast<int64_t>(d[i]) - (i < o.d.size() ? o.d[i] : 0u) - borrow;
            borrow = y < 0;
            if (y < 0) y += int64_t{1} << 32;
            d[i] = static_cast<uint32_t>(y);
        }
        while (!d.empty() && d.back() == 0) d.pop_back();
    }
    long double value() const {
        long double v = 0.0L;
        for (size_t i = d.size(); i-- > 0;) v = v * 4294967296.0L + d[i];
        return v;
    }
};

// n! / m! for 0 <= m <= n, as a factor list applied to a big integer
void mul_falling(Big& x, int n, int m) {
    for (int k = m + 1; k <= n; ++k) x.mul(static_cast<uint32_t>(k));
}

}  // namespace

namespace {
double sixj_exact(int a, int b, int c, int d, int e, int f);
}

double sixj(int a, int b, int c, int d, int e, int f) {
    if (!(triangle(a, b, c) && triangle(a, e, f) && triangle(d, b, f) && triangle(d, e, c))) return 0.0;
    for (int x : {a, b, c, d, e, f})
        if (x > kMaxSpin) throw Error(SYM_E_UNSUPPORTED, "spin above 60 in a 6j symbol");
    // memoised: plans ask for the same symbols many times
    static std::mutex mu;
    static std::unordered_map<uint64_t, double> memo;
    uint64_t key = 0;
    for (int x : {a, b, c, d, e, f}) key = key << 8 | static_cast<uint64_t>(x);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = memo.find(key);
        if (it != memo.end()) return it->second;
    }
    const double v = sixj_exact(a, b, c, d, e, f);
    std::lock_guard<std::mutex> lk(mu);
    memo.emplace(key, v);
    return v;
}

namespace {

double sixj_exact(int a, int b, int c, int d, int e, int f) {
    const int abc = (a + b + c) / 2, aef = (a + e + f) / 2, dbf = (d + b + f) / 2, dec = (d + e + c) / 2;
    const int abde = (a + b + d + e) / 2, bcef = (b + c + e + f) / 2, cafd = (c + a + f + d) / 2;
    int tlo = abc;
    if (aef > tlo) tlo = aef;
    if (dbf > tlo) tlo = dbf;
    if (dec > tlo) tlo = dec;
    int thi = abde;
    if (bcef < thi) thi = bcef;
    if (cafd < thi) thi = cafd;
    // term(t) = (t+1)! / [(t-abc)! (t-aef)! (t-dbf)! (t-dec)! (abde-t)! (bcef-t)! (cafd-t)!];
    // times D = (thi-abc)! (thi-aef)! (thi-dbf)! (thi-dec)! (abde-tlo)! (bcef-tlo)! (cafd-tlo)!
    // it is the integer (t+1)! prod (thi-x)!/(t-x)! prod (y-tlo)!/(y-t)!
    Big pos, neg;
    for (int t = tlo; t <= thi; ++t) {
        Big term(1);
        mul_falling(term, t + 1, 1);
        for (int x : {abc, aef, dbf, dec}) mul_falling(term, thi - x, t - x);
        for (int y : {abde, bcef, cafd}) mul_falling(term, y - tlo, y - t);
        (t % 2 ? neg : pos).add(term);
    }
    long double mag;
    bool negative = false;
    if (pos.less(neg)) {
        neg.sub(pos);
        mag = neg.value();
        negative = true;
    } else {
        pos.sub(neg);
        mag = pos.value();
    }
    if (mag == 0.0L) return 0.0;
    // the common denominator and the prefactor: products of positive factors
    long double den = 1.0L;
    for (int x : {abc, aef, dbf, dec}) den *= fact(thi - x);
    for (int y : {abde, bcef, cafd}) den *= fact(y - tlo);
    const long double pref = std::sqrt(delta2(a, b, c) * delta2(a, e, f) * delta2(d, b, f) * delta2(d, e, c));
    const long double v = pref * (mag / den);
    return static_cast<double>(negative ? -v : v);
}

}  // namespace

double fmove_coeff(int tA, int tB, int tC, int tJ, int tD, int tE) {
    const double s6 = sixj(tA, tB, tD, tC, tJ, tE);
    if (s6 == 0.0) return 0.0;
    const int ph = (tA + tB + tC + tJ) / 2;
    return ((ph % 2) ? -1.0 : 1.0) * std::sqrt(static_cast<double>((tD + 1) * (tE + 1))) * s6;
}

}  // namespace sym

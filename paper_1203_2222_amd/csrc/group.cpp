// SU(2) group tables on the host: 6j symbols by Racah's closed formula and
// the recoupling coefficients F of eq:sixj, evaluated in long double and
// stored as FP64.  Spins are doubled integers throughout.
#include <cmath>
#include <mutex>
#include <unordered_map>

#include "internal.hpp"

namespace sym {
namespace {

long double fact(int n) {
    static std::vector<long double> table;
    static std::once_flag once;
    std::call_once(once, [] {
        table.resize(171);
        table[0] = 1.0L;
        for (int i = 1; i < 171; ++i) table[static_cast<size_t>(i)] = table[static_cast<size_t>(i - 1)] * i;
    });
    if (n < 0 || n > 170) throw Error(SYM_E_UNSUPPORTED, "spin too large for the 6j table");
    return table[static_cast<size_t>(n)];
}

// Square of the triangle coefficient Delta(a,b,c), doubled spins.
long double delta2(int a, int b, int c) {
    return fact((a + b - c) / 2) * fact((a - b + c) / 2) * fact((-a + b + c) / 2) / fact((a + b + c) / 2 + 1);
}

}  // namespace

double sixj(int a, int b, int c, int d, int e, int f) {
    if (!(triangle(a, b, c) && triangle(a, e, f) && triangle(d, b, f) && triangle(d, e, c))) return 0.0;
    const int abc = (a + b + c) / 2, aef = (a + e + f) / 2, dbf = (d + b + f) / 2, dec = (d + e + c) / 2;
    const int abde = (a + b + d + e) / 2, bcef = (b + c + e + f) / 2, cafd = (c + a + f + d) / 2;
    int tlo = abc;
    if (aef > tlo) tlo = aef;
    if (dbf > tlo) tlo = dbf;
    if (dec > tlo) tlo = dec;
    int thi = abde;
    if (bcef < thi) thi = bcef;
    if (cafd < thi) thi = cafd;
    long double sum = 0.0L;
    for (int t = tlo; t <= thi; ++t) {
        long double term = fact(t + 1) /
            (fact(t - abc) * fact(t - aef) * fact(t - dbf) * fact(t - dec) *
             fact(abde - t) * fact(bcef - t) * fact(cafd - t));
        sum += (t % 2) ? -term : term;
    }
    const long double pref = std::sqrt(delta2(a, b, c) * delta2(a, e, f) * delta2(d, b, f) * delta2(d, e, c));
    return static_cast<double>(pref * sum);
}

double fmove_coeff(int tA, int tB, int tC, int tJ, int tD, int tE) {
    const double s6 = sixj(tA, tB, tD, tC, tJ, tE);
    if (s6 == 0.0) return 0.0;
    const int ph = (tA + tB + tC + tJ) / 2;
    return ((ph % 2) ? -1.0 : 1.0) * std::sqrt(static_cast<double>((tD + 1) * (tE + 1))) * s6;
}

}  // namespace sym

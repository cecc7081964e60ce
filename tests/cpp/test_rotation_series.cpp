// Host check of the rotation factors used by the kernels' update (exact Rodrigues
// rotation, Section 3.2.3): for th^2 in [0, 1) the series st = sin(th)/th and
// c1 = (1 - cos th)/th^2 must agree with the trigonometric definitions, evaluated in long
// double, to within 2 units in the last place of the type (FP32 and FP64).
#include "fit_device.h"

#include <cmath>
#include <cstdio>
#include <limits>

template <typename T>
static int check(const char* name) {
    const long double ulp = std::numeric_limits<T>::epsilon();
    int bad = 0;
    long double worst_s = 0, worst_c = 0;
    for (int i = 0; i < 4096; ++i) {
        // dense near 0 (the late iterations) and up to just below 1
        const T th2 = i < 2048 ? T(std::ldexp(double(i), -40)) : T((i - 2048) / 2048.0);
        if (!(th2 < T(1))) continue;
        T st, c1;
        qc::rotation_series(th2, st, c1);
        const long double th = sqrtl((long double)th2);
        const long double s_ref = th > 0 ? sinl(th) / th : 1.0L;
        const long double h = sinl(th / 2);
        const long double c_ref = th > 0 ? 2 * h * h / (th * th) : 0.5L;
        const long double es = fabsl(st - s_ref) / s_ref / ulp, ec = fabsl(c1 - c_ref) / c_ref / ulp;
        worst_s = es > worst_s ? es : worst_s;
        worst_c = ec > worst_c ? ec : worst_c;
        if (es > 2 || ec > 2) {
            if (bad < 5) std::printf("%s th2=%.9g st=%.17g (ref %.17Lg) c1=%.17g (ref %.17Lg)\n", name,
                                     double(th2), double(st), s_ref, double(c1), c_ref);
            ++bad;
        }
    }
    std::printf("%s worst %.2Lf / %.2Lf ulp\n", name, worst_s, worst_c);
    return bad;
}

int main() {
    const int bad = check<float>("fp32") + check<double>("fp64");
    std::printf(bad ? "FAIL\n" : "OK\n");
    return bad ? 1 : 0;
}

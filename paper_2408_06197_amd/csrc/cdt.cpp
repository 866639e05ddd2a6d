// Cumulative table of the rounded Gaussian error (sigma = 3.2, support
// [-19, 19]) in binary128 arithmetic.  Entry k is floor(2^64 * P(X <= k - 19))
// for k = 0..37; the threshold of t = 19 is 2^64 and stays implicit.  The
// paper leaves X_err open (Methods, CKKS Scheme Description); sigma 3.2 is the
// workload's.  Built with g++ (quadmath).
#include <quadmath.h>
#include <stdint.h>

namespace lc {

void cdt_thresholds(uint64_t out[38])
{
    const int tail = 19;
    __float128 sigma = 32;
    sigma /= 10;
    __float128 two_s2 = 2 * sigma * sigma;
    __float128 rho[2 * tail + 1], total = 0;
    for (int t = -tail; t <= tail; t++) {
        rho[t + tail] = expq(-((__float128)t * t) / two_s2);
    }
    // sum smallest terms first
    for (int t = tail; t >= 0; t--) {
        total += rho[t + tail];
        if (t) total += rho[-t + tail];
    }
    __float128 two64 = ldexpq(1, 64), acc = 0;
    for (int k = 0; k < 2 * tail; k++) {
        acc += rho[k];
        __float128 v = floorq(acc / total * two64);
        out[k] = (uint64_t)v;
    }
}

}  // namespace lc

"""Coefficients of the FP64 scaled complementary error function used by the
FP64 walk: erfcx(u) = exp(u^2) erfc(u) on 0 <= u <= 3 as a polynomial of
degree 25 in t = 2u/3 - 1, fitted by Chebyshev interpolation in 40-digit
arithmetic (mpmath) and printed in Horner order (highest degree first).
Evaluated in FP64 by Horner's rule its relative error is below 1e-15 on the
interval.  Usage: python gen_erfcx64.py  (prints the C++ initialiser)."""
import mpmath as mp

U = 3
TERMS = 26


def scaled_erfc(t):
    u = U * (t + 1) / 2
    return mp.erfc(u) * mp.exp(u * u)


def main():
    mp.mp.dps = 40
    poly, err = mp.chebyfit(scaled_erfc, [-1, 1], TERMS, error=True)
    print("// fit error %.1e" % float(err))
    print("constexpr double kErfcx64[%d] = {" % TERMS)
    for i in range(0, TERMS, 3):
        print("    " + ", ".join("%.17g" % float(a) for a in poly[i:i + 3]) + ",")
    print("};")


if __name__ == "__main__":
    main()

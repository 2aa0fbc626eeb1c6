"""Prints the Taylor coefficients of 1/Gamma(1+z) about z = 0 (40 digits).

Used once to produce the kRGamma table in matern.hip (the coefficients of
Abramowitz & Stegun 6.1.34, shifted by one index).  Needs mpmath.
"""
import mpmath as mp

if __name__ == "__main__":
    mp.mp.dps = 40
    for k, v in enumerate(mp.taylor(lambda z: 1 / mp.gamma(1 + z), 0, 25)):
        print(f"    {mp.nstr(v, 20)},  // a_{k}")

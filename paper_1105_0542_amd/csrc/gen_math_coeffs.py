"""Print the FP64 constants of pimc_math.hpp, each rounded once to nearest from its exact value.

  LOG_P[k]  = 2/(2k+3)                    ln m = 2s + s^3 * sum_k LOG_P[k] s^(2k),  s = (m-1)/(m+1)
  SIN_C[i]  = (-1)^i (2 pi)^(2i+1)/(2i+1)!  sin(2 pi r) = r * sum_i SIN_C[i] r^(2i)
  COS_C[i]  = (-1)^i (2 pi)^(2i)/(2i)!      cos(2 pi r) = sum_i COS_C[i] r^(2i)
  LN2_HI + LN2_LO = ln 2, LN2_HI with 21 trailing zero bits (E*LN2_HI exact for |E| < 2^21)
Usage: python gen_math_coeffs.py
"""
import mpmath as mp

mp.mp.prec = 200


def hexd(x):
    return float(x).hex()


def main():
    print("// LOG_P[k] = 2/(2k+3), k = 0..9")
    print(", ".join(hexd(mp.mpf(2) / (2 * k + 3)) for k in range(10)))
    tp = 2 * mp.pi
    print("// SIN_C[i] = (-1)^i (2pi)^(2i+1)/(2i+1)!, i = 0..8")
    print(", ".join(hexd((-1) ** i * tp ** (2 * i + 1) / mp.factorial(2 * i + 1)) for i in range(9)))
    print("// COS_C[i] = (-1)^i (2pi)^(2i)/(2i)!, i = 0..9")
    print(", ".join(hexd((-1) ** i * tp ** (2 * i) / mp.factorial(2 * i)) for i in range(10)))
    ln2 = mp.log(2)
    hi = mp.mpf(int(mp.floor(ln2 * 2 ** 32))) / 2 ** 32          # 32 significant bits
    lo = ln2 - hi
    print("// LN2_HI, LN2_LO")
    print(hexd(hi), hexd(lo))
    print("// SQRT_HALF (rounded)")
    print(hexd(mp.sqrt(mp.mpf(1) / 2)))


if __name__ == "__main__":
    main()

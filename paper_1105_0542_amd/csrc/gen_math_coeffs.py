"""Print the FP64 constants of pimc_math.hpp, each rounded once to nearest from its exact value.

  LOG_P[k]  = 2/(2k+3)                    ln m = 2s + s^3 * sum_k LOG_P[k] s^(2k),  s = (m-1)/(m+1)
  SIN_C[i]  = (-1)^i (2 pi)^(2i+1)/(2i+1)!  sin(2 pi r) = r * sum_i SIN_C[i] r^(2i)
  COS_C[i]  = (-1)^i (2 pi)^(2i)/(2i)!      cos(2 pi r) = sum_i COS_C[i] r^(2i)
  LN2_HI + LN2_LO = ln 2, LN2_HI with 21 trailing zero bits (E*LN2_HI exact for |E| < 2^21)
  BM_LOG_P[n-1] = 2 (-1)^n / n, n = 1..8      -2 log1p(r) = r * sum_n BM_LOG_P[n-1] r^(n-1), |r| <= 1/128
  BM_SIN[i] = (-1)^i (2 pi 2^-53)^(2i+1)/(2i+1)!, i = 0..3   sin(2 pi J 2^-53) = J * sum_i BM_SIN[i] J^(2i)
  BM_COS[i] = (-1)^(i+1) (2 pi 2^-53)^(2i+2)/(2i+2)!, i = 0..3   cos(2 pi J 2^-53) - 1 = J^2 * sum_i BM_COS[i] J^(2i)
  BM_TABLE: 64 log entries {1/c_i rounded, -2 T_i} then 64 angle entries {sin, cos}(2 pi k / 64)
    (c_i = 1 + (i + 1/2)/64; T_i = -ln(1/c_i rounded), minus ln 2 for i >= 27; entry 63 is {1/2, 0})
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
    print("// -2 LN2_HI, -2 LN2_LO")
    print(hexd(-2 * hi), hexd(-2 * lo))
    print("// BM_LOG_P[n-1] = 2 (-1)^n / n, n = 1..8")
    print(", ".join(hexd(mp.mpf(2) * (-1) ** n / n) for n in range(1, 9)))
    x = 2 * mp.pi * mp.mpf(2) ** -53
    print("// BM_SIN[i], i = 0..3")
    print(", ".join(hexd((-1) ** i * x ** (2 * i + 1) / mp.factorial(2 * i + 1)) for i in range(4)))
    print("// BM_COS[i], i = 0..3")
    print(", ".join(hexd((-1) ** (i + 1) * x ** (2 * i + 2) / mp.factorial(2 * i + 2)) for i in range(4)))
    print("// BM_TABLE: log entries {inv, A}, i = 0..63")
    ent = []
    for i in range(64):
        if i == 63:
            inv, A = mp.mpf(1) / 2, mp.mpf(0)
        else:
            c = 1 + (mp.mpf(i) + mp.mpf(1) / 2) / 64
            inv = mp.mpf(float(1 / c))                      # rounded once to FP64
            T = -mp.log(inv) - (ln2 if i >= 27 else 0)
            A = -2 * T
        ent += [hexd(inv), hexd(A)]
    print(", ".join(ent))
    print("// BM_TABLE: angle entries {sin, cos}(2 pi k / 64), k = 0..63")
    ent = []
    for k in range(64):
        a = 2 * mp.pi * k / 64
        ent += [hexd(mp.sin(a)), hexd(mp.cos(a))]
    print(", ".join(ent))


if __name__ == "__main__":
    main()

"""Writes the closed-form fixtures under tests/golden/ (plain math; no project code).

ridge_penumbra.txt: flat plane with a one-texel straight ridge of height h_r
lit along the ridge normal.  A point at horizontal distance x before the crest
sees the crest at elevation atan(h_r/x); the sun centre is at elevation e, so
the angular clearance is e - atan(h_r/x) and the visible part of the sun disc
(radius r_L) is the circular-segment fraction S(d) with d = clearance/r_L
(Sec. 3.4, Eq. 5-6, circular segment).  The umbra ends where the clearance is
-r_L, i.e. x = h_r/tan(e + r_L); full light begins at x = h_r/tan(e - r_L).

disc_fraction.txt: S(d) = (pi - acos d + d sqrt(1 - d^2))/pi, the part of a unit
disc above a chord at signed distance d below the centre, tabulated by
integrating the chord length 2 sqrt(1 - y^2) from y = -d to 1 (scipy quad).
"""
import math
import os

from scipy.integrate import quad

HERE = os.path.dirname(os.path.abspath(__file__))
RL = math.radians(0.267)


def main():
    with open(os.path.join(HERE, "ridge_penumbra.txt"), "w") as f:
        f.write("# straight-ridge penumbra on a plane (Sec. 3.4 circular segment)\n")
        f.write("# elev_deg h_r_m umbra_end_m light_begin_m width_m\n")
        for e_deg in (1.5, 3.0):
            e = math.radians(e_deg)
            for hr in (100.0,):
                a = hr / math.tan(e + RL)
                b = hr / math.tan(e - RL)
                f.write(f"{e_deg:.1f} {hr:.1f} {a:.6f} {b:.6f} {b - a:.6f}\n")
    with open(os.path.join(HERE, "disc_fraction.txt"), "w") as f:
        f.write("# visible fraction of a unit disc above a chord at distance d below its centre\n")
        f.write("# d  fraction (numerical integral of chord length / pi)\n")
        for k in range(-10, 11):
            d = k / 10.0
            val, _ = quad(lambda y: 2.0 * math.sqrt(max(0.0, 1.0 - y * y)), -d, 1.0,
                          epsabs=1e-13, epsrel=1e-13, limit=200)
            f.write(f"{d:+.1f} {val / math.pi:.15f}\n")


if __name__ == "__main__":
    main()

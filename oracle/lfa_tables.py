"""The paper's LFA numbers recomputed at the paper's sampling step.

Test infrastructure (see the package header): prints, for the paper's own
LFA smoother (lexicographic economic Vanka, `lfa.LexVanka`) under its
scalar smoothing-symbol reading, Table 1 (Section 5.1) and the statements
of Section 4.3 (Figures 3 and 4) beside the printed values, and the
two-grid factor of the whole sweep symbol and of the production red-black
full-Vanka smoother for comparison.  Run as `python -m oracle.lfa_tables
[step]` from the repository root (step 0.01 rad as in the paper: a few
minutes on one core); `python -m oracle.lfa_tables 3d [step]` prints the
3D tuning table (`tune_3d`).
"""
import sys

import numpy as np

from . import lfa

H = 1 / 1024
MEDIA = dict(gamma=0.0, lam=500.0, mu=1.0, rho=1.0)


def _lfa(beta, w, alpha, omega, smoother="lex-economic", scalar=True):
    return lfa.LFA(2, h=H, omega=omega, beta=beta, alpha=alpha, w=w, smoother=smoother,
                   scalar_smoother=scalar, **MEDIA)


def main(step):
    print("Table 1 (lambda 500, mu = rho = 1, h = 1/1024; sampled every %g rad)" % step)
    print("beta  w     omega     alpha | rho_loc paper-reading (printed) | whole-symbol | red-black full"
          " | mu_loc^2 (printed)")
    printed = {1.0: ((0.73, 0.81, 0.75), (0.35, 0.38, 0.44)), 2 / 3: ((0.37, 0.40, 0.47), (0.31, 0.34, 0.39))}
    for beta, w in ((1.0, 0.75), (2 / 3, 0.65)):
        for i, (od, a) in enumerate(((5, 0.15), (4, 0.2), (3.3, 0.3))):
            om = np.pi / (od * H)
            r = _lfa(beta, w, a, om).rho_loc(step=step)
            r0 = _lfa(beta, w, a, om, scalar=False).rho_loc(step=step)
            rb = _lfa(beta, w, a, om, smoother="red-black", scalar=False).rho_loc(step=max(step, 0.05))
            m = _lfa(beta, w, a, om).mu_loc(step=step)
            print("%.3f %.2f  pi/%.1fh  %.2f  | %.3f (%.2f) | %.3f | %.3f | %.3f (%.2f)"
                  % (beta, w, od, a, r, printed[beta][0][i], r0, rb, m * m, printed[beta][1][i]), flush=True)
    om10 = 2 * np.pi / (10 * H)
    print("Figure 3(a), alpha 0.1, 10 points per wavelength: mu_loc over w")
    for beta in (2 / 3, 1.0):
        ws = np.round(np.arange(0.55, 0.851, 0.05), 2)
        mus = [_lfa(beta, w, 0.1, om10).mu_loc(step=step) for w in ws]
        print("  beta %.3f: " % beta + " ".join("%.2f:%.3f" % x for x in zip(ws, mus)), flush=True)
    print("Figure 3(b), alpha 0.1, w 0.7: rho_loc over beta (paper-reading)")
    for ppw in (10, 8):
        bs = np.round(np.arange(0.5, 1.001, 0.02), 2)
        rs = [_lfa(b, 0.7, 0.1, 2 * np.pi / (ppw * H)).rho_loc(step=max(step, 0.02)) for b in bs]
        i = int(np.argmin(rs))
        print("  %d points per wavelength: min %.3f at beta %.2f" % (ppw, rs[i], bs[i]), flush=True)
    print("Figure 4(a), 10 points per wavelength, w 0.7: rho_loc over alpha")
    for beta in (2 / 3, 1.0):
        al = (0.02, 0.03, 0.04, 0.1, 0.11, 0.12, 0.13)
        print("  beta %.3f: " % beta + " ".join("%.2f:%.2f" % (a, _lfa(beta, 0.7, a, om10).rho_loc(step=max(step, 0.02)))
                                           for a in al), flush=True)
    print("Figure 4(b), alpha 0.1, w 0.7: rho_loc over points per wavelength")
    for beta in (2 / 3, 1.0):
        pp = (6.0, 6.5, 7.0, 10.0, 10.5, 11.0, 12.0)
        print("  beta %.3f: " % beta + " ".join(
            "%.1f:%.2f" % (p, _lfa(beta, 0.7, 0.1, 2 * np.pi / (p * H)).rho_loc(step=max(step, 0.02))) for p in pp),
            flush=True)


def tune_3d(step):
    """3D two-grid factors over beta (the paper leaves 3D tuning open,
    Section 5.3): the production red-black full-Vanka cycle and the
    lexicographic economic sweep, whole symbols, lambda 500, mu = rho = 1"""
    h = 1 / 256
    betas = (0.3, 0.4, 0.5, 0.6, 2 / 3, 0.7, 0.8, 0.9, 1.0)
    print("3D rho_loc over beta (sampled every %g rad)" % step)
    for smoother, w in (("red-black", 0.6), ("red-black", 0.7), ("lex-economic", 0.65)):
        for ppw, alpha in ((10, 0.15), (8, 0.15), (10, 0.3)):
            rs = [lfa.LFA(3, h=h, omega=2 * np.pi / (ppw * h), beta=b, alpha=alpha, w=w, smoother=smoother,
                          **MEDIA).rho_loc(step=step) for b in betas]
            print("  %-12s w %.2f  %2d ppw alpha %.2f: " % (smoother, w, ppw, alpha)
                  + " ".join("%.2f:%.3f" % x for x in zip(betas, rs)), flush=True)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "3d":
        tune_3d(float(sys.argv[2]) if len(sys.argv) > 2 else 0.2)
    else:
        main(float(sys.argv[1]) if len(sys.argv) > 1 else 0.01)

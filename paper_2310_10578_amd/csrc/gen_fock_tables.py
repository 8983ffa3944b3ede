"""Generate the piecewise-polynomial Fock-function tables of the GPU library.

The creeping-wave and reflection coefficients of the off-surface UTD (the
transfer and reflection dyadics of Eqs. (3)-(4), Pathak-Burnside-Marhefka
1980) need the soft/hard Pekeris functions p*_s, p*_h and the Kouyoumjian-
Pathak transition function F(X).  The device code evaluates them from short
polynomial pieces held in LDS; this script computes those pieces once, with
multiple-precision arithmetic (mpmath), and writes ``fock_tables.h``.

Functions tabulated (xi real):
  PT : Ptilde_p(xi) = p*_p(xi) + e^{-j pi/4}/(2 sqrt(pi) xi)       xi in [PT_LO, PT_HI]
  DS : p*_p(xi) itself (the creeping-wave modes)                   xi in [PT_HI, DS_HI]
  CL : c_p(t) = sqrt(-4/xi) e^{-j xi^3/12} p*_p(xi), t = (PT_LO/xi)^3 in (0, 1]
  FA : G(u) = F(X)/sqrt(X) = 2j A(u),
       A(u) = e^{j u^2} Int_u^inf e^{-j s^2} ds                     u in [0, FA_HI]
  FH : -H(v) = (1 - F(X)) X, v = 1/X                              v in [0, 1/FA_HI^2]
with F(X) = 2j sqrt(X) A(sqrt(X)), u = sqrt(X).

Evaluation routes (multiple precision, 30 digits):
  * PT: the Fourier integral split at t = 0; t > 0 on the real axis with
    V/W2, t < 0 rotated onto t = -r e^{j pi/6} where -(j/2) W1/W2 decays;
    composite Gauss-Legendre nodes, Airy functions from mpmath.
  * DS: residue series over 60 zeros of Ai (soft) or Ai' (hard), from
    mpmath.airyaizero.
  * CL: p* as the full-line integral of -(j/2) W1/W2 e^{-j xi t}, moved onto
    the steepest-descent line through the saddle t = -xi^2/4, composite
    Gauss-Legendre panels scaled with sqrt(|xi|).
  * FA/FH: A(u) = (sqrt(pi)/2) e^{-j pi/4} e^{j u^2} erfc(e^{j pi/4} u).

Each piece is a degree-DEG polynomial fitted by Chebyshev interpolation (at
DEG+1 Chebyshev points) and stored as monomial coefficients for Horner
evaluation: in s = 2 (w - j) - 1 in [-1, 1] for the double set (FP64 kernel),
in sigma = w - j in [0, 1) for the float set (FP32 kernel: one operation less
per lookup; at degree 4 the shifted basis rounds no worse in FP32).  The script prints
the maximum error of every table on a dense check grid.

Layout.  The device locates a segment with one affine map, so the pieces are
laid out on a common index axis w (segment j covers w in [j, j + 1], s =
2 (w - j) - 1):
  regime table  [CL | PT | DS]:  w = NCL t for xi < PT_LO (t = (PT_LO/xi)^3),
                w = NCL + RW (xi - PT_LO) for xi >= PT_LO, PT and DS sharing
                the width 1/RW, so one map covers both;
  transition    [FA | FH]:       w = NT u / FA_HI for u < FA_HI,
                w = 2 NT - NT FA_HI^2 / X beyond (FH stored with its
                variable reversed, so w grows with u across the junction).
(s or sigma above is the local variable of segment j = floor(w).)
Run:  python gen_fock_tables.py  (takes a few minutes)
"""
import os
import sys

import mpmath as mp
import numpy as np

mp.mp.dps = 30
HERE = os.path.dirname(os.path.abspath(__file__))

PT_LO, PT_HI = -3.0, 2.0
DS_HI = 24.0
FA_HI = 4.0

# per precision: polynomial degree, regime segments per unit xi (PT and DS),
# deep-lit segments, transition segments (FA and FH each)
LAYOUT = {
    "f32": dict(deg=4, rw=8, ncl=16, nt=32),
    "f64": dict(deg=11, rw=8, ncl=32, nt=32),
}

SQPI = mp.sqrt(mp.pi)
EM4 = mp.exp(-1j * mp.pi / 4)
W3 = mp.exp(2j * mp.pi / 3)


# ---------------------------------------------------------------------------
# Fock-Airy functions (multiple precision)
# ---------------------------------------------------------------------------

def V(t):
    return SQPI * mp.airyai(t), SQPI * mp.airyai(t, derivative=1)


def W1(t):
    c = 2 * SQPI * mp.exp(1j * mp.pi / 6)
    z = t * W3
    return c * mp.airyai(z), c * W3 * mp.airyai(z, derivative=1)


def W2(t):
    c = 2 * SQPI * mp.exp(-1j * mp.pi / 6)
    z = t / W3
    return c * mp.airyai(z), c / W3 * mp.airyai(z, derivative=1)


# ---------------------------------------------------------------------------
# Ptilde by contour quadrature with cached integrand values
# ---------------------------------------------------------------------------

_pt_cache = None


def _gl_panels(a, b, width, n):
    x, w = np.polynomial.legendre.leggauss(n)
    edges = np.linspace(a, b, int(round((b - a) / width)) + 1)
    pts, wts = [], []
    for lo, hi in zip(edges[:-1], edges[1:]):
        pts.extend((hi - lo) / 2 * x + (hi + lo) / 2)
        wts.extend((hi - lo) / 2 * w)
    return np.array(pts), np.array(wts)


def _pt_nodes():
    global _pt_cache
    if _pt_cache is not None:
        return _pt_cache
    psi = mp.pi / 6
    e = mp.exp(1j * psi)
    t, wt = _gl_panels(0.0, 14.0, 0.25, 24)
    r, wr = _gl_panels(0.0, 20.0, 0.25, 24)
    gs, gh, hs, hh = [], [], [], []
    for ti in t:
        v, vp = V(mp.mpf(ti))
        w2, w2p = W2(mp.mpf(ti))
        gs.append(complex(v / w2))
        gh.append(complex(vp / w2p))
    for ri in r:
        tau = -mp.mpf(ri) * e
        w1, w1p = W1(tau)
        w2, w2p = W2(tau)
        hs.append(complex(-0.5j * w1 / w2 * e))
        hh.append(complex(-0.5j * w1p / w2p * e))
    ec = complex(e)
    _pt_cache = dict(t=t, wt=wt, r=r, wr=wr, gs=np.array(gs), gh=np.array(gh),
                     hs=np.array(hs), hh=np.array(hh), e=ec)
    return _pt_cache


def ptilde(xi):
    """(Ptilde_s, Ptilde_h) at real xi in [PT_LO, PT_HI]."""
    c = _pt_nodes()
    k1 = np.exp(-1j * xi * c["t"]) * c["wt"]
    k2 = np.exp(1j * xi * c["r"] * c["e"]) * c["wr"]
    pre = complex(EM4 / SQPI)
    s = pre * (np.sum(c["gs"] * k1) + np.sum(c["hs"] * k2))
    h = pre * (np.sum(c["gh"] * k1) + np.sum(c["hh"] * k2))
    return s, h


# ---------------------------------------------------------------------------
# Residue series
# ---------------------------------------------------------------------------

NRES = 60
_res = None


def residues():
    global _res
    if _res is None:
        rot = mp.exp(-5j * mp.pi / 6)
        pre = -mp.exp(-1j * mp.pi / 12) / (2 * SQPI)
        zs, ws, zh, wh = [], [], [], []
        for n in range(1, NRES + 1):
            a = -mp.airyaizero(n)                  # alpha_n > 0
            b = -mp.airyaizero(n, derivative=1)    # beta_n > 0
            zs.append(a * rot)
            ws.append(pre / mp.airyai(-a, derivative=1) ** 2)
            zh.append(b * rot)
            wh.append(pre / (b * mp.airyai(-b) ** 2))
        _res = (zs, ws, zh, wh)
    return _res


def dshadow(xi):
    """(p*_s, p*_h) at xi >= PT_HI from the residue series."""
    zs, ws, zh, wh = residues()
    x = mp.mpf(xi)
    s = mp.fsum(w * mp.exp(z * x) for z, w in zip(zs, ws))
    h = mp.fsum(w * mp.exp(z * x) for z, w in zip(zh, wh))
    return complex(s), complex(h)


# ---------------------------------------------------------------------------
# Deep lit: steepest-descent line
# ---------------------------------------------------------------------------

def clit_xi(xi):
    """(c_s, c_h) at xi < 0 via the full-line integral on the saddle line
    t = -xi^2/4 + v e^{j pi/4}.  Near the saddle the integrand is Gaussian
    with width of order sqrt(|xi|) in v; composite Gauss-Legendre panels cover
    [-10 w, 60 w] with w = sqrt(|xi|) (upper-right tail decays like
    exp(-|xi| v / sqrt 2), lower-left super-exponentially)."""
    x = mp.mpf(xi)
    s0 = x * x / 4
    e = mp.exp(1j * mp.pi / 4)
    phase0 = x ** 3 / 12
    w = mp.sqrt(abs(x))
    gx, gw = np.polynomial.legendre.leggauss(24)
    edges = [-10, -6, -4, -3, -2, -1.5, -1, -0.5, 0, 0.5, 1, 1.5, 2, 3, 4, 6, 10, 16, 24, 36, 60]
    acc_s = mp.mpc(0)
    acc_h = mp.mpc(0)
    for lo, hi in zip(edges[:-1], edges[1:]):
        for xx, ww in zip(gx, gw):
            v = w * (mp.mpf(hi - lo) / 2 * mp.mpf(xx) + mp.mpf(hi + lo) / 2)
            wt = w * mp.mpf(hi - lo) / 2 * mp.mpf(ww)
            tau = -s0 + v * e
            w1, w1p = W1(tau)
            w2, w2p = W2(tau)
            ex = mp.exp(-1j * x * tau - 1j * phase0) * e * wt * (-0.5j)
            acc_s += w1 / w2 * ex
            acc_h += w1p / w2p * ex
    pre = mp.sqrt(-4 / x) * EM4 / SQPI
    return complex(pre * acc_s), complex(pre * acc_h)


def clit_t(t):
    xi = PT_LO / mp.cbrt(mp.mpf(t))
    return clit_xi(xi)


# ---------------------------------------------------------------------------
# Transition function pieces
# ---------------------------------------------------------------------------

def A_of_u(u):
    u = mp.mpf(u)
    return complex(SQPI / 2 * EM4 * mp.exp(1j * u * u) * mp.erfc(mp.exp(1j * mp.pi / 4) * u))


def H_of_v(v):
    if v == 0:
        return 0.5j
    v = mp.mpf(v)
    u = 1 / mp.sqrt(v)
    A = SQPI / 2 * EM4 * mp.exp(1j * u * u) * mp.erfc(mp.exp(1j * mp.pi / 4) * u)
    F = 2j * u * A
    return complex((F - 1) / v)


# ---------------------------------------------------------------------------
# Fitting
# ---------------------------------------------------------------------------

def _call(args):
    name, x = args
    return FUNS[name][0](x)


def build_table(name, lo, hi, nseg, deg, pool):
    """Chebyshev interpolation (DEG+1 points) on each of nseg equal segments,
    converted to monomial coefficients in s in [-1, 1] for Horner."""
    n = deg + 1
    s = np.cos(np.pi * (np.arange(n) + 0.5) / n)
    edges = np.linspace(lo, hi, nseg + 1)
    xs = [(edges[i] + edges[i + 1]) / 2 + (edges[i + 1] - edges[i]) / 2 * s for i in range(nseg)]
    vals = pool.map(_call, [(name, float(x)) for seg in xs for x in seg])
    vals = np.array(vals).reshape(nseg, n, -1)
    V = np.polynomial.chebyshev.chebvander(s, deg)
    segs = []
    for i in range(nseg):
        cheb = np.linalg.solve(V, vals[i])
        cols = []
        for j in range(vals.shape[2]):
            mono = np.polynomial.chebyshev.cheb2poly(cheb[:, j])
            cols.append(np.pad(mono, (0, deg + 1 - mono.size)))
        segs.append(np.array(cols).T)
    return np.array(segs)   # (nseg, deg+1, nfun) complex


def to_sigma(tab):
    """Monomial coefficients in s in [-1, 1] -> in sigma = (s + 1)/2 in [0, 1]."""
    out = np.zeros_like(tab)
    for k in range(tab.shape[1]):
        c = np.polynomial.polynomial.polypow([-1.0, 2.0], k)   # (2 sigma - 1)^k
        for m in range(k + 1):
            out[:, m, :] += tab[:, k, :] * c[m]
    return out


def eval_table(tab, lo, hi, x, dtype, sigma=False):
    nseg = tab.shape[0]
    w = (hi - lo) / nseg
    idx = np.clip(np.floor((x - lo) / w).astype(int), 0, nseg - 1)
    s = (x - lo) / w - idx
    if not sigma:
        s = s * 2 - 1
    s = s.astype(dtype)
    out = np.zeros((x.size, tab.shape[2]), complex)
    for j in range(tab.shape[2]):
        re = tab[idx, -1, j].real.astype(dtype)
        im = tab[idx, -1, j].imag.astype(dtype)
        for k in range(tab.shape[1] - 2, -1, -1):
            re = re * s + tab[idx, k, j].real.astype(dtype)
            im = im * s + tab[idx, k, j].imag.astype(dtype)
        out[:, j] = re.astype(float) + 1j * im.astype(float)
    return out


def _fa(u):
    return (2j * A_of_u(u),)


def _fh(v):
    return (H_of_v(v),)


def _fhr(r):
    # -H on the reversed variable r = 1 - FA_HI^2 / X in [0, 1]
    return (-H_of_v((1.0 - r) / FA_HI ** 2),)


FUNS = {
    "PT": (ptilde, PT_LO, PT_HI),
    "DS": (dshadow, PT_HI, DS_HI),
    "CL": (clit_t, 0.0, 1.0),
    "FA": (_fa, 0.0, FA_HI),
    "FH": (_fh, 0.0, 1.0 / FA_HI ** 2),
    "FHR": (_fhr, 0.0, 1.0),
}


def check(name, tab, prec, pool, npts=41):
    fn, lo, hi = FUNS[name]
    x = lo + (hi - lo) * (np.arange(npts) + 0.37) / npts
    ref = np.array(pool.map(_call, [(name, float(xx)) for xx in x]))
    got = eval_table(tab, lo, hi, x, np.float32 if prec == "f32" else np.float64, sigma=(prec == "f32"))
    return np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-3))


def emit_array(fh, cname, tab, ctype):
    """tab (nseg, deg+1, nfun complex) -> C array [nseg][deg+1][2*nfun] of
    (re, im) pairs per function."""
    nseg, nc, nf = tab.shape
    fh.write("FT_QUAL %s %s[%d][%d][%d] = {\n" % (ctype, cname, nseg, nc, 2 * nf))
    fmt = "%.9e" if ctype == "float" else "%.17e"
    suf = "f" if ctype == "float" else ""
    for i in range(nseg):
        fh.write("  {")
        for k in range(nc):
            vals = []
            for j in range(nf):
                vals += [tab[i, k, j].real, tab[i, k, j].imag]
            fh.write("{" + ",".join((fmt % v) + suf for v in vals) + "}" + ("," if k < nc - 1 else ""))
        fh.write("}%s\n" % ("," if i < nseg - 1 else ""))
    fh.write("};\n")


def emit_concat(fh, cname, tabs, ctype):
    """Concatenate tables along the segment axis and emit them as one array."""
    emit_array(fh, cname, np.concatenate(tabs, axis=0), ctype)


def main(out_path):
    import multiprocessing as mproc
    zs, ws, zh, wh = residues()
    _pt_nodes()
    tables = {}
    report = []
    with mproc.get_context("fork").Pool(min(8, os.cpu_count() or 1)) as pool:
        for prec, lay in LAYOUT.items():
            deg, rw, ncl, nt = lay["deg"], lay["rw"], lay["ncl"], lay["nt"]
            npt = int(round(rw * (PT_HI - PT_LO)))
            nds = int(round(rw * (DS_HI - PT_HI)))
            assert npt == rw * (PT_HI - PT_LO) and nds == rw * (DS_HI - PT_HI)
            lay.update(npt=npt, nds=nds)
            for name, nseg in (("CL", ncl), ("PT", npt), ("DS", nds), ("FA", nt), ("FHR", nt)):
                fn, lo, hi = FUNS[name]
                tab = build_table(name, lo, hi, nseg, deg, pool)
                if prec == "f32":
                    tab = to_sigma(tab)
                err = check(name, tab, prec, pool, npts=397)
                report.append("%s %s nseg=%d deg=%d max rel err %.2e" % (prec, name, nseg, deg, err))
                print(report[-1], flush=True)
                tables[(prec, name)] = tab
    with open(out_path, "w") as fh:
        fh.write("// Generated by gen_fock_tables.py -- do not edit.\n")
        fh.write("// Piecewise polynomials (Horner in s in [-1,1] per segment) of the\n")
        fh.write("// Pekeris/Fock functions and the transition function; see the generator\n")
        fh.write("// for the functions and the index layout.\n")
        for line in report:
            fh.write("// %s\n" % line)
        fh.write("#pragma once\n")
        fh.write("#ifndef FT_QUAL\n#define FT_QUAL static const\n#endif\n")
        fh.write("#define FT_PT_LO (%.17g)\n#define FT_PT_HI (%.17g)\n" % (PT_LO, PT_HI))
        fh.write("#define FT_DS_HI (%.17g)\n#define FT_FA_HI (%.17g)\n" % (DS_HI, FA_HI))
        for prec, lay in LAYOUT.items():
            P = prec.upper()
            for key in ("deg", "rw", "ncl", "npt", "nds", "nt"):
                fh.write("#define FT_%s_%s %d\n" % (P, key.upper(), lay[key]))
        # first creeping-mode exponents, for xi > DS_HI
        fh.write("#define FT_Z1S_RE (%.17e)\n#define FT_Z1S_IM (%.17e)\n" % (complex(zs[0]).real, complex(zs[0]).imag))
        fh.write("#define FT_Z1H_RE (%.17e)\n#define FT_Z1H_IM (%.17e)\n" % (complex(zh[0]).real, complex(zh[0]).imag))
        for prec in LAYOUT:
            ctype = "float" if prec == "f32" else "double"
            emit_concat(fh, "ft_%s_reg" % prec, [tables[(prec, n)] for n in ("CL", "PT", "DS")], ctype)
            emit_concat(fh, "ft_%s_tf" % prec, [tables[(prec, n)] for n in ("FA", "FHR")], ctype)
    print("wrote", out_path)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(HERE, "fock_tables.h"))

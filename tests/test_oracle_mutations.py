"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle source (on the CPU), builds it, and
checks that at least one pin then fails.  The oracle itself is never modified."""
import os
import subprocess
import tempfile

import pytest

from oracle import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "trips_oracle.c")

MUTATIONS = [
    # (name, original text, planted mistake)
    ("layer weights swapped", "p->iota[0] = 2.0 - t;", "p->iota[0] = t - 1.0;"),
    ("eps rule", "p->iota[0] = eps + (1.0 - eps) * s;", "p->iota[0] = eps + s;"),
    ("texel centre at corner", "float uf = ldexpf((float)p->x, -L) - 0.5f;",
     "float uf = ldexpf((float)p->x, -L);"),
    ("upper layer index", "p->L[1] = e + 1;", "p->L[1] = e + 2;"),
    ("clamp at wrong size", "} else if (s >= smax) {", "} else if (s > 2.0 * smax) {"),
    ("y uses fx", "float y = fmaf(fy, qy, cy);", "float y = fmaf(fx, qy, cy);"),
    ("rotation transposed", "float Xc = fmaf(R[0], Xf, fmaf(R[1], Yf, fmaf(R[2], Zf, t[0])));",
     "float Xc = fmaf(R[0], Xf, fmaf(R[3], Yf, fmaf(R[6], Zf, t[0])));"),
    ("depth order reversed", "if (x->z != y->z) return x->z < y->z ? -1 : 1;",
     "if (x->z != y->z) return x->z > y->z ? -1 : 1;"),
    ("index tie order reversed", "if (x->idx != y->idx) return x->idx < y->idx ? -1 : 1;",
     "if (x->idx != y->idx) return x->idx > y->idx ? -1 : 1;"),
    ("transmittance not updated", "      T = T * (1.0 - f->gamma);\n    }\n    /* an empty list",
     "    }\n    /* an empty list"),
    ("weight drops beta", "f->gamma = ((wx * wy) * p->iota[sel]) * alpha;",
     "f->gamma = p->iota[sel] * alpha;"),
    ("adjoint recurrence sign", "double dgam = Tm[m] * (gm - B);", "double dgam = Tm[m] * (gm + B);"),
    ("adjoint x sign", "double sx = f->di ? 1.0 : -1.0;", "double sx = f->di ? -1.0 : 1.0;"),
    ("chain rule drops size term",
     "gys[p] * fy * q->Yc / Zc + gss[p] * q->s) / Zc;", "gys[p] * fy * q->Yc / Zc) / Zc;"),
    ("size gradient uses fy", "gSW[p] = gss[p] * fx / Zc;", "gSW[p] = gss[p] * fy * 1.5 / Zc;"),
    ("descriptor gradient misses T", "double w = Tm[m] * f->gamma;\n      for (int d = 0; d < D; ++d) gDESC",
     "double w = f->gamma;\n      for (int d = 0; d < D; ++d) gDESC"),
    ("coverage is the transmittance", "if (alpha) alpha[pix] = 1.0 - T;", "if (alpha) alpha[pix] = T;"),
    ("background not behind the list", "pyr[pix * D + d] = col[d] + (bg ? T * bg[pix * D + d] : 0.0);",
     "pyr[pix * D + d] = col[d] + (bg ? bg[pix * D + d] : 0.0);"),
    ("adjoint ignores the background", "      for (int d = 0; d < D; ++d) B += g[d] * bg[pix * D + d];",
     "      for (int d = 0; d < D; ++d) B += 0.0 * bg[pix * D + d];"),
    ("background gradient misses T", "for (int d = 0; d < D; ++d) gbg[pix * D + d] = T * g[d];",
     "for (int d = 0; d < D; ++d) gbg[pix * D + d] = g[d];"),
    ("coverage gradient dropped", "if (Galpha) gm += Galpha[pix];", "if (Galpha) gm += 0.0;"),
    ("rotation gradient transposed", "gcam[3 * r + k] += dX[r] * Xw[k];", "gcam[3 * k + r] += dX[r] * Xw[k];"),
    ("focal gradient drops size term", "gcam[12] += gxs[p] * q->Xc / Zc + gss[p] * sw / Zc;",
     "gcam[12] += gxs[p] * q->Xc / Zc;"),
    ("inclusion: coarser layer first on ties", "if (x->L != y->L) return x->L < y->L ? -1 : 1;",
     "if (x->L != y->L) return x->L > y->L ? -1 : 1;"),
    ("inclusion: wrong covering texel", "int64_t q = base[L + k] + (j >> k) * layer_w(W, L + k) + (i >> k);",
     "int64_t q = base[L + k] + (j >> k) * layer_w(W, L + k) + ((i + 1) >> k);"),
    ("inclusion: parent layer only", "for (int k = 0; L + k < nlayers; ++k) {",
     "for (int k = 0; L + k < nlayers && k < 2; ++k) {"),
    ("inclusion: mask misses ancestors", "if (m[base[L] + j * WL + i]) m[base[L + 1] + (j >> 1) * WP + (i >> 1)] = 1;",
     "if (m[base[L] + j * WL + i]) m[base[L + 1] + (j >> 1) * WP + (i >> 1)] = 0;"),
    ("principal point gradient swapped", "gcam[14] += gxs[p];\n      gcam[15] += gys[p];",
     "gcam[14] += gys[p];\n      gcam[15] += gxs[p];"),
]

PIN_FILES = ["tests/test_oracle_pins.py", "tests/test_oracle_backward.py",
             "tests/test_oracle_extras.py", "tests/test_oracle_coarser.py"]


def _run_pins_with(lib_path):
    """Run the pin tests in a subprocess against the mutated library; True if all pass."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, TRIPS_ORACLE_LIB=lib_path)
    r = subprocess.run(["python", "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + PIN_FILES,
                       cwd=root, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode == 0, r.stdout[-2000:]


@pytest.mark.parametrize("name,orig,mutant", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(name, orig, mutant):
    src = open(SRC).read()
    assert src.count(orig) == 1, "mutation anchor not found: %s" % name
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "mut.c")
        so = os.path.join(d, "libmut.so")
        open(c, "w").write(src.replace(orig, mutant))
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", so, c,
                               "-lm"])
        passed, out = _run_pins_with(so)
    assert not passed, "no pin caught the planted mistake '%s'" % name

"""Plant plausible mistakes in copies of the oracle; the pins must catch each.

Each mutant is a textual change to ``oracle/wilson_oracle.c`` (a dropped term,
a flipped sign, a wrong index, a transposed or un-daggered link, a misplaced
boundary phase, ...), compiled on the CPU into a temporary library. The test
passes when at least one pin in ``tests/pins.py`` fails on the mutant, which
shows the pins are tight enough to notice that class of mistake.
"""
import pytest

import oracle
from tests import pins

# (name, original text, replacement)
MUTANTS = [
    ("forward projector sign", "one_minus[a][b] = d - GAM[mu][a][b];",
     "one_minus[a][b] = d + GAM[mu][a][b];"),
    ("backward projector sign", "one_plus[a][b] = d + GAM[mu][a][b];",
     "one_plus[a][b] = d - GAM[mu][a][b];"),
    ("backward link not daggered", "acc += conj(u[j * 3 + i]) * v[a][j];",
     "acc += u[i * 3 + j] * v[a][j];"),
    ("backward link conjugated only", "acc += conj(u[j * 3 + i]) * v[a][j];",
     "acc += conj(u[i * 3 + j]) * v[a][j];"),
    ("forward link transposed", "acc += u[i * 3 + j] * v[a][j];",
     "acc += u[j * 3 + i] * v[a][j];"),
    ("backward link taken at x", "const cplx *u = U + (sb * 4 + mu) * 9;",
     "const cplx *u = U + (s * 4 + mu) * 9;"),
    ("forward link taken at x+mu", "const cplx *u = U + (s * 4 + mu) * 9;",
     "const cplx *u = U + (sf * 4 + mu) * 9;"),
    ("backward phase not conjugated", "cplx pb = (c[mu] == 0) ? conj(ph[mu]) : 1.0;",
     "cplx pb = (c[mu] == 0) ? ph[mu] : 1.0;"),
    ("forward phase on wrong face", "cplx pf = (c[mu] == L[mu] - 1) ? ph[mu] : 1.0;",
     "cplx pf = (c[mu] == 0) ? ph[mu] : 1.0;"),
    ("backward phase dropped", "cplx pb = (c[mu] == 0) ? conj(ph[mu]) : 1.0;",
     "cplx pb = 1.0;"),
    ("kappa sign", "m[a][i] = own[a][i] - kappa * h[a][i];",
     "m[a][i] = own[a][i] + kappa * h[a][i];"),
    ("time direction dropped",
     "    memset(out, 0, sizeof(cplx) * 12);\n    for (int mu = 0; mu < 4; ++mu) {",
     "    memset(out, 0, sizeof(cplx) * 12);\n    for (int mu = 0; mu < 3; ++mu) {"),
    ("backward neighbour wrong", "cb[mu] = (c[mu] - 1 + L[mu]) % L[mu];",
     "cb[mu] = (c[mu] + 1) % L[mu];"),
    ("gamma lower block sign", "GAM[k][2 + a][b] = I * sigma[k][a][b];",
     "GAM[k][2 + a][b] = -I * sigma[k][a][b];"),
    ("sigma_2 sign", "sigma[1][0][1] = -I; sigma[1][1][0] = I;",
     "sigma[1][0][1] = I; sigma[1][1][0] = -I;"),
    ("dagger misses output gamma5",
     "    if (dagger)\n        spin_apply(GAM5, m, out);\n    else\n        memcpy(out, m, sizeof m);",
     "    memcpy(out, m, sizeof m);"),
    ("eo mask on wrong parity", "hop_site(U, psi, L, ph, s, dagger, out_parity, h);",
     "hop_site(U, psi, L, ph, s, dagger, 1 - out_parity, h);"),
    ("schur kappa not squared", "psi[s * 12 + k] - kappa * kappa * tmp2[s * 12 + k]",
     "psi[s * 12 + k] - kappa * tmp2[s * 12 + k]"),
    ("cg residual update uses p", "r[i] -= alpha * q[i];", "r[i] -= alpha * p[i];"),
    ("cg beta inverted", "double beta = rr_new / rr;", "double beta = rr / rr_new;"),
    ("bicgstab x misses omega s", "x[i] += alpha * p[i] + omega * s[i];",
     "x[i] += alpha * p[i];"),
    ("eo source sign", "bh[i] = even[i / 12] ? b[i] + kappa * w1[i] : 0.0;",
     "bh[i] = even[i / 12] ? b[i] - kappa * w1[i] : 0.0;"),
    ("eo reconstruction sign", "x[i] = even[i / 12] ? xe[i] : b[i] + kappa * w1[i];",
     "x[i] = even[i / 12] ? xe[i] : b[i] - kappa * w1[i];"),
    ("eo normal equations without the adjoint",
     "        schur_into(U, p, t, L, ph, kappa, 0, 0, w1, w2);\n            double pap",
     "        schur_into(U, p, t, L, ph, kappa, 0, 1, w1, w2);\n            double pap"),
    ("twist sign kept in the adjoint",
     "double tw = dagger ? -2.0 * kappa * mu : 2.0 * kappa * mu;",
     "double tw = 2.0 * kappa * mu;"),
    ("twist without its factor 2",
     "double tw = dagger ? -2.0 * kappa * mu : 2.0 * kappa * mu;",
     "double tw = dagger ? -kappa * mu : kappa * mu;"),
    ("twist misses gamma5", "out[a][i] = w[a][i] + I * tw * g5psi[a][i];",
     "out[a][i] = w[a][i] + I * tw * raw[a][i];"),
    ("twisted schur: A^-1 not inverted",
     "(tmp[s * 12 + a * 3 + i] - I * t * g5v[a][i]) / (1.0 + t * t);",
     "(tmp[s * 12 + a * 3 + i] + I * t * g5v[a][i]);"),
    ("twisted schur: twist dropped on psi",
     "? psi[k] + I * t * g5p[a][i] - kappa * kappa * tmp2[k]",
     "? psi[k] - kappa * kappa * tmp2[k]"),
    ("meson: source-side gamma5 on the wrong side",
     "matmul4((const cplx(*)[4])G[n], (const cplx(*)[4])GAM5, B[n]);   /* Gamma g5 */",
     "matmul4((const cplx(*)[4])GAM5, (const cplx(*)[4])G[n], B[n]);   /* Gamma g5 */"),
    ("meson: S not conjugated", "tr_ += conj(S[j][i]) * ASB[j][i];",
     "tr_ += S[j][i] * ASB[j][i];"),
    ("meson: time not counted from t0", "int tr = ((c[3] - t0) % Lt + Lt) % Lt;",
     "int tr = c[3];"),
    ("philox: key schedule constant", "k1 += 0xBB67AE85u;", "k1 += 0xBB67AE86u;"),
    ("kp: cosine not squared", "double l2 = -(log(u[0]) + c * c * log(u[2])) / (2.0 * alpha);",
     "double l2 = -(log(u[0]) + c * log(u[2])) / (2.0 * alpha);"),
    ("x0 draw: disk radius not a square root",
     "double x = sqrt(u[0]) * cos(2.0 * M_PI * u[1]);",
     "double x = u[0] * cos(2.0 * M_PI * u[1]);"),
    ("x0 draw: disk acceptance sign", "if (u[2] <= exp(alpha * (x - 1.0))) {",
     "if (u[2] <= exp(-alpha * (x - 1.0))) {"),
    ("x0 draw: switch to Kennedy-Pendleton too early", "if (alpha < 1.0) {",
     "if (alpha < 0.01) {"),
    ("heatbath: beta not scaled by 2/3",
     "if (kp_draw(2.0 * beta * k / 3.0, (uint32_t)s, tag, sweep, key, &x0) != 0) continue;",
     "if (kp_draw(beta * k, (uint32_t)s, tag, sweep, key, &x0) != 0) continue;"),
    ("heatbath: staple misses its lower half",
     "        su3_dag_mul(m, U + (xmnu * 4 + nu) * 9, t2);\n        for (int k = 0; k < 9; ++k) A[k] += t2[k];",
     "        su3_dag_mul(m, U + (xmnu * 4 + nu) * 9, t2);"),
    ("plaquette misses a conjugate",
     "acc += ab[i * 3 + k] * conj(e[j * 3 + k]);",
     "acc += ab[i * 3 + k] * e[j * 3 + k];"),
    ("site index stride", "return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));",
     "return c[0] + (long)L[0] * (c[1] + (long)L[2] * (c[2] + (long)L[1] * c[3]));"),
]

# cheaper pin arguments for the mutant sweep (same facts, smaller lattices)
FAST = {
    "pin_solvers_lapack": dict(dims=(2, 4, 2, 4), maxiter=400),
    "pin_free_field_solve": dict(dims=(4, 2, 4, 4)),
    "pin_gamma5_hermiticity": dict(dims=(2, 4, 2, 4)),
    "pin_heatbath_unitary_and_strong_coupling": dict(dims=(2, 2, 2, 4)),
    "pin_eo_solve_odd_rows": dict(dims=(2, 2, 4, 4)),
}


def _caught(orc, first=False):
    """Pins that fail on `orc` (with `first`, stop at the first one)."""
    failures = []
    for pin in pins.ALL_PINS:
        try:
            pin(orc, **FAST.get(pin.__name__, {}))
        except Exception as e:  # noqa: BLE001 - any failure counts as caught
            failures.append((pin.__name__, type(e).__name__))
            if first:
                break
    return failures


def test_mutants_are_distinct_edits():
    src = oracle.source_text()
    for name, old, new in MUTANTS:
        assert src.count(old) >= 1, name
        assert old != new


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(tmp_path, name, old, new):
    src = oracle.source_text()
    lib = oracle.compile_copy(src.replace(old, new, 1),
                              str(tmp_path / "liboracle_mutant.so"))
    orc = oracle.Oracle(lib)
    failures = _caught(orc, first=True)
    assert failures, "no pin caught the planted mistake: %s" % name


def test_unmutated_copy_passes_all(tmp_path):
    lib = oracle.compile_copy(oracle.source_text(),
                              str(tmp_path / "liboracle_copy.so"))
    assert _caught(oracle.Oracle(lib)) == []

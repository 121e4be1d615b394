"""Planted mistakes in the oracle: each mutant is the oracle's C source with
one plausible error written in (a flipped sign, a dropped term, a shifted
index, a wrong operand or radius, transposed coefficients, a wrong
normalisation), built with gcc in a temporary directory.  The oracle's pins
(the operator, identity, closed-form and physics checks of the other oracle
test modules) run against the mutant, cheapest first, and at least one of
them must reject it.  The oracle itself is untouched.

The staggered material averages (the face density as the mean of the two
adjacent cells, the shear modulus of an edge node as the harmonic mean of its
four cells) keep the scheme symmetric under the plausible alternatives
written here (energy, reciprocity, skew-adjointness and the transposed step
all still hold), so the physics pins cannot see them; the hand-derived
coefficient values of ``test_oracle_averages`` reject them."""
import concurrent.futures
import gc
import os
import subprocess

import pytest

import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "cwell_oracle.c")

# name: (original text, its replacement), or a list of such pairs for a
# mistake made consistently in two places; each original occurs once in the source
MUTANTS = {
    "azimuthal derivatives of s_rt in v_r and of v_r in g_rt both doubled (a consistent pair)": [
        ("((at(s, srt, i, j, k) - at(s, srt, i, j - 1, k)) / s->dth",
         "((at(s, srt, i, j, k) - at(s, srt, i, j - 1, k)) / (0.5 * s->dth)"),
        ("((at(s, vr, i, j + 1, k) - at(s, vr, i, j, k)) / s->dth",
         "((at(s, vr, i, j + 1, k) - at(s, vr, i, j, k)) / (0.5 * s->dth)")],
    "the same pair doubled in the transposed step as well (consistent throughout)": [
        ("((at(s, srt, i, j, k) - at(s, srt, i, j - 1, k)) / s->dth",
         "((at(s, srt, i, j, k) - at(s, srt, i, j - 1, k)) / (0.5 * s->dth)"),
        ("((at(s, vr, i, j + 1, k) - at(s, vr, i, j, k)) / s->dth",
         "((at(s, vr, i, j + 1, k) - at(s, vr, i, j, k)) / (0.5 * s->dth)"),
        ("  addv(s, vr, i, j + 1, k, c * B / s->dth);\n  addv(s, vr, i, j, k, -c * B / s->dth);",
         "  addv(s, vr, i, j + 1, k, c * B / (0.5 * s->dth));\n  addv(s, vr, i, j, k, -c * B / (0.5 * s->dth));"),
        ("  addv(s, srt, i, j, k, c * B / s->dth);\n  addv(s, srt, i, j - 1, k, -c * B / s->dth);",
         "  addv(s, srt, i, j, k, c * B / (0.5 * s->dth));\n  addv(s, srt, i, j - 1, k, -c * B / (0.5 * s->dth));")],
    "v_r curvature term with the wrong sign": (
        "        - 0.5 * (at(s, stt, i + 1, j, k) + at(s, stt, i, j, k)));",
        "        + 0.5 * (at(s, stt, i + 1, j, k) + at(s, stt, i, j, k)));"),
    "v_theta update without the 2 s_rt / r term": (
        "        + (at(s, srt, i, j, k) + at(s, srt, i - 1, j, k)));",
        "        );"),
    "v_z azimuthal difference shifted by one row": (
        "((at(s, stz, i, j, k) - at(s, stz, i, j - 1, k)) / s->dth",
        "((at(s, stz, i, j + 1, k) - at(s, stz, i, j, k)) / s->dth"),
    "v_z radial difference with the wrong sign": (
        "*Dr = (at(s, srz, i, j, k) - at(s, srz, i - 1, j, k)) / s->dr;",
        "*Dr = (at(s, srz, i - 1, j, k) - at(s, srz, i, j, k)) / s->dr;"),
    "g_rt bracket at the cell-centre radius": (
        "  *B = (1.0 / rf_(s, i)) *\n       ((at(s, vr, i, j + 1, k)",
        "  *B = (1.0 / rc_(s, i)) *\n       ((at(s, vr, i, j + 1, k)"),
    "e_tt curvature term from one face only": (
        "          + 0.5 * (at(s, vr, i, j, k) + at(s, vr, i - 1, j, k)));",
        "          + at(s, vr, i, j, k));"),
    "g_tz depth difference of the wrong field": (
        "  *Dz = (at(s, vt, i, j, k + 1) - at(s, vt, i, j, k)) / s->dz;",
        "  *Dz = (at(s, vz, i, j, k + 1) - at(s, vz, i, j, k)) / s->dz;"),
    "lambda and mu exchanged in s_tt": (
        "double d_tt = dt * (lam * tr + 2.0 * mu * ett);",
        "double d_tt = dt * (mu * tr + 2.0 * lam * ett);"),
    "layer recursion with a and b exchanged": (
        "s->psi[q][p] = b * s->psi[q][p] + a * X;",
        "s->psi[q][p] = a * s->psi[q][p] + b * X;"),
    "layer coefficient a with the wrong sign": (
        "*a = d > 0.0 ? d * (*b - 1.0) / (d + alpha) : 0.0;",
        "*a = d > 0.0 ? d * (1.0 - *b) / (d + alpha) : 0.0;"),
    "ring source volume without the factor 2 pi": (
        "double vol = (j < 0) ? 2.0 * M_PI * rad * s->dr * s->dz",
        "double vol = (j < 0) ? rad * s->dr * s->dz"),
    "pressure receiver without the factor 1/3": (
        "if (q->kind == REC_PRESSURE) return -acc / (3.0 * (j1 - j0));",
        "if (q->kind == REC_PRESSURE) return -acc / (j1 - j0);"),
    "Courant limit without the azimuthal term": (
        "double g = sqrt(1.0 / (s->dr * s->dr) + 1.0 / (ra * ra) + 1.0 / (s->dz * s->dz));",
        "double g = sqrt(1.0 / (s->dr * s->dr) + 1.0 / (s->dz * s->dz));"),
    "transposed layer recursion returning the memory instead of the input": (
        "  pb[q][p] = b * t;\n  return outb + a * t;",
        "  pb[q][p] = b * t;\n  return a * t;"),
    "transposed e_rr scattered to the wrong ring": (
        "  addv(s, vr, i, j, k, err / s->dr);\n  addv(s, vr, i - 1, j, k, -err / s->dr);",
        "  addv(s, vr, i + 1, j, k, err / s->dr);\n  addv(s, vr, i, j, k, -err / s->dr);"),
    "transposed g_tz depth part with the wrong sign": (
        "  addv(s, fb[VT], i, j, k + 1, Dz / s->dz);\n  addv(s, fb[VT], i, j, k, -Dz / s->dz);",
        "  addv(s, fb[VT], i, j, k + 1, -Dz / s->dz);\n  addv(s, fb[VT], i, j, k, Dz / s->dz);"),
    "Ricker pulse delayed by 1/f0 instead of 2/f0": (
        "double tau = t - 2.0 / f0;",
        "double tau = t - 1.0 / f0;"),
    "face density from the theta neighbour instead of the depth neighbour": (
        "s->b_z[p] = 2.0 / (rho[p] + rho[IDX(s, i, j, k1)]);",
        "s->b_z[p] = 2.0 / (rho[p] + rho[IDX(s, i, j1, k)]);"),
    "edge shear modulus as the arithmetic mean of the four cells": (
        "  return 4.0 / (1.0 / a + 1.0 / b + 1.0 / c + 1.0 / d);",
        "  return 0.25 * (a + b + c + d);"),
    "azimuthal neighbour of the averages clamped instead of wrapped": (
        "int j1 = (j + 1) % s->nt;",
        "int j1 = j + 1 < s->nt ? j + 1 : s->nt - 1;"),
}

# The pin that rejected each mutant when this table was written, for the
# mutants the cheap first pins do not catch.  The test runs it first and then
# every other pin in order, so a stale entry costs time, never a verdict.
FIRST_PIN = {
    "layer recursion with a and b exchanged": "transposed step, layer True",
    "Courant limit without the azimuthal term": "Courant margin next to the axis",
    "azimuthal derivatives of s_rt in v_r and of v_r in g_rt both doubled (a consistent pair)":
        "transposed step, layer False",
    "ring source volume without the factor 2 pi": "closed-form point source",
    "layer coefficient a with the wrong sign": "torsional casing wave",
    "the same pair doubled in the transposed step as well (consistent throughout)":
        "operators against the paper's matrices",
    "transposed g_tz depth part with the wrong sign": "transposed step, layer False",
    "pressure receiver without the factor 1/3": "closed-form point source",
    "transposed layer recursion returning the memory instead of the input": "transposed step, layer True",
    "transposed e_rr scattered to the wrong ring": "transposed step, layer False",
}


def _pins():
    """(name, callable) of the oracle pins, cheapest first."""
    import test_oracle_adjoint as ta
    import test_oracle_averages as tav
    import test_oracle_physics as tph
    import test_oracle_pins as tp
    import test_oracle_rigid_pipe as trp
    pins = [("Ricker zeros and extrema", tp.test_ricker_properties),
            ("hand-derived staggered averages", tav.test_coefficient_tables_match_hand_values)]
    pins += [("impulse response applies the averages, %s" % c, (lambda cc=c: tav.test_step_applies_hand_values(cc)))
             for c in sorted(tav.IMPULSE)]
    pins += [("energy conservation", tp.test_energy_conserved)]
    pins += [("skew-adjointness %s" % (shape,), (lambda sh=shape: tp.test_operators_skew_adjoint(sh)))
             for shape in [(6, 8, 7), (5, 1, 9), (3, 2, 4)]]
    pins += [("transposed step, layer %s" % layer, (lambda ly=layer: ta.test_adjoint_step_is_the_transpose(ly)))
             for layer in (False, True)]
    pins += [("theta invariance", tp.test_theta_invariance_bitwise),
             ("P-SV / SH decoupling", tp.test_decoupling),
             ("reciprocity", tp.test_reciprocity),
             ("closed-form point source", tp.test_point_source_closed_form),
             ("Courant margin", tp.test_cfl_margin),
             ("Courant margin next to the axis", tp.test_cfl_margin_near_axis),
             ("operators against the paper's matrices", tp.test_operators_match_paper_matrices),
             ("rigid pipe: plane wave against the 1-D scheme", trp.test_rigid_pipe_plane_wave_matches_1d_scheme),
             ("torsional casing wave", tph.test_torsion_wave_in_casing),
             ("layer reflection bound", tph.test_pml_reflection_bound)]
    return pins


def _edits(m):
    return m if isinstance(m, list) else [m]


def _build(tmpdir, name, mutation):
    src = open(SRC).read()
    for orig, repl in _edits(mutation):
        assert src.count(orig) == 1, name
        src = src.replace(orig, repl)
    tag = "m%08x" % (hash(name) & 0xffffffff)
    c = os.path.join(tmpdir, tag + ".c")
    so = os.path.join(tmpdir, tag + ".so")
    with open(c, "w") as f:
        f.write(src)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                           "-fno-fast-math", "-Wl,-Bsymbolic", c, "-o", so, "-lm"])
    return so


@pytest.fixture(scope="module")
def mutant_libs(tmp_path_factory):
    d = str(tmp_path_factory.mktemp("oracle_mutants"))
    todo = dict(MUTANTS)
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        futs = {n: ex.submit(_build, d, n, m) for n, m in todo.items()}
        return {n: f.result() for n, f in futs.items()}


def _first_pin_that_fails(path, monkeypatch, first=None):
    """Name of the first pin that fails on the oracle built from `path`
    (None if all pass).  The pin named `first` runs before the others."""
    monkeypatch.setattr(oracle, "_lib", None)
    monkeypatch.setattr(oracle, "_LIB", path)
    monkeypatch.setattr(oracle, "build", lambda force=False: path)
    pins = sorted(_pins(), key=lambda p: p[0] != first)      # stable: the rest keep their order
    try:
        for name, fn in pins:
            try:
                fn()
            except (AssertionError, ValueError, FloatingPointError):
                return name
        return None
    finally:
        gc.collect()          # mutant simulations are freed by the library that made them


@pytest.mark.parametrize("name", list(MUTANTS))
def test_pins_reject_mutant(name, mutant_libs, monkeypatch):
    caught = _first_pin_that_fails(mutant_libs[name], monkeypatch, FIRST_PIN.get(name))
    print("%s: rejected by %s" % (name, caught))
    assert caught is not None, "no pin rejects the mutant: " + name


def test_sources_are_unique_and_the_original_passes():
    """Every planted text occurs exactly once, and the unmutated source
    passes the cheap pins (so a rejection is the mutation's doing)."""
    src = open(SRC).read()
    for name, m in MUTANTS.items():
        for orig, repl in _edits(m):
            assert src.count(orig) == 1 and orig != repl, name
    pin_names = {n for n, _ in _pins()}
    for name, pin in FIRST_PIN.items():
        assert name in MUTANTS and pin in pin_names, (name, pin)
    import test_oracle_pins as tp
    tp.test_energy_conserved()
    tp.test_reciprocity()


# ---- the refined-grid oracle (numpy): mutants of its source, loaded as a
# separate module and swapped in for the refined-oracle pins

REFINED_MUTANTS = {
    "half-integer phase shift with the wrong sign": (
        "    return 0.5 * (2.0 * math.pi / nf) - 0.5 * (2.0 * math.pi / nc)",
        "    return 0.5 * (2.0 * math.pi / nc) - 0.5 * (2.0 * math.pi / nf)"),
    "fine-to-coarse map without the factor 1/2": (
        "    x = np.fft.ifft(c, axis=0) * 0.5",
        "    x = np.fft.ifft(c, axis=0) * 1.0"),
    "half-integer fields interpolated as if on integer nodes": (
        "        half = name in HALF",
        "        half = False"),
}


def _refined_pins():
    """(name, callable) of every refined-oracle pin, parametrizations expanded."""
    import itertools
    import test_oracle_refined as tr
    out = []
    for name in sorted(n for n in dir(tr) if n.startswith("test_")):
        fn = getattr(tr, name)
        marks = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
        grids = [[(m.args[0], v) for v in m.args[1]] for m in marks]
        for combo in itertools.product(*grids):
            kw = dict(combo)
            out.append(("%s%s" % (name, kw or ""), (lambda f=fn, k=kw: f(**k))))
    return out


def _refined_mutant(mutation):
    import types
    from oracle import refined
    src = open(refined.__file__).read()
    for orig, repl in _edits(mutation):
        assert src.count(orig) == 1, orig
        src = src.replace(orig, repl)
    mod = types.ModuleType("refined_mutant")
    mod.__file__ = refined.__file__
    exec(compile(src, refined.__file__, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", list(REFINED_MUTANTS))
def test_refined_pins_reject_mutant(name, monkeypatch):
    import test_oracle_refined as tr
    monkeypatch.setattr(tr, "R", _refined_mutant(REFINED_MUTANTS[name]))
    caught = None
    for pin, fn in _refined_pins():
        try:
            fn()
        except (AssertionError, ValueError, FloatingPointError):
            caught = pin
            break
    print("%s: rejected by %s" % (name, caught))
    assert caught is not None, "no refined-grid pin rejects the mutant: " + name


def test_refined_unmutated_module_passes():
    """The loader itself changes nothing: the unmutated source, loaded the
    same way, passes every refined-grid pin."""
    import test_oracle_refined as tr
    saved = tr.R
    tr.R = _refined_mutant([])
    try:
        for pin, fn in _refined_pins():
            fn()
    finally:
        tr.R = saved

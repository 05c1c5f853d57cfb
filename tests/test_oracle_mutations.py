"""The oracle's pins catch plausible mistakes.

Each mutant below plants one mistake of the kind the pins are meant to
catch (a dropped term, a wrong sign, a wrong wall or index, the wrong
operand order) in a temporary copy of ``oracle/``; the oracle pin suite is
then run against that copy in a subprocess and must fail.  The unmutated
copy must pass, which checks the harness itself.  Nothing here touches the
repository's ``oracle/``.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_TESTS = ["test_oracle_energy.py", "test_oracle_dynamics.py", "test_oracle_adjoint.py"]

# (name, file under oracle/, text, replacement); the text occurs exactly once.
MUTANTS = [
    ("energy_sign", "spring_ising.py",
     'e = -np.einsum("ir,ij,jr->r", Si, U, Si)', 'e = np.einsum("ir,ij,jr->r", Si, U, Si)'),
    ("energy_full_matrix", "spring_ising.py",
     "U = np.triu(J, 1).astype(np.int64)", "U = J.astype(np.int64)"),
    ("energy_field_sign", "spring_ising.py",
     "e = e - np.asarray(h, dtype=np.int64) @ Si", "e = e + np.asarray(h, dtype=np.int64) @ Si"),
    ("real_energy_diagonal_included", "spring_ising.py",
     "U = np.triu(J, 1)\n        Sf", "U = np.triu(J, 0)\n        Sf"),
    ("readout_zero_is_down", "spring_ising.py",
     "np.where(Q < 0, -1, 1)", "np.where(Q <= 0, -1, 1)"),
    ("cut_weight_sign", "spring_ising.py",
     "W = -np.triu(J, 1)", "W = np.triu(J, 1)"),
    ("step_mass_dropped", "spring_ising.py",
     "U = Q + (dt / m) * P\n        V", "U = Q + dt * P\n        V"),
    ("step_spring_sign", "spring_ising.py",
     "V = P + dt * (-k * Q + zeta * F)\n        Pn = np.clip(V, -pmax, pmax)\n    elif",
     "V = P + dt * (k * Q + zeta * F)\n        Pn = np.clip(V, -pmax, pmax)\n    elif"),
    ("step_zeta_dropped", "spring_ising.py",
     "V = P + dt * (-k * Q + zeta * F)\n        Pn = np.clip(V, -pmax, pmax)\n    elif",
     "V = P + dt * (-k * Q + F)\n        Pn = np.clip(V, -pmax, pmax)\n    elif"),
    ("step_paper_order_uses_new_p", "spring_ising.py",
     "U = Q + (dt / m) * P\n        V = P + dt * (-k * Q + zeta * F)\n        Pn = np.clip(V, -pmax, pmax)",
     "V = P + dt * (-k * Q + zeta * F)\n        Pn = np.clip(V, -pmax, pmax)\n        U = Q + (dt / m) * Pn"),
    ("step_symplectic_uses_old_p", "spring_ising.py",
     "U = Q + (dt / m) * Pn", "U = Q + (dt / m) * P"),
    ("step_q_wall_is_pmax", "spring_ising.py",
     "Qn = np.clip(U, -qmax, qmax)", "Qn = np.clip(U, -pmax, pmax)"),
    ("step_p_wall_is_qmax", "spring_ising.py",
     "V = P + dt * (-k * Q + zeta * F)\n        Pn = np.clip(V, -pmax, pmax)\n    elif",
     "V = P + dt * (-k * Q + zeta * F)\n        Pn = np.clip(V, -qmax, qmax)\n    elif"),
    ("step_inelastic_keeps_p", "spring_ising.py",
     "Pn = np.where(np.abs(U) > qmax, 0.0, Pn)", "Pn = Pn"),
    ("step_field_sign", "spring_ising.py",
     "F = F + np.asarray(h, dtype=np.float64)[:, None]",
     "F = F - np.asarray(h, dtype=np.float64)[:, None]"),
    ("step_coupling_upper_triangle_only", "spring_ising.py",
     "F = J @ Q  #", "F = np.triu(J) @ Q  #"),
    ("step_coupling_replicas_mixed", "spring_ising.py",
     "F = J @ Q  #", "F = J @ Q[:, ::-1]  #"),
    ("schedule_last_stair_short", "spring_ising.py",
     "(s / (K - 1))", "(s / K)"),
    ("schedule_index_shifted", "spring_ising.py",
     "s = n // stair_len", "s = (n + 1) // stair_len"),
    ("constant_zeta_end", "spring_ising.py",
     "zeta_end=10.0 * 0.05,", "zeta_end=10.0 * 0.5,"),
    ("constant_qmax", "spring_ising.py",
     "qmax=math.sqrt(2.0),", "qmax=1.0,"),
    ("hamiltonian_kinetic_factor", "spring_ising.py",
     "(P * P).sum(axis=0) / (2.0 * m)", "(P * P).sum(axis=0) / m"),
    ("hamiltonian_zeta_dropped", "spring_ising.py",
     "+ zeta * ising", "+ ising"),
    ("relaxed_energy_half_dropped", "spring_ising.py",
     "per = -0.5 * np.einsum", "per = -1.0 * np.einsum"),
    ("adjoint_spring_term_sign", "adjoint.py",
     "lam_q = ubar - dt[n] * k * vbar", "lam_q = ubar + dt[n] * k * vbar"),
    ("adjoint_mass_dropped", "adjoint.py",
     "lam_p = (dt[n] / m) * ubar + vbar", "lam_p = dt[n] * ubar + vbar"),
    ("adjoint_wall_mask_ignored", "adjoint.py",
     "ubar = np.where(umask[n], lam_q, 0.0)", "ubar = lam_q"),
    ("adjoint_zeta_gradient_missing_dt", "adjoint.py",
     "g_zeta[n] = dt[n] * (Jv * qn).sum()", "g_zeta[n] = (Jv * qn).sum()"),
    ("adjoint_seed_sign", "adjoint.py",
     "lam_q = -(1.0 / R) * JQ", "lam_q = (1.0 / R) * JQ"),
    ("bruteforce_bit_order", "bruteforce.py",
     "bits = (idx >> np.arange(n, dtype=np.int64)[None, :]) & 1",
     "bits = (idx >> np.arange(n, dtype=np.int64)[None, ::-1]) & 1"),
    ("bruteforce_diagonal_included", "bruteforce.py",
     "U = np.triu(J, 1).astype(dt)", "U = np.triu(J, 0).astype(dt) - np.diag(np.ones(n)).astype(dt)"),
]


def _copy_tree(dst, mutant):
    """Copy what the oracle pin tests import into dst, applying the mutant."""
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(dst, "oracle"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    os.makedirs(os.path.join(dst, "tests"))
    for f in PIN_TESTS + ["conftest.py", "closed_forms.py"]:
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(dst, "tests", f))
    pkg = os.path.join(dst, "paper_2305_07187_amd")
    os.makedirs(pkg)
    for f in ("__init__.py", "instances.py"):
        shutil.copy(os.path.join(ROOT, "paper_2305_07187_amd", f), os.path.join(pkg, f))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), os.path.join(dst, "pytest.ini"))
    if mutant is not None:
        _, fname, old, new = mutant
        path = os.path.join(dst, "oracle", fname)
        text = open(path).read()
        assert text.count(old) == 1, (mutant[0], text.count(old))
        open(path, "w").write(text.replace(old, new))


def _run_pins(dst):
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1", OMP_NUM_THREADS="1",
               OPENBLAS_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider"] + [os.path.join("tests", f) for f in PIN_TESTS],
                       cwd=dst, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, (r.stdout + r.stderr)[-600:]


def test_mutants_are_killed(tmp_path):
    cases = [("control", None)] + [(m[0], m) for m in MUTANTS]

    def one(case):
        name, mutant = case
        dst = tmp_path / name
        dst.mkdir()
        _copy_tree(str(dst), mutant)
        return name, _run_pins(str(dst))

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = dict(ex.map(one, cases))
    rc, tail = results.pop("control")
    assert rc == 0, f"the unmutated copy must pass its pins:\n{tail}"
    survivors = [name for name, (rc, _) in results.items() if rc == 0]
    assert not survivors, f"mutants not caught by any pin: {survivors}"
    # a mutant must fail a test, not crash the run (exit code 1 = failures)
    crashed = {name: tail for name, (rc, tail) in results.items() if rc not in (0, 1)}
    assert not crashed, crashed

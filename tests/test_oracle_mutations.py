"""Plant plausible mistakes in the oracle and check that a pin catches each.

Each mutation rewrites one line of one oracle function (a dropped term, a
wrong sign or index, a transposed operand, a wrong constant), re-executes the
function in the oracle's namespace, runs every pin, and requires at least one
pin to fail.  The oracle is restored afterwards.
"""
import inspect
import os
import sys
import textwrap

import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle_pins as P  # noqa: E402
from oracle import dls, l2, learned  # noqa: E402
from oracle import globalbasis  # noqa: E402

MODULES = {"dls": dls, "learned": learned, "l2": l2, "globalbasis": globalbasis}

# (function, original text, planted mistake); functions of oracle.learned are
# prefixed "learned."
MUTATIONS = [
    ("rank_one_verify", "return float(np.trace(G)) - theta <= tau, theta",
     "return float(np.trace(G)) - theta < tau, theta"),
    ("leading_vector", "i = int(np.argmax(np.diag(G)))", "i = int(np.argmin(np.diag(G)))"),
    ("rank_one_verify", "theta = float(q @ (G @ q))", "theta = float(q @ q)"),
    ("leading_vector", "for _ in range(iters):", "for _ in range(iters // 3):"),
    ("sketch_points", "return min(m, max(1, SKETCH_POINTS // px) * px)", "return min(m, SKETCH_POINTS)"),
    ("encode_block_sketch", "ok, theta = rank_one_verify(G, q, tau)",
     "ok, theta = rank_one_verify(xg[:, :s] @ xg[:, :s].T, q, tau)"),
    ("learned.moments", "f[11] = float(np.mean((x[2:] - mu) * (x[:-2] - mu))) / var",
     "f[11] = float(np.mean((x[1:] - mu) * (x[:-1] - mu))) / var"),
    ("learned.moments", "f[13] = math.log10(max(sd / eps, 1e-15))", "f[13] = math.log10(max(var / eps, 1e-15))"),
    ("learned.moments", "f[10] = float(np.mean((x[1:] - mu) * (x[:-1] - mu))) / var",
     "f[10] = float(np.mean((x[1:] - mu) * (x[:-1] - mu))) / sd"),
    ("nrmse", "return 100.0 * float(np.sqrt(np.sum(d * d)) / np.sqrt(np.sum(a * a)))",
     "return 100.0 * float(np.sum(d * d) / np.sum(a * a))"),
    ("nrmse", "d = a - uh.astype(np.float64)", "d = a - uh.astype(np.float32)"),
    ("canonical_signs", "i = int(np.argmax(np.abs(V[:, k])))",
     "i = V.shape[0] - 1 - int(np.argmax(np.abs(V[::-1, k])))"),
    ("tail_energies", "t[r] = t[r + 1] + lam[r]", "t[r] = t[r + 1] + lam[min(r + 1, lam.size - 1)]"),
    ("choose_rank", "if tail[r] <= tau:", "if tail[r - 1] <= tau:"),
    ("encode_block", "code = encode_with_basis(xs, eps, V[:, :r], lam, tau, dtype)",
     "code = encode_with_basis(xs, eps, V[:, 1:r + 1] if V.shape[1] > r else V[:, :r], lam, tau, dtype)"),
    ("encode_with_basis", "A = x.T @ Vr", "A = x @ Vr[:x.shape[1]] if False else x.T @ Vr[::-1]"),
    ("encode_with_basis", "q = np.rint((x - xhat) * (1.0 / (2.0 * eps)))", "q = np.rint((x - xhat) * (1.0 / eps))"),
    ("encode_with_basis", "xhat = S.astype(np.float64) * c", "xhat = -S.astype(np.float64) * c"),
    ("encode_with_basis", "qV = np.rint(Vr * float(1 << BASIS_BITS)).astype(np.int64)",
     "qV = np.rint(Vr * float(1 << (BASIS_BITS - 1))).astype(np.int64)"),
    ("encode_block", "tau = KAPPA * eps * eps * m * wb", "tau = KAPPA * eps * m * wb"),
    ("encode_block", "G = xg @ xg.T", "G = xg @ xg.T - np.diag(np.diag(xg @ xg.T)) * 0.5"),
    ("round_bf16", "np.ldexp(m, 8)", "np.ldexp(m, 9)"),
    ("eig_desc", "order = np.argsort(-lam, kind=\"stable\")", "order = np.argsort(lam, kind=\"stable\")"),
    ("canonical_signs", "if V[i, k] < 0:", "if V[i, k] > 0:"),
    ("gradient_magnitude", "d[s(1, n - 1)] = (f[s(2, n)] - f[s(0, n - 2)]) * 0.5",
     "d[s(1, n - 1)] = (f[s(2, n)] - f[s(0, n - 2)])"),
    ("percentile80", "int(math.floor(0.8 * (v.size - 1)))", "int(math.ceil(0.8 * (v.size - 1)))"),
    ("lattice_values", "n = S + q * (1 << RES_SHIFT)", "n = S + q * (1 << (RES_SHIFT - 1))"),
    ("zigzag8", "-2 * q - 1", "-2 * q + 1"),
    ("encode_with_basis", "big = np.abs(q) > Q_LIMIT", "big = np.abs(q) > 2 * Q_LIMIT"),
    ("l2.first_rank", "tau = TAIL_SHARE * e2", "tau = 0.4 * e2"),
    ("l2.first_rank", "if tail[0] <= tau:", "if tail[1] <= tau:"),
    ("l2.first_rank", "for r in range(1, rcap + 1):", "for r in range(2, rcap + 1):"),
    ("l2.encode_block", "step = STEP_SHARE * math.sqrt(e2 / (r * m))", "step = STEP_SHARE * math.sqrt(e2 / m)"),
    ("l2.encode_block", "qV = np.rint(Vr * 2.0 ** BASIS_BITS).astype(np.int64)",
     "qV = np.rint(Vr * 2.0 ** 16).astype(np.int64)"),
    ("l2.encode_block", "A = x.T @ Vr", "A = xg.T @ Vr"),
    ("l2.decode_block", "vt = qV[:, k].astype(np.float64) * 2.0 ** -BASIS_BITS",
     "vt = qV[:, k].astype(np.float64) * 2.0 ** -16"),
    ("l2.decode_block", "ck = qA[:, k].astype(np.float64) * step", "ck = qA[:, k].astype(np.float64) / step"),
    ("l2.variable_budgets", "c.append(float(targets[v]) ** 2 * norm2 / float(field[v].size))",
     "c.append(float(targets[v]) * norm2 / float(field[v].size))"),
    ("l2.block_budget", "return c_v * b.m * b.w", "return c_v * b.m"),
    ("l2.nrmse_fraction", "return float(np.sqrt(np.sum(d * d)) / np.sqrt(np.sum(np.where(fin, a * a, 0.0))))",
     "return float(np.sum(d * d) / np.sum(np.where(fin, a * a, 0.0)))"),
    ("globalbasis.SplitMix64", "z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK",
     "z = ((z ^ (z >> 31)) * 0xBF58476D1CE4E5B9) & _MASK"),
    ("globalbasis.cosine_basis", "math.sqrt((1.0 if a == 0 else 2.0) / n)", "math.sqrt(2.0 / n)"),
    ("globalbasis.cosine_basis", "math.cos(math.pi * (2 * i + 1) * a / (2 * n))",
     "math.cos(math.pi * (2 * i + 1) * a / n)"),
    ("globalbasis.sample_matrix", "patch = field[v, 0, z0:z0 + p.pz, y0:y0 + p.py, x0:x0 + p.px]",
     "patch = field[v, 1, z0:z0 + p.pz, y0:y0 + p.py, x0:x0 + p.px]"),
    ("globalbasis.sample_positions", "x0 = g.next() % (p.nx - p.px + 1)", "x0 = g.next() % (p.nx - p.px + 2)"),
    ("globalbasis.learn_basis", "_, V = dls.eig_desc(Q.T @ Q)", "_, V = dls.eig_desc(Q.T @ Q[::-1])"),
    ("globalbasis.variable_budgets", "c.append(float(targets[v]) ** 2 * float(np.sum(x * x))",
     "c.append(float(targets[v]) * float(np.sum(x * x))"),
    ("globalbasis.encode_patch", "order = np.argsort(-np.abs(alpha), kind=\"stable\")",
     "order = np.argsort(np.abs(alpha), kind=\"stable\")"),
    ("globalbasis.encode_patch", "if tail[j] <= TAIL_SHARE * e2", "if tail[j] <= e2"),
    ("globalbasis.step_exponent", "return e - 1", "return e"),
    ("globalbasis.encode_patch", "kept = np.sort(order[:n])", "kept = order[:n]"),
    ("globalbasis.decode_patch", "acc = acc + phi[idx, s] * (float(qs) * d)",
     "acc = acc + phi[s, idx] * (float(qs) * d)"),
]


def _mutate(qual, old, new):
    mod, name = qual.split(".") if "." in qual else ("dls", qual)
    module = MODULES[mod]
    fn = getattr(module, name)
    src = textwrap.dedent(inspect.getsource(fn))
    assert old in src, (qual, old)
    ns = dict(vars(module))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    return module, name, ns[name]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] + ":" + m[2][:30] for m in MUTATIONS])
def test_mutation_is_caught(name, old, new, monkeypatch):
    module, fname, mutant = _mutate(name, old, new)
    monkeypatch.setattr(module, fname, mutant)
    # functions that call the mutated one resolve it through the module globals
    caught = []
    for pin in P.ALL_PINS:
        try:
            pin()
        except Exception:  # AssertionError or a crash both count as caught
            caught.append(pin.__name__)
    assert caught, "no pin caught mutation %s: %s -> %s" % (name, old, new)

"""Block-by-block bars for single-precision results against the double-precision oracle.

A single-precision factor (or vector) is judged block by block (cell by cell): block b passes when
its relative error is within max(1e-5, C s_b), where s_b is the relative change of the oracle's
block b when its inputs, and every iterate the single-precision path stores between sweeps, are
perturbed by one float unit in the last place, normwise per block (each value moved by up to 2^-24
times the largest magnitude in its block, random signs): the block's sensitivity to float-sized
errors, the largest response over 4 independent perturbations (one random direction can miss a
block's ill-conditioned direction: the ratio of two random responses is heavy-tailed). Well-conditioned blocks get the stated 1e-5; blocks that
depend on an ill-conditioned diagonal block get its conditioning. Under the initial guess L = A the
first sweep forms U_ii = A_ii - sum A_ik A_ki, whose condition number reaches 8e6 on the
aspect-ratio-1000 layers; storing that U_ii in float moves its inverse by up to cond x 2^-24 even
where perturbing A alone moves it far less, which is why the stored iterates are perturbed too. Each result is compared both with the oracle on the double inputs and
with the oracle on the inputs rounded to float (what the FP32 path reads), which separates the
arithmetic error from the input rounding. A wrong family of blocks, however small its share of the
norm, fails its own bar.
"""
import numpy as np

from tests.dense_ref import block_rel, rel

C = 32.0      # float error allowed per block, in units of the block's float sensitivity
SAMPLES = 4   # independent perturbations; a block's sensitivity is the largest response among them
FLOOR = 1e-5  # the stated single-precision bar
CAP = 0.5     # no block may be off by more than half its size, however ill-conditioned


def f32(a):
    return None if a is None else np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def _perturb(a, g):
    """Normwise float-sized perturbation of every block (an [n,4,4] array) or every cell's 4-vector
    (a vector of 4n values): each value moved by up to 2^-24 times the largest magnitude in its
    block, with random signs. Float block arithmetic errs normwise (Gaussian elimination with
    partial pivoting is normwise backward stable; a rounded product of blocks errs by a float ulp
    of the sums of products), so a componentwise perturbation would miss blocks whose entries
    differ greatly in size."""
    a = np.asarray(a, np.float64)
    bs = 16 if a.ndim == 3 else (4 if a.ndim == 1 and a.size % 4 == 0 else 1)
    blocks = a.reshape(-1, bs)
    scale = np.abs(blocks).max(axis=1, keepdims=True)
    return (blocks + g.uniform(-1.0, 1.0, blocks.shape) * 2.0 ** -24 * scale).reshape(a.shape)


def _judge(name, got, ref, ref32, sens, what, shape=None):
    if shape:
        got, ref, ref32 = got.reshape(shape), ref.reshape(shape), ref32.reshape(shape)
    bar = np.minimum(CAP, np.maximum(FLOOR, C * sens))
    e, e32 = block_rel(got, ref), block_rel(got, ref32)
    k, k32 = int(np.argmax(e / bar)), int(np.argmax(e32 / bar))
    assert e[k] <= bar[k], (what, name, "vs oracle", k, e[k], bar[k], sens[k])
    assert e32[k32] <= bar[k32], (what, name, "vs oracle on inputs rounded to float", k32, e32[k32], bar[k32])
    return (rel(got, ref), rel(got, ref32), float(e[k] / bar[k]), float(e32[k32] / bar[k32]),
            int((bar > FLOOR).sum()), len(bar))


def perturb(a, g):
    """a perturbed by one float unit in the last place, normwise per block (see _perturb)."""
    return _perturb(a, g)


class FactorBars:
    """run(A, X0) -> (X, Dinv): an oracle factorisation. Holds its result on A, on A (and X0)
    rounded to float, and the per-block sensitivities of X and Dinv. perturbed(g) -> (X, Dinv), if
    given, is the oracle run with A and every stored iterate perturbed (default: A and X0 only)."""

    def __init__(self, run, A, X0=None, seed=23, perturbed=None):
        self.Xo, self.Do = run(A, X0)
        self.X32, self.D32 = run(f32(A), f32(X0))
        self.sX = self.sD = None
        for q in range(SAMPLES):
            g = np.random.default_rng(seed + 1000 * q)
            if perturbed is not None:
                Xp, Dp = perturbed(g)
            else:
                Xp, Dp = run(_perturb(A, g), None if X0 is None else _perturb(X0, g))
            sX, sD = block_rel(Xp, self.Xo), block_rel(Dp, self.Do)
            del Xp, Dp
            self.sX = sX if self.sX is None else np.maximum(self.sX, sX)
            self.sD = sD if self.sD is None else np.maximum(self.sD, sD)

    def check(self, X, D, what=""):
        return {"X": _judge("X", X, self.Xo, self.X32, self.sX, what),
                "Dinv": _judge("Dinv", D, self.Do, self.D32, self.sD, what)}


class VectorBars:
    """run(X, Dinv, r) -> z: an oracle application, with the factor already as float storage holds
    it. Holds its result on r rounded to float and the per-cell sensitivities."""

    def __init__(self, run, X, D, r, seed=29):
        self.ref = run(X, D, f32(r))
        self.sens = None
        for q in range(SAMPLES):
            g = np.random.default_rng(seed + 1000 * q)
            refp = run(_perturb(X, g), _perturb(D, g), _perturb(f32(r), g))
            s = block_rel(refp.reshape(-1, 4), self.ref.reshape(-1, 4))
            self.sens = s if self.sens is None else np.maximum(self.sens, s)

    def check(self, z, what=""):
        """Every cell within its bar and the whole vector within 1e-5."""
        e, _, worst, _, _, _ = _judge("z", z, self.ref, self.ref, self.sens, what, shape=(-1, 4))
        assert e <= FLOOR, (what, e)
        return e, worst


def report(what, out):
    print(what + ": " + "; ".join(f"{n}: rel {a:.2e} (input-rounded oracle {b:.2e}), worst block at {r:.2f} "
                                  f"({r32:.2f}) of its bar, {w} of {nb} bars above 1e-5"
                                  for n, (a, b, r, r32, w, nb) in out.items()))

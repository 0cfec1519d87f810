"""tersoff_compute_static -- the evaluation with no allocation, its buffers in
a fixed device array of the library -- against tersoff_compute on the same
inputs: two calls in a row, the second with a smaller input (and another
kernel instance), in every precision.  The two entry points run the same
kernels in the same launch configuration, so their results must agree bit
for bit; both are also held to the oracle at the stated tolerances.  A build
above the array's capacity is refused on the host."""
import numpy as np
import pytest

from paper_1710_00882_amd import workloads as W

from gpu_helpers import assert_parity, oracle_eval, say, to_dev

pytestmark = pytest.mark.gpu


def _eval(m, pos, prec, static):
    import torch
    out, F = m.compute(pos, prec, static=static)
    torch.cuda.synchronize()
    return out.cpu().numpy(), F.cpu().numpy()


@pytest.mark.parametrize("precision", ["mixed", "fp64", "single"])
def test_static_entry_point_matches_compute(precision):
    from paper_1710_00882_amd import Tersoff
    systems = [("si_11520", W.diamond(12, 12, 10, jitter=0.1, seed=31), W.si_table()),
               ("disordered_1500", W.disordered(1500, seed=32), W.two_species_table())]
    models, inputs, ref = [], [], []
    for name, s, table in systems:
        m = Tersoff(table)
        pos, types = to_dev(s)
        m.build_neighbors(pos, types, s.box, skin=W.SKIN)
        models.append(m)
        inputs.append(pos)
        ref.append(_eval(m, pos, precision, static=False))
    # two static calls in a row, the second on the smaller input
    got = [_eval(m, pos, precision, static=True) for m, pos in zip(models, inputs)]
    for (name, s, table), m, (o_ref, F_ref), (o, F) in zip(systems, models, ref, got):
        m.check()
        say(f"[static] {name} {precision}: n={s.n}")
        assert np.array_equal(o, o_ref), f"{name}: energy / virial differ from tersoff_compute"
        assert np.array_equal(F, F_ref), f"{name}: forces differ from tersoff_compute"
        assert_parity(o[0], F, o[1:], o_ref[0], F_ref, o_ref[1:], s.n, precision, f"{name} static vs compute")
        Eo, Fo, Vo, _, _ = oracle_eval(s, table)
        assert_parity(o[0], F, o[1:], Eo, Fo, Vo, s.n, precision, f"{name} static vs oracle")


def test_static_entry_point_refuses_large_builds():
    from paper_1710_00882_amd import Tersoff
    from paper_1710_00882_amd._lib import TersoffError
    s = W.diamond(13, 13, 13, jitter=0.05, seed=33)      # 17,576 atoms > 16,384
    m = Tersoff(W.si_table())
    pos, types = to_dev(s)
    m.build_neighbors(pos, types, s.box, skin=W.SKIN)
    with pytest.raises(TersoffError) as e:
        m.compute(pos, "mixed", static=True)
    assert e.value.status == -1
    out, F = _eval(m, pos, "mixed", static=False)   # the allocating entry point still serves it
    assert np.isfinite(out).all()

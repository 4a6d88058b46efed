"""Exchange schedule of the domain-decomposed training loop (Algorithm 1:
exchange at iterations i with i mod I_comm = 0, plus the documented initial
exchange before iteration 1).  Host logic only: a stand-in context records
the calls."""
import pytest

from paper_2602_15883_amd.trainer import DDTrainer


class _Sub:
    class _T:
        def numel(self):
            return 1
    gh_up = _T()


class _Ctx:
    def __init__(self):
        self.subs = [_Sub(), _Sub()]
        self.calls = []

    def exchange(self, faces, x_anc, targets, stream=None):
        self.calls.append(("x", self.t_next))

    def step(self, t, stream=None):
        self.calls.append(("s", t))
        return "loss", None


def _run(i_comm, n, initial=True):
    ctx = _Ctx()
    tr = DDTrainer(ctx, [(0, 1, 0, 4)], [1.0, 1.0], i_comm=i_comm, initial_exchange=initial)
    for t in range(1, n + 1):
        ctx.t_next = t
        tr.step()
    return ctx.calls


def test_every_iteration_at_icomm_1():
    calls = _run(1, 4)
    assert calls == [("x", 1), ("s", 1), ("x", 2), ("s", 2), ("x", 3), ("s", 3), ("x", 4), ("s", 4)]


def test_algorithm_phase_at_icomm_3():
    ex = [t for k, t in _run(3, 7) if k == "x"]
    assert ex == [1, 3, 6]              # initial exchange, then i mod 3 == 0
    ex = [t for k, t in _run(3, 7, initial=False) if k == "x"]
    assert ex == [3, 6]                 # Algorithm 1 exactly


def test_exchange_precedes_the_step_of_its_iteration():
    calls = _run(2, 4)
    assert calls.index(("x", 2)) == calls.index(("s", 2)) - 1


def test_bad_interval_rejected():
    with pytest.raises(ValueError):
        DDTrainer(_Ctx(), [], [0.0, 0.0], i_comm=0)

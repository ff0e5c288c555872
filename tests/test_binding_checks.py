"""The Python binding checks the extents of every tensor it passes against
the sizes it passes with them, before any library call: the C ABI receives
bare pointers and cannot see a short buffer. Runs on the CPU with a context
whose library handle fails the test if it is touched."""
import pytest
import torch

from paper_2509_26222_amd import api


class _NoLib:
    def __getattr__(self, name):
        raise AssertionError(f"library call {name} reached with a bad argument")


def _ctx():
    c = api.Context.__new__(api.Context)
    c.lib = _NoLib()
    c.device = 0
    c.h = None
    return c


def _grid(n):
    g = api.Grid.__new__(api.Grid)
    g.h = None
    g.N = n
    g.max_candidates = 40
    return g


F64 = torch.float64
P = api.Params()


def t(*shape, dtype=F64):
    return torch.zeros(shape, dtype=dtype)


@pytest.mark.parametrize("call, match", [
    (lambda c, g: c.update(P, g, t(100), t(100, 100), t(50, 3), t(50)), "xy"),
    (lambda c, g: c.update(P, g, t(100), t(100, 100), t(50, 2), t(49)), "z"),
    (lambda c, g: c.update(P, g, t(99), t(100, 100), t(50, 2), t(50)), "w"),
    (lambda c, g: c.update(P, g, t(100), t(100, 99), t(50, 2), t(50)), "P"),
    (lambda c, g: c.update(P, g, t(100), t(100, 200)[:, ::2], t(50, 2), t(50)), "P"),
    (lambda c, g: c.update_active(P, g, t(100), t(100, 100), t(50, 2), t(51)), "z"),
    (lambda c, g: c.update_active(P, g, t(100), t(100, 100), t(50, 2), t(50),
                                  active=t(99, dtype=torch.int32)), "active"),
    (lambda c, g: c.eval(P, g, t(100), t(10, 4)), "pts"),
    (lambda c, g: c.eval(P, g, t(100), t(10, 3)), "pose"),
    (lambda c, g: c.eval(P, g, t(100), t(10, 2), pose=(torch.eye(3), t(3))), "pose"),
    (lambda c, g: c.eval(P, g, t(90), t(10, 2)), "w"),
    (lambda c, g: c.eval(P, g, t(100), t(10, 2, dtype=torch.int32)), "pts"),
    (lambda c, g: c.eval_gn(P, g, t(100), t(10, 2), pose=(torch.eye(3), t(3))), "pts"),
    (lambda c, g: c.eval_gn(P, g, t(101), t(10, 3), pose=(torch.eye(3), t(3))), "w"),
    (lambda c, g: c.eval_adjoint(P, g, t(100), t(10, 2), gbar_f=t(9)), "gbar_f"),
    (lambda c, g: c.eval_adjoint(P, g, t(100), t(10, 3), pose=(torch.eye(3), t(3)),
                                 gbar_r=t(11)), "gbar_r"),
    (lambda c, g: c.eval_adjoint(P, g, t(100), t(10, 2), gbar_f=t(10), d_w=t(50)), "d_w"),
    (lambda c, g: c.eval_adjoint(P, g, t(100), t(10, 3), pose=(torch.eye(3), t(3)),
                                 d_pose=t(5)), "d_pose"),
    (lambda c, g: c.sort_points(g, t(20, 2), t(19)), "z"),
    (lambda c, g: c.assemble_phi(P, g, t(20)), "xy"),
    (lambda c, g: c.assemble_gram(P, g, t(20, 2), t(20), t(100, dtype=torch.int64),
                                  t(500, dtype=torch.int32)), "rowptr"),
    (lambda c, g: c.assemble_gram(P, g, t(20, 2), t(20), t(101, dtype=torch.int64),
                                  t(500, dtype=torch.int32), vals=t(499)), "vals"),
    (lambda c, g: c.assemble_gram(P, g, t(20, 2), t(20), t(101, dtype=torch.int64),
                                  t(500, dtype=torch.int32), vals=t(500), b=t(99)), "b"),
    (lambda c, g: c.solve(t(101, dtype=torch.int64), t(500, dtype=torch.int32), t(500),
                          t(99)), "B"),
    (lambda c, g: c.solve(t(101, dtype=torch.int64), t(500, dtype=torch.int32), t(500),
                          t(100, 2), X=t(100, 3)), "X"),
    (lambda c, g: c.refine(P, t(101, dtype=torch.int64), t(500, dtype=torch.int32), t(500),
                           t(100), t(100, 100), t(99)), "w"),
    (lambda c, g: c.refine(P, t(101, dtype=torch.int64), t(500, dtype=torch.int32), t(500),
                           t(98), t(100, 100), t(100)), "b"),
    (lambda c, g: c.select_centers(t(30, 3), (0, 0, 1, 1), 0.5, 0.5, 4), "xy"),
    (lambda c, g: c.state_grow(P, t(10), t(20, 20), 0, 20), "w"),
    (lambda c, g: c.state_grow(P, t(20), t(19, 20), 0, 20), "P"),
])
def test_mismatched_extents_raise_before_any_call(call, match):
    with pytest.raises((ValueError, TypeError), match=match):
        call(_ctx(), _grid(100))


def test_batched_patch_extents_checked_before_plan():
    g = _grid(100)
    base = dict(grid=g, w=t(100), P=t(100, 100), xy=t(40, 2), z=t(40), pts=t(30, 3),
                pose=(torch.eye(3), t(3)), f=t(30), grad=t(30, 2), resid=t(30), jac=t(30, 6))
    for key, bad in [("z", t(39)), ("w", t(101)), ("P", t(100, 99)), ("f", t(29)),
                     ("grad", t(30, 3)), ("resid", t(31)), ("jac", t(30, 5)),
                     ("pts", t(30, 2))]:
        patch = dict(base)
        patch[key] = bad
        with pytest.raises(ValueError, match=key):
            api.Batched(_ctx(), P, [patch], dim=3)

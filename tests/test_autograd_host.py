"""Host logic of the torch.autograd binding, on the CPU with a stand-in
context (a quadratic map with known derivatives): every autograd entry
(backward, forward_ad, torch.func.jvp/grad/vjp) reaches the context with
plain tensors that have storage, and returns the context's results."""
import torch

from paper_2209_04481_amd.autograd import residual


class QuadraticContext:
    """R(U, b) = U^2 + sum(b).  Like the library binding, it takes data
    pointers of every argument and writes results into tensors it allocates
    (both fail on tensors wrapped by torch.func transforms)."""

    def _plain(self, *ts):
        for t in ts:
            if t is not None:
                t.data_ptr()
                assert t.is_contiguous()

    def _out(self, like, value):
        o = torch.empty(like.shape, dtype=like.dtype)
        self._plain(o)
        with torch.no_grad():
            o.copy_(value)
        return o

    def set_inner_br(self, br):
        self._plain(br)
        self.br = br.clone()

    def residual(self, U):
        self._plain(U)
        return self._out(U, U ** 2 + self.br.sum())

    def jvp(self, U, v, dbr=None):
        self._plain(U, v, dbr)
        return self._out(U, 2 * U * v + (0.0 if dbr is None else dbr.sum()))

    def vjp(self, U, w, want_br=True):
        self._plain(U, w)
        gb = self._out(self.br, w.sum() * torch.ones_like(self.br)) if want_br else None
        return self._out(U, 2 * U * w), gb


def _inputs():
    g = torch.Generator().manual_seed(3)
    U = torch.randn(9, 5, dtype=torch.float64, generator=g)
    br = torch.randn(4, dtype=torch.float64, generator=g)
    return U, br, torch.randn(9, 5, dtype=torch.float64, generator=g), torch.randn(4, dtype=torch.float64, generator=g)


def test_reverse_mode_entries():
    c = QuadraticContext()
    U, br, w, _ = _inputs()
    Ur, brr = U.clone().requires_grad_(True), br.clone().requires_grad_(True)
    (residual(Ur, brr, c) * w).sum().backward()
    assert torch.allclose(Ur.grad, 2 * U * w) and torch.allclose(brr.grad, w.sum() * torch.ones_like(br))
    g = torch.func.grad(lambda a: (residual(a, br, c) * w).sum())(U)
    assert torch.allclose(g, 2 * U * w)
    gU, gb = torch.func.vjp(lambda a, b: residual(a, b, c), U, br)[1](w)
    assert torch.allclose(gU, 2 * U * w) and torch.allclose(gb, w.sum() * torch.ones_like(br))


def test_forward_mode_entries():
    c = QuadraticContext()
    U, br, v, db = _inputs()
    R, Jv = torch.func.jvp(lambda a, b: residual(a, b, c), (U, br), (v, db))
    assert torch.allclose(R, U ** 2 + br.sum()) and torch.allclose(Jv, 2 * U * v + db.sum())
    import torch.autograd.forward_ad as fwAD
    with fwAD.dual_level():
        out = residual(fwAD.make_dual(U, v), br, c)
        assert torch.allclose(fwAD.unpack_dual(out).tangent, 2 * U * v)

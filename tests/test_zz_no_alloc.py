"""The allocation-free dot products (cfv_dots_noalloc) through the C ABI,
against cfv_dots of a context on the same vectors: bitwise equal results on
two calls in a row, the second with fewer vectors of a smaller shell (the
static partial-sum array keeps the first call's contents), and the size
limit of that array refused before any device work."""
import pytest
import torch

import coronal_inputs as ci

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def vectors(ncells, k, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    V = torch.randn(k, 9 * ncells, dtype=torch.float64, device="cuda", generator=g)
    w = torch.randn(9 * ncells, dtype=torch.float64, device="cuda", generator=g)
    return V, w


def test_dots_noalloc_equals_dots_on_two_calls():
    from paper_2209_04481_amd import Context, Grid
    from paper_2209_04481_amd.binding import dots_noalloc
    print("case: cfv_dots_noalloc vs cfv_dots, 6x24x24x40 with 32 vectors then 6x8x8x5 with 3", flush=True)
    for (N, Nr, k, seed) in ((24, 40, 32, 1), (8, 5, 3, 2)):
        inst = ci.make_instance(N, Nr, "log", lmax=0, seed=seed)
        ctx = Context(Grid(inst.N, inst.Nr, inst.r_nodes))
        V, w = vectors(inst.ncells, k, seed)
        got = dots_noalloc(V, w)
        want = ctx.dots(V, w)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (N, Nr, k)
        # and the plain sums, to rounding
        ref = (V * w[None]).sum(1)
        assert torch.allclose(got, ref, rtol=1e-12, atol=1e-12 * float(ref.abs().max()))


def test_dots_noalloc_refuses_more_vectors_than_its_array_holds():
    from paper_2209_04481_amd import CfvError
    from paper_2209_04481_amd.binding import dots_noalloc
    V, w = vectors(10, 33, 3)
    with pytest.raises(CfvError, match="1..32"):
        dots_noalloc(V, w)

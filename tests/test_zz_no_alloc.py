"""he_fk_propagate_noalloc (the entry point for callers that cannot allocate device
memory) against he_fk_propagate on the same ensembles, through the C ABI: two calls in
a row, the second on a smaller ensemble with fewer sample rows, so the static scratch
holds the first call's larger set of partial rows when the second one runs.  The two
entry points share their kernels, so the results agree bitwise; a call whose partial
rows exceed the static scratch is refused before any launch."""
import numpy as np
import pytest

from paper_1703_08977_amd import _lib, api
from paper_1703_08977_amd import workloads as W

from hefk_testutil import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an AMD Instinct GPU")]


def _pair(cfg, n_walkers, n_steps, sample_every):
    import torch
    ens_a = api.Ensemble(cfg, n_walkers=n_walkers).init()
    ens_b = api.Ensemble(cfg, n_walkers=n_walkers).init()
    ns = n_steps // sample_every + 1
    sa = ens_a.propagate(0, n_steps, sample_every)
    sb = torch.full((ns, 8), float("nan"), dtype=torch.float64, device="cuda")
    api.he_fk_propagate_noalloc(ens_b.p, ens_b.walkers(), 0, n_steps, sample_every, sb.data_ptr(), 0, 0)
    torch.cuda.synchronize()
    return ens_a, ens_b, sa.cpu().numpy(), sb.cpu().numpy()


@pytest.mark.parametrize("name,over,first,second", [
    ("he_2P_pz_16m", dict(), (1 << 20, 600, 5), (3001, 200, 20)),
    ("he_2P_pz_16m", dict(precision="fp64"), (200000, 400, 4), (257, 100, 50)),
    ("he_1s_pade_1m", dict(dt=0.002), (1 << 20, 500, 5), (1, 20, 10)),
], ids=["pz_mixed", "pz_fp64", "pade_fp64"])
def test_noalloc_matches_the_workspace_entry_point(name, over, first, second):
    cfg = W.get(name, **over)
    for n, k, se in (first, second):
        print("noalloc vs workspace: %s %s n=%d steps=%d every=%d" % (name, over, n, k, se), flush=True)
        a, b, sa, sb = _pair(cfg, n, k, se)
        assert np.array_equal(sa, sb)
        for t in ("x", "lnw", "el"):
            ta, tb = getattr(a, t).cpu().numpy(), getattr(b, t).cpu().numpy()
            assert np.array_equal(ta, tb, equal_nan=True), t


def test_noalloc_refuses_rows_beyond_its_scratch():
    import torch
    cfg = W.get("he_2P_pz_16m")
    e = api.Ensemble(cfg, n_walkers=1 << 22).init()
    n_steps, se = 4000, 1                   # 4001 sample rows per block
    need = api.he_fk_propagate_workspace_bytes(e.p, n_steps, se)
    assert need > _lib.NOALLOC_SCRATCH_BYTES
    s = torch.empty((n_steps // se + 1, 8), dtype=torch.float64, device="cuda")
    lnw0 = e.lnw.clone()
    with pytest.raises(_lib.HeFkError) as ei:
        api.he_fk_propagate_noalloc(e.p, e.walkers(), 0, n_steps, se, s.data_ptr(), 0, 0)
    assert ei.value.code == _lib.HE_FK_ESCRATCH
    torch.cuda.synchronize()
    assert torch.equal(lnw0, e.lnw)         # nothing ran

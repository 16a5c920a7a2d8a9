"""One GPU's share of a mesh split into z slabs (DG_ZHALO): two slab contexts on
one GPU, their halo planes exchanged by device copies before every stage (the
transfer a second GPU would make over xGMI), reproduce the whole periodic mesh
bit for bit, with the driving placed by dg_set_slab.  Expected values come from
the library's own whole-mesh run, which the other GPU tests pin to the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

G = 5.0 / 3.0


@pytest.fixture(scope="module")
def dgm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_09079_amd import dg
    dg.lib()
    return dg


def driving(dgm):
    from paper_1602_09079_amd import synth
    nvec = synth.forcing_modes(1.0, 3.0)
    th = synth.ou_stationary_start(11, len(nvec))
    z = synth.ou_normals(11, len(nvec), 1)[0]
    _, ah = dgm.ou_update(nvec, th, z, 0.9, 1.0, 1.0, 1.0, 3.0)
    return nvec, ah


@pytest.mark.parametrize("prec,k", [("fp64", 2), ("fp32", 3), ("bf16x3", 3), ("bf16", 1), ("fp32", 0),
                                    ("fp64", 3), ("fp64", 4), ("fp32", 4)])
@pytest.mark.parametrize("nslab", [2, 3])
def test_slabs_reproduce_whole_mesh(dgm, prec, k, nslab):
    from paper_1602_09079_amd import synth
    nx, ny, nz = 20, 9, 12
    whole = dgm.Solver(k, (nx, ny, nz), gamma=G, precision=prec, forcing=True)
    nvec, ah = driving(dgm)
    whole.set_forcing(nvec, ah)
    qp = synth.turbulence((nx, ny, nz), dgm.gauss_nodes(k + 1), seed=21, mach=0.5, device="cuda", dtype=whole.dtype)
    y = whole.project(qp)
    h = 0.5 * whole.dt(y)
    dz = nz // nslab
    slabs = []
    for j in range(nslab):
        s = dgm.Solver(k, (nx, ny, dz), box=(1.0, 1.0, dz / nz), gamma=G, precision=prec, forcing=True, zhalo=True)
        s.set_slab(j * dz, nz)
        s.set_forcing(nvec, ah)
        slabs.append(s)
    ys = [y[j * dz:(j + 1) * dz].clone() for j in range(nslab)]
    w1s = [torch.empty_like(v) for v in ys]
    w2s = [torch.empty_like(v) for v in ys]
    halos = [(torch.empty_like(v[0]), torch.empty_like(v[0])) for v in ys]
    for j, s in enumerate(slabs):
        s.set_halo(*halos[j])

    def exchange(inputs):
        for j in range(nslab):
            halos[j][0].copy_(inputs[(j - 1) % nslab][-1])  # the plane below: the lower slab's top plane
            halos[j][1].copy_(inputs[(j + 1) % nslab][0])   # the plane above: the upper slab's bottom plane

    # one SSP-RK3 step, stage by stage
    w1, w2 = torch.empty_like(y), torch.empty_like(y)
    whole.stage(y, y, w1, 0.0, 1.0, h)
    whole.stage(y, w1, w2, 0.75, 0.25, h)
    whole.stage(y, w2, w1, 1 / 3, 2 / 3, h)
    exchange(ys)
    for j, s in enumerate(slabs):
        s.stage(ys[j], ys[j], w1s[j], 0.0, 1.0, h)
    exchange(w1s)
    for j, s in enumerate(slabs):
        s.stage(ys[j], w1s[j], w2s[j], 0.75, 0.25, h)
    exchange(w2s)
    for j, s in enumerate(slabs):
        s.stage(ys[j], w2s[j], w1s[j], 1 / 3, 2 / 3, h)
    got = torch.cat(w1s)
    assert torch.equal(got, w1), (got - w1).abs().max().item()


def test_slab_errors(dgm):
    s = dgm.Solver(1, (8, 8, 4), gamma=G, precision="fp64", zhalo=True)
    y = torch.ones(s.state_shape(), dtype=torch.float64, device="cuda")
    with pytest.raises(dgm.DGError) as e:
        s.rhs(y)  # no halo planes yet
    assert e.value.status == dgm.DG_ERR_STATE
    with pytest.raises(dgm.DGError) as e:
        s.set_slab(6, 8)  # 6 + 4 > 8
    assert e.value.status == dgm.DG_ERR_ARG
    s.set_halo(y[0].clone(), y[0].clone())
    with pytest.raises(dgm.DGError) as e:
        s.step(y, 1, 1e-3)  # halos cannot be exchanged between dg_step's stages
    assert e.value.status == dgm.DG_ERR_UNSUPPORTED
    plain = dgm.Solver(1, (8, 8, 4), gamma=G, precision="fp64")
    with pytest.raises(dgm.DGError) as e:
        plain.set_halo(y[0], y[0])
    assert e.value.status == dgm.DG_ERR_STATE

"""The streaming-rate probe (a measurement aid beside the sweeps' roofline):
every output block is the elementwise sum of the input blocks, at sizes that
end inside a workgroup tile, with grids above and below the tile count."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nin,nout,count,nwg", [(1, 1, 2, 0), (3, 2, 1000, 0), (10, 1, 131074, 512),
                                                  (16, 4, 4096 * 8 + 6, 7), (2, 0, 512, 3)])
def test_stream_probe_sums_its_inputs(nin, nout, count, nwg):
    import paper_1604_01713_amd as bg
    dev = torch.device("cuda:0")
    g = torch.Generator(device="cpu").manual_seed(1000 + nin)
    ins = [torch.randn(count, generator=g, dtype=torch.float64).to(dev) for _ in range(nin)]
    outs = [torch.full((count,), float("nan"), dtype=torch.float64, device=dev) for _ in range(nout)]
    bg.bgcr_stream_probe(ins, outs, nwg)
    torch.cuda.synchronize()
    ref = torch.zeros(count, dtype=torch.float64)
    for t in ins:
        ref = ref + t.cpu()
    for o in outs:
        # the kernel adds the inputs in index order, as the reference does
        assert torch.equal(o.cpu(), ref)

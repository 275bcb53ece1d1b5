"""The library's launches captured in a HIP graph (the calls are
stream-ordered and enqueue no memset): every replay, with eager work and
synchronisations between replays, reproduces the eager result exactly."""
import pytest
import torch

from gpu_util import inputs

pytestmark = pytest.mark.gpu


def ops():
    from paper_2604_08542_amd import ops
    return ops


@pytest.mark.parametrize("io,save_ckpt", [("f32", True), ("bf16", False)])
def test_forward_graph_replays(gpu, io, save_ckpt):
    N, H, h, M, eta = 2000, 2, 256, 300, 0.05
    _, dev = inputs(N, H, h, seed=900, io=io)
    O = torch.empty_like(dev["Q"])
    prob = ops().problem(dev["Q"], h, N, M, eta, ops()._flags(True, save_ckpt=save_ckpt))
    ws = ops().workspace(prob, 1, dev["Q"].device)
    ck = {}

    def run():
        r = ops().chunk_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], eta, M, out=O, ws=ws,
                            save_ckpt=save_ckpt)
        ck["r"] = r
    run()
    torch.cuda.synchronize()
    ref_o = O.clone()
    ref_w = ck["r"]["W1_T"].clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        run()
    torch.cuda.synchronize()
    captured = ck["r"]
    for i in range(3):
        O.zero_()
        captured["W1_T"].zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(O, ref_o), i
        assert torch.equal(captured["W1_T"], ref_w), i
        # eager work between replays
        run()
        torch.cuda.synchronize()
        assert torch.equal(O, ref_o), i


def test_backward_graph_replays(gpu):
    N, H, h, M, eta = 1200, 2, 256, 400, 0.05
    _, dev = inputs(N, H, h, seed=910, io="bf16", with_dO=True)
    f = ops().chunk_fwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], eta, M, save_ckpt=True)
    out = {}

    def run():
        out["g"] = ops().chunk_bwd(dev["Q"], dev["K"], dev["V"], dev["W1"], dev["W2"], eta, M, f["ckpt"], dev["dO"])
    run()
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in out["g"].items()}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        run()
    torch.cuda.synchronize()
    captured = out["g"]
    for i in range(3):
        for v in captured.values():
            v.zero_()
        g.replay()
        torch.cuda.synchronize()
        for k, v in ref.items():
            assert torch.equal(captured[k], v), (i, k)
        run()
        torch.cuda.synchronize()

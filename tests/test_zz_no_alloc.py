"""The allocation-free training step (gbp_mlp_train_step_static) against the
workspace form (gbp_mlp_train_step), both through the C ABI: two calls in a
row, the second on a smaller batch, must give bitwise the same loss,
gradient, master weights, Adam moments and BF16 copy."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _state(torch, theta0, dev):
    st = dict(theta=torch.as_tensor(theta0.copy()).to(dev),
              m=torch.zeros(theta0.size, dtype=torch.float32, device=dev),
              v=torch.zeros(theta0.size, dtype=torch.float32, device=dev),
              w=torch.zeros(theta0.size, dtype=torch.int16, device=dev),
              grad=torch.zeros(theta0.size, dtype=torch.float32, device=dev),
              loss=torch.zeros(1, dtype=torch.float32, device=dev))
    return st


def test_static_training_step_matches_workspace_form():
    import torch
    from paper_2003_03134_amd import _capi, init_mlp_params
    lib = _capi.load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    P = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    gen = torch.Generator(device="cuda").manual_seed(7)
    n_rows = 20000
    x = torch.randn(n_rows, 16, device=dev, generator=gen)
    y = torch.rand(n_rows, 2, device=dev, generator=gen)
    mask = (torch.rand(n_rows, 2, device=dev, generator=gen) > 0.3).float()
    theta0 = init_mlp_params(3)
    a, b = _state(torch, theta0, dev), _state(torch, theta0, dev)
    nbytes = C.c_size_t(0)
    assert lib.gbp_mlp_train_workspace_bytes(_capi.GBP_MLP_STATIC_MAX_BATCH, C.byref(nbytes)) == 0
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream(dev)
    sp = C.c_void_p(stream.cuda_stream)
    # the full fixed capacity first, then a smaller, ragged batch with an
    # out-of-range index (a zero-weight sample)
    batches = [torch.randint(0, n_rows, (_capi.GBP_MLP_STATIC_MAX_BATCH,), device=dev, generator=gen,
                             dtype=torch.int32),
               torch.cat([torch.randint(0, n_rows, (1000,), device=dev, generator=gen, dtype=torch.int32),
                          torch.tensor([n_rows + 5], dtype=torch.int32, device=dev)])]
    for step, idx in enumerate(batches, start=1):
        print(f"static training step: call {step}, batch {idx.numel()}", flush=True)
        st = lib.gbp_mlp_train_step(P(x), P(y), P(mask), n_rows, P(idx), idx.numel(), P(a["theta"]), P(a["m"]),
                                    P(a["v"]), P(a["w"]), C.c_float(1e-3), step, P(a["grad"]), P(a["loss"]),
                                    P(ws), ws.numel(), sp)
        assert st == 0, lib.gbp_last_error(None)
        st = lib.gbp_mlp_train_step_static(P(x), P(y), P(mask), n_rows, P(idx), idx.numel(), P(b["theta"]),
                                           P(b["m"]), P(b["v"]), P(b["w"]), C.c_float(1e-3), step,
                                           P(b["grad"]), P(b["loss"]), sp)
        assert st == 0, lib.gbp_last_error(None)
        torch.cuda.synchronize()
        for key in a:
            assert torch.equal(a[key], b[key]), (step, key)
        assert float(b["loss"].item()) > 0.0
    # a batch beyond the fixed scratch is refused before any device work
    big = torch.zeros(_capi.GBP_MLP_STATIC_MAX_BATCH + 1, dtype=torch.int32, device=dev)
    st = lib.gbp_mlp_train_step_static(P(x), P(y), P(mask), n_rows, P(big), big.numel(), P(b["theta"]),
                                       P(b["m"]), P(b["v"]), P(b["w"]), C.c_float(1e-3), 3, P(b["grad"]),
                                       P(b["loss"]), sp)
    assert st == _capi.GBP_EINVAL and b"exceeds" in lib.gbp_last_error(None)

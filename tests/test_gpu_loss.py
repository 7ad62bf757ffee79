"""The fused L1 loss (the objective the reverse pass trains against) and its
autograd wrapper against the plain definition: mean |image - target| and
dL/dimage = sign(image - target) / n, zero where they are equal.  The loss
is a float32 sum with atomically added block partials (within 1e-5
relative); the gradient is one rounding of 1 / n times a sign, so it equals
torch's to the last bit up to the rounding of 1 / n."""
import pytest
import torch

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("offset", [0, 1])
@pytest.mark.parametrize("n", [1, 3, 4, 1000, 4099, 3 * 1280 * 720 + 7])
def test_l1_loss_and_grad_match_definition(n, offset):
    """offset 1 starts the images one float into their buffers (the
    unaligned path; aligned buffers take four floats per load)."""
    need_gpu()
    import paper_2407_00435_amd as g
    say(f"l1 loss n={n} offset={offset}")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(n)
    img = torch.rand(n + offset, device="cuda", generator=gen)[offset:]
    tgt = torch.rand(n + offset, device="cuda", generator=gen)[offset:]
    tgt[::5] = img[::5]  # ties take a zero gradient
    a = img.clone().requires_grad_(True)
    b = img.clone().requires_grad_(True)
    la = g.l1_loss(a, tgt)
    la.backward()
    lb = (b - tgt).abs().mean()
    lb.backward()
    assert la.shape == ()
    assert abs(la.item() - lb.item()) <= 1e-5 * lb.item() + 1e-30
    torch.testing.assert_close(a.grad, b.grad, rtol=2e-7, atol=0)
    assert torch.all(a.grad[::5] == 0)
    # an upstream gradient scales the result
    a.grad = None
    (3.0 * g.l1_loss(a, tgt)).backward()
    torch.testing.assert_close(a.grad, 3.0 * b.grad, rtol=2e-7, atol=0)

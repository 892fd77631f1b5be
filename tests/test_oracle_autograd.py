"""FP64 gradcheck of an oracle-backed autograd Function (CPU).

The same backward structure as the GPU Function (transpose map for the data,
delay derivative for the sound speed), built from the oracle alone: pins the
adjoint formulas against torch's numerical Jacobian.
"""
import numpy as np

import oracle


def test_gradcheck_oracle_backed_function():
    # FP64 gradcheck of a tiny oracle-backed Function with the same backward
    # structure (transpose map for e, delay derivative for c): pins the
    # adjoint formulas themselves, independently of the GPU.
    import torch
    from synth.configs import MM, describe
    d = describe("forces", (5, 5), (0.3 * MM, 0.3 * MM), 3, 4, 120, 20e6, 5e6, (3, 1, 4),
                 (-0.5 * MM, 0, 1.5 * MM), (0.5 * MM, 0, 2.5 * MM), f_number=0.8)

    class OracleDas(torch.autograd.Function):
        @staticmethod
        def forward(ctx, e, c):
            ctx.save_for_backward(e, c)
            return torch.from_numpy(oracle.das(d, e.detach().numpy(), c=float(c)))

        @staticmethod
        def backward(ctx, g):
            e, c = ctx.saved_tensors
            G = g.detach().numpy()
            ge = torch.from_numpy(oracle.das_adjoint_e(d, G, c=float(c)))
            gc = float(np.sum(G * oracle.das_dc(d, e.detach().numpy(), c=float(c))))
            return ge, torch.tensor(gc, dtype=torch.float64)

    rng = np.random.default_rng(0)
    e = torch.tensor(rng.normal(size=(3, 4, 120)), dtype=torch.float64, requires_grad=True)
    c = torch.tensor(1530.0, dtype=torch.float64, requires_grad=True)
    assert torch.autograd.gradcheck(OracleDas.apply, (e, c), eps=1e-3, atol=1e-5, rtol=1e-3)

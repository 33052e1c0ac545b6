"""The paper's learning objective (SFSeg++) on the GPU against the FP64
oracle: Eq. 9's sigmoid-affine combination and its backward, the per-frame
Focal-Dice loss of Eq. 12 and its gradient, and the whole objective
(continuous and soft-binarised iterations of Alg. 1) end to end: loss and
dL/dw, dL/db in FP64 (<= 1e-9 relative) and FP32 (<= 1e-4), torch gradcheck
in FP64, and AdamW training that lowers the loss on the channel workload."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import Kernel as OK

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def L():
    import paper_2212_08058_amd as P
    from paper_2212_08058_amd import learn
    return P, learn


def okf(k):
    return OK(float(np.float32(k.sigma_s)), float(np.float32(k.sigma_t)), k.r_s, k.r_t)


def _case(seed, C=4, shape=(4, 20, 28)):
    rng = np.random.default_rng(seed)
    fc = rng.uniform(0.0, 1.0, (C,) + shape)
    gt = (rng.uniform(size=shape) > 0.6)
    return fc, gt, rng.standard_normal(C) * 0.8, 0.3


@pytest.mark.parametrize("dtype,bar", [(torch.float64, 1e-12), (torch.float32, 2e-6)])
def test_combine_sigmoid_and_focal_dice(L, dtype, bar):
    P, Lm = L
    from paper_2212_08058_amd import _native as N
    fc, gt, w, b = _case(1)
    if dtype == torch.float32:
        fc = fc.astype(np.float32).astype(np.float64)
    fcd = torch.from_numpy(fc).to(DEV).to(dtype)
    wd = torch.from_numpy(w).to(DEV)
    bd = torch.tensor([b], dtype=torch.float64, device=DEV)
    f = torch.empty(fc.shape[1:], dtype=dtype, device=DEV)
    code = N.STPI_F64 if dtype == torch.float64 else N.STPI_F32
    n = f.numel()
    N.check(N.lib.stpi_combine_sigmoid_fwd(4, n, code, fcd.data_ptr(), wd.data_ptr(), bd.data_ptr(), f.data_ptr(),
                                           None))
    fr = oracle.combine_sigmoid(fc, w, b)
    assert np.max(np.abs(f.double().cpu().numpy() - fr)) <= bar
    g_f = np.random.default_rng(2).standard_normal(fr.shape)
    gwb = torch.empty(5, dtype=torch.float64, device=DEV)
    aux = torch.empty(N.AUX_WS_BYTES, dtype=torch.uint8, device=DEV)
    N.check(N.lib.stpi_combine_sigmoid_bwd(4, n, code, fcd.data_ptr(), f.data_ptr(),
                                           torch.from_numpy(g_f).to(DEV).to(dtype).data_ptr(), gwb.data_ptr(),
                                           aux.data_ptr(), aux.numel(), None))
    gw, gb = oracle.combine_sigmoid_bwd(fc, w, b, g_f.astype(np.float32).astype(np.float64) if dtype == torch.float32
                                        else g_f)
    got = gwb.cpu().numpy()
    assert np.max(np.abs(got[:4] - gw)) <= 1e3 * bar * np.max(np.abs(gw)) and abs(got[4] - gb) <= 1e3 * bar * abs(gb)
    x = np.random.default_rng(3).uniform(0.0, 1.0, gt.shape)
    if dtype == torch.float32:
        x = x.astype(np.float32).astype(np.float64)
    loss = Lm.focal_dice(torch.from_numpy(x).to(DEV).to(dtype).requires_grad_(), torch.from_numpy(gt).to(DEV))
    J, gx = oracle.focal_dice(x, gt, 0.75, 1.0)
    loss.backward()
    print(dtype, "focal dice", float(loss), J)
    assert abs(float(loss) - J) <= 10 * bar * J


@pytest.mark.parametrize("n_iter,n_cont", [(6, 3), (5, 5), (4, 0)])
def test_objective_end_to_end_fp64(L, n_iter, n_cont):
    P, Lm = L
    fc, gt, w, b = _case(4)
    kern = P.Kernel(2.0, 1.0, 2, 1)
    fcd = torch.from_numpy(fc).to(DEV)
    wd = torch.from_numpy(w).to(DEV).requires_grad_()
    bd = torch.tensor(b, dtype=torch.float64, device=DEV, requires_grad=True)
    x = Lm.sfseg_pp(fcd, wd, bd, kern, n_iter, n_cont, 2.0, 1.0)
    J = Lm.focal_dice(x, torch.from_numpy(gt).to(DEV))
    J.backward()
    Jr, gw, gb, tape = oracle.loss_and_grad_pp(fc, w, b, gt.astype(np.float64), okf(kern), n_iter, n_cont, 2.0, 1.0)
    xerr = float(np.linalg.norm(x.detach().cpu().numpy() - tape["xs"][-1]) / np.linalg.norm(tape["xs"][-1]))
    gerr = float(np.max(np.abs(wd.grad.cpu().numpy() - gw)) / np.max(np.abs(gw)))
    print(f"n_iter {n_iter} n_cont {n_cont}: x {xerr:.2e}, J {float(J):.12g} vs {Jr:.12g}, dJ/dw {gerr:.2e}, "
          f"dJ/db {float(bd.grad):.10g} vs {gb:.10g}")
    assert xerr <= 1e-12 and abs(float(J) - Jr) <= 1e-12 * Jr
    assert gerr <= 1e-9 and abs(float(bd.grad) - gb) <= 1e-9 * max(1.0, abs(gb))


def test_objective_fp32_and_gradcheck(L):
    P, Lm = L
    fc, gt, w, b = _case(5, C=3, shape=(4, 16, 16))
    kern = P.Kernel(2.0, 1.0, 2, 1)
    # FP32 forward and gradient against the FP64 oracle on the float-rounded input
    fc32 = fc.astype(np.float32)
    wd = torch.from_numpy(w).to(DEV).requires_grad_()
    bd = torch.tensor(b, dtype=torch.float64, device=DEV, requires_grad=True)
    x = Lm.sfseg_pp(torch.from_numpy(fc32).to(DEV), wd, bd, kern, 6, 3, 2.0, 1.0)
    J = Lm.focal_dice(x, torch.from_numpy(gt).to(DEV))
    J.backward()
    Jr, gw, gb, _ = oracle.loss_and_grad_pp(fc32, w, b, gt.astype(np.float64), okf(kern), 6, 3, 2.0, 1.0)
    gerr = float(np.max(np.abs(wd.grad.cpu().numpy() - gw)) / np.max(np.abs(gw)))
    print(f"fp32: J {float(J):.8g} vs {Jr:.8g}, dJ/dw {gerr:.2e}")
    assert abs(float(J) - Jr) <= 1e-5 * Jr and gerr <= 1e-4
    # gradcheck through the library's kernels, FP64
    fcd = torch.from_numpy(fc).to(DEV)
    gtd = torch.from_numpy(gt).to(DEV)

    def fn(w_, b_):
        return Lm.focal_dice(Lm.sfseg_pp(fcd, w_, b_, kern, 4, 2, 2.0, 1.0), gtd)

    assert torch.autograd.gradcheck(fn, (torch.from_numpy(w).to(DEV).requires_grad_(),
                                         torch.tensor(b, dtype=torch.float64, device=DEV, requires_grad=True)),
                                    eps=1e-6, atol=1e-7, rtol=1e-5)


def test_training_lowers_the_focal_dice_loss(L):
    """The channel workload (C = 8: three channels with U noise, five with 20%
    salt-and-pepper, random dilation / erosion) at 16 x 120 x 216: AdamW on the
    library's gradients lowers the Focal-Dice objective."""
    P, Lm = L
    fc, gt = synth.channel_stack(8, 16, 120, 216, seed=7)
    kern = P.Kernel(2.0, 1.0, 4, 2)
    fcd = torch.from_numpy(fc).to(DEV)
    gtd = torch.from_numpy(gt).to(DEV)
    w = torch.zeros(8, dtype=torch.float64, device=DEV, requires_grad=True)
    b = torch.zeros((), dtype=torch.float64, device=DEV, requires_grad=True)
    opt = Lm.AdamW([w, b.reshape(1)], lr=0.05, weight_decay=0.0)
    losses = []
    for _ in range(12):
        w.grad = None
        b.grad = None
        J = Lm.focal_dice(Lm.sfseg_pp(fcd, w, b, kern, 10, 6, 2.0, 1.0), gtd)
        J.backward()
        opt.step([w.grad, b.grad.reshape(1)])
        losses.append(float(J))
    print("focal-dice losses", [round(v, 4) for v in losses], "weights", w.detach().cpu().numpy().round(3))
    assert losses[-1] < losses[0]


def test_learned_weights_favour_the_clean_channels(L):
    """The paper's noise study (Sec. 5, learned channel weights): trained with
    its own objective (Eq. 9 sigmoid-affine combination, soft-binarised
    iterations, Focal-Dice), the weights favour the channels with mild noise
    over those with salt-and-pepper noise. Channel workload (C = 8,
    32 x 240 x 432: channels 0-2 with U[0, 0.1] noise, 3-7 with 20%
    salt-and-pepper), 90 AdamW steps from w = 0, b = 0."""
    P, Lm = L
    c = synth.CONFIGS["channels"]
    fc, gt = synth.channel_stack(c["C"], c["T"], c["H"], c["W"], seed=c["seed"])
    kern = P.Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    fcd = torch.from_numpy(fc).to(DEV)
    gtd = torch.from_numpy(gt).to(DEV)
    w = torch.zeros(c["C"], dtype=torch.float64, device=DEV, requires_grad=True)
    b = torch.zeros((), dtype=torch.float64, device=DEV, requires_grad=True)
    opt = Lm.AdamW([w, b.reshape(1)], lr=0.05, weight_decay=0.0)
    losses = []
    for _ in range(90):
        w.grad = None
        b.grad = None
        J = Lm.focal_dice(Lm.sfseg_pp(fcd, w, b, kern, 15, 10, 2.0, 1.0), gtd)
        J.backward()
        opt.step([w.grad, b.grad.reshape(1)])
        losses.append(float(J.detach()))
    wv = w.detach().cpu().numpy()
    clean, sp = wv[:3].mean(), wv[3:].mean()
    print(f"losses {losses[0]:.4f} -> {losses[-1]:.4f}, weights {np.round(wv, 3)}, clean mean {clean:.3f}, "
          f"salt-and-pepper mean {sp:.3f}")
    assert losses[-1] < losses[0]
    assert clean > 1.2 * sp > 0

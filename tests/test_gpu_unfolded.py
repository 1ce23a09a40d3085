"""Unfolded TASER (per-iteration step sizes) and its hand-written adjoint,
through the C ABI, against the FP64 oracle: the forward against
oracle.taser_iterate / oracle.unfolded_forward, the gradient against torch
autograd through oracle.unfolded_forward and against finite differences of
the HIP forward itself (torch.autograd.gradcheck in FP64)."""
import numpy as np
import pytest

import oracle
import sim
from oracle.unfolded import last_row_mse, unfolded_forward as oracle_unfolded
from parity import L_REL_TOL, rel_frobenius, unpack_lower

pytestmark = pytest.mark.gpu


def problem(B, U, mod, V, snr, seed):
    """FP64 preprocessing by the oracle: T~, D, ||T~||_2 and the target sbar."""
    d = sim.gen_mimo(B, U, mod, V, 1, snr, seed)
    s = d["s"]
    T = oracle.build_T_coherent(d["H"], d["y"], mod)
    D, Tt, deg = oracle.precondition(T)
    assert not deg.any()
    lam = oracle.spectral_norm(Tt)
    sbar = np.concatenate([s.real, s.imag], axis=-1) if mod == oracle.QPSK else s.real
    return Tt, D, lam, np.sign(sbar)


def to_dev(dtype, *arrays):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda() for a in arrays]


def oracle_grad(Tt, D, lam, alpha, sbar, pin_last=True):
    import torch
    Tt_, D_, lam_, s_ = (torch.from_numpy(np.asarray(a, dtype=np.float64)) for a in (Tt, D, lam, sbar))
    a = torch.tensor(alpha, dtype=torch.float64, requires_grad=True)
    L = oracle_unfolded(Tt_, D_, lam_, a, pin_last=pin_last)
    loss = last_row_mse(L, D_, s_)
    loss.backward()
    return L.detach().numpy(), loss.item(), a.grad.numpy()


def gpu_grad(taser, unf, Tt, D, lam, alpha, sbar, dtype, ckpt_every=None, literal_last=False):
    import torch
    Tt_, D_, lam_, s_ = to_dev(dtype, Tt, D, lam, sbar)
    a = torch.tensor(alpha, dtype=dtype, device="cuda", requires_grad=True)
    L = unf.unfolded(a, Tt_, D_, lam_, ckpt_every, literal_last)
    loss = unf.mse_loss(L, D_, s_)
    loss.backward()
    torch.cuda.synchronize()
    N = Tt.shape[-1]
    return unpack_lower(L.detach().cpu().numpy().astype(np.float64), N), loss.item(), \
        a.grad.cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def unf(gpu_lib):
    import paper_1609_01797_amd.unfolded as u
    return u


@pytest.mark.parametrize("B,U,mod,t_max,alpha", [
    (64, 16, oracle.QPSK, 10, 0.5),      # N = 33
    (32, 8, oracle.BPSK, 7, 0.9),        # N = 9
    (128, 63, oracle.BPSK, 3, 0.5),      # N = 64, the largest
])
def test_constant_schedule_is_algorithm_1(gpu_lib, unf, B, U, mod, t_max, alpha):
    """alpha_t = alpha for all t gives the paper's algorithm (FP64 and FP32)."""
    import torch
    Tt, D, lam, _ = problem(B, U, mod, 24, 8.0, sim.seed_for(40, t_max))
    L_ref, _ = oracle.taser_iterate(Tt, D, alpha / lam, t_max)
    N = Tt.shape[-1]
    for dtype, tol in ((torch.float64, 1e-12), (torch.float32, L_REL_TOL)):
        Tt_, D_, lam_ = to_dev(dtype, Tt, D, lam)
        a = torch.full((t_max,), alpha, dtype=dtype, device="cuda")
        L, _, _ = gpu_lib.unfolded_forward(Tt_, D_, lam_, a)
        torch.cuda.synchronize()
        got = unpack_lower(L.cpu().numpy().astype(np.float64), N)
        assert np.max(rel_frobenius(got, L_ref)) <= tol, dtype


@pytest.mark.parametrize("literal_last", [False, True])
def test_schedule_forward_and_gradient_fp64(gpu_lib, unf, literal_last):
    """A varying schedule: forward and dLoss/dalpha equal torch autograd
    through the oracle in FP64."""
    Tt, D, lam, sbar = problem(32, 8, oracle.QPSK, 40, 6.0, sim.seed_for(41))
    import torch
    alpha = np.linspace(0.3, 1.1, 9)
    L_ref, loss_ref, g_ref = oracle_grad(Tt, D, lam, alpha, sbar, pin_last=not literal_last)
    L, loss, g = gpu_grad(gpu_lib, unf, Tt, D, lam, alpha, sbar, torch.float64,
                          literal_last=literal_last)
    assert np.max(np.abs(L - L_ref)) <= 1e-12 * np.max(np.abs(L_ref))
    assert abs(loss - loss_ref) <= 1e-12 * abs(loss_ref)
    assert np.max(np.abs(g - g_ref)) <= 1e-10 * np.max(np.abs(g_ref)), (g, g_ref)


def test_gradcheck_fp64(gpu_lib, unf):
    """Finite differences of the HIP forward against the HIP adjoint, on
    every entry of L (N = 9: U = 4 QPSK, B = 16, 4 vectors, t_max = 5)."""
    import torch
    Tt, D, lam, _ = problem(16, 4, oracle.QPSK, 4, 5.0, sim.seed_for(42))
    Tt_, D_, lam_ = to_dev(torch.float64, Tt, D, lam)
    a = torch.tensor([0.4, 0.7, 0.5, 0.9, 0.6], dtype=torch.float64, device="cuda",
                     requires_grad=True)
    for c in (1, 2, 5):
        assert torch.autograd.gradcheck(lambda x: unf.unfolded(x, Tt_, D_, lam_, c), (a,),
                                        eps=1e-6, atol=1e-8, rtol=1e-6)


def test_checkpoint_interval_does_not_change_gradient(gpu_lib, unf):
    """Recomputing segments from checkpoints repeats the forward bit for bit:
    every checkpoint interval gives the same gradient, and two backward
    passes are identical (the batch reduction has a fixed order)."""
    import torch
    Tt, D, lam, sbar = problem(64, 16, oracle.QPSK, 300, 8.0, sim.seed_for(43))
    alpha = np.linspace(0.2, 0.9, 12)
    ref = None
    for c in (1, 3, 4, 12, 20):
        for _ in range(2):
            _, loss, g = gpu_grad(gpu_lib, unf, Tt, D, lam, alpha, sbar, torch.float32, ckpt_every=c)
            if ref is None:
                ref = (loss, g)
            assert loss == ref[0] and np.array_equal(g, ref[1]), c


def test_fp32_gradient_close_to_fp64(gpu_lib, unf):
    """The FP32 adjoint on a B = 64, U = 16 QPSK batch at 0 dB (N = 33,
    t_max = 20) against the FP64 oracle gradient."""
    import torch
    Tt, D, lam, sbar = problem(64, 16, oracle.QPSK, 200, 0.0, sim.seed_for(44))
    alpha = np.full(20, 0.5) + 0.02 * np.arange(20)
    L_ref, loss_ref, g_ref = oracle_grad(Tt, D, lam, alpha, sbar)
    L, loss, g = gpu_grad(gpu_lib, unf, Tt, D, lam, alpha, sbar, torch.float32)
    assert abs(loss - loss_ref) <= 1e-4 * abs(loss_ref)
    assert np.max(np.abs(g - g_ref)) <= 1e-3 * np.max(np.abs(g_ref)), (g, g_ref)


@pytest.mark.parametrize("dtype_name", ["float32", "float64"])
def test_empty_batch_backward_gives_zero_gradient(gpu_lib, dtype_name):
    """dLoss/dalpha is a sum over the batch, so an empty batch has gradient
    zero: the backward of V = 0 writes zeros into its uninitialised output
    (a NaN-filled block of the same size is freed just before, so the
    caching allocator hands that memory back)."""
    import torch
    dt = getattr(torch, dtype_name)
    N, t_max = 33, 6
    Tt = torch.empty((0, N, N), dtype=dt, device="cuda")
    D = torch.empty((0, N), dtype=dt, device="cuda")
    lam = torch.empty((0,), dtype=dt, device="cuda")
    alpha = torch.full((t_max,), 0.5, dtype=dt, device="cuda")
    L, ckpt, u = gpu_lib.unfolded_forward(Tt, D, lam, alpha)
    assert L.shape == (0, N * (N + 1) // 2)
    dL = torch.empty((0, N * (N + 1) // 2), dtype=dt, device="cuda")
    junk = torch.full((t_max,), float("nan"), dtype=dt, device="cuda")
    del junk
    torch.cuda.synchronize()
    g = gpu_lib.unfolded_backward(u, Tt, D, lam, alpha, ckpt, dL)
    torch.cuda.synchronize()
    assert torch.equal(g, torch.zeros_like(g))


def test_training_lowers_loss(gpu_lib, unf):
    """A few Adam steps on the step sizes (FP32 kernels) lower the training
    loss on fresh batches, and the schedule stays finite."""
    import torch
    B, U, mod, t_max = 64, 16, oracle.QPSK, 10
    alpha = torch.full((t_max,), 0.1, dtype=torch.float32, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([alpha], lr=0.05)

    def batch(i):
        d = sim.gen_training_batch(B, U, mod, 512, 4.0, 16.0, sim.seed_for(45, 0, i))
        T = oracle.build_T_coherent(d["H"], d["y"], mod)
        D, Tt, _ = oracle.precondition(T)
        s = d["s"]
        sbar = np.concatenate([s.real, s.imag], axis=-1)
        return to_dev(torch.float32, Tt, D, oracle.spectral_norm(Tt), sbar)

    test = batch(1000)

    def test_loss():
        with torch.no_grad():
            L = unf.unfolded(alpha, *test[:3])
            return float(unf.mse_loss(L, test[1], test[3]))

    before = test_loss()
    for i in range(30):
        Tt_, D_, lam_, s_ = batch(i)
        opt.zero_grad()
        loss = unf.mse_loss(unf.unfolded(alpha, Tt_, D_, lam_), D_, s_)
        loss.backward()
        opt.step()
    after = test_loss()
    assert torch.isfinite(alpha).all()
    assert after < 0.9 * before, (before, after)


@pytest.mark.parametrize("B,U,mod,V,literal", [
    (64, 16, oracle.QPSK, 25, False),   # N = 33, two vectors per wave, odd batch (one idle half)
    (32, 8, oracle.QPSK, 31, True),     # N = 17, two vectors per wave, literal L~_NN
    (48, 40, oracle.BPSK, 7, False),    # N = 41, one vector per wave
])
def test_fp32_layouts_forward_and_gradient(gpu_lib, unf, B, U, mod, V, literal):
    """FP32 forward and gradient against the FP64 oracle for the wave
    layouts the kernels choose between (two vectors per wave with an idle
    half, literal last column, one vector per wave)."""
    import torch
    Tt, D, lam, sbar = problem(B, U, mod, V, 1.0, sim.seed_for(46, V))
    alpha = np.linspace(0.4, 0.9, 6)
    L_ref, loss_ref, g_ref = oracle_grad(Tt, D, lam, alpha, sbar, pin_last=not literal)
    L, loss, g = gpu_grad(gpu_lib, unf, Tt, D, lam, alpha, sbar, torch.float32, literal_last=literal)
    assert np.max(rel_frobenius(L, L_ref)) <= L_REL_TOL
    assert abs(loss - loss_ref) <= 1e-4 * abs(loss_ref)
    assert np.max(np.abs(g - g_ref)) <= 1e-3 * np.max(np.abs(g_ref)), (g, g_ref)


def test_training_batch_full_size(gpu_lib, unf):
    """The training configuration: 16,384 vectors of 64x16 QPSK with SNR
    U[4, 16] dB, t_max = 20.  The forward is checked against the oracle on
    256 sampled vectors; the batch gradient, which no sample can check, by a
    property that holds at any size: the gradient of the mean loss over the
    batch is the size-weighted mean of the gradients over two halves."""
    import torch
    d = sim.gen_training_batch(64, 16, oracle.QPSK, 16384, 4.0, 16.0, sim.seed_for(4, 7, 0))
    T = oracle.build_T_coherent(d["H"], d["y"], oracle.QPSK)
    D, Tt, _ = oracle.precondition(T)
    lam = oracle.spectral_norm(Tt)
    s = d["s"]
    sbar = np.concatenate([s.real, s.imag], axis=-1)
    alpha = np.linspace(0.3, 1.0, 20)
    Tt_, D_, lam_, s_ = to_dev(torch.float32, Tt, D, lam, sbar)
    a = torch.tensor(alpha, dtype=torch.float32, device="cuda", requires_grad=True)
    L = unf.unfolded(a, Tt_, D_, lam_)
    unf.mse_loss(L, D_, s_).backward()
    g_full = a.grad.clone()
    idx = np.sort(np.random.default_rng(5).choice(16384, size=256, replace=False))
    import torch as _t
    Lref = oracle_unfolded(*(_t.from_numpy(np.asarray(x, dtype=np.float64)) for x in (Tt[idx], D[idx], lam[idx])),
                           _t.tensor(alpha, dtype=_t.float64))
    got = unpack_lower(L.detach().cpu().numpy()[idx].astype(np.float64), 33)
    assert np.max(rel_frobenius(got, Lref.numpy())) <= L_REL_TOL
    halves = []
    for sl in (slice(0, 10000), slice(10000, 16384)):
        a2 = torch.tensor(alpha, dtype=torch.float32, device="cuda", requires_grad=True)
        L2 = unf.unfolded(a2, Tt_[sl].contiguous(), D_[sl].contiguous(), lam_[sl].contiguous())
        unf.mse_loss(L2, D_[sl], s_[sl]).backward()
        halves.append(a2.grad.clone())
    combo = (10000 * halves[0] + 6384 * halves[1]) / 16384
    torch.cuda.synchronize()
    assert torch.allclose(g_full, combo, rtol=1e-4, atol=1e-6 * float(g_full.abs().max())), (g_full, combo)

"""Pins of the oracle's decoder sampler (the CVAE decoder of App. A used for
inference: z ~ N(0, I) through the decoder MLP with the observation o, then
Alg. 1 from those samples): the MLP against PyTorch's own layers in FP64,
the latent draws against the structured sampler's normals and N(0, I), the
sample moments against numpy, and the plan that starts from given samples
against the plan that draws the same samples itself."""
import numpy as np
import pytest

from paper_2212_02224_amd import workload


def torch_decoder(dec):
    torch = pytest.importorskip("torch")
    layers = []
    for i in range(5):
        lin = torch.nn.Linear(dec.W[i].shape[1], dec.W[i].shape[0]).double()
        bn = torch.nn.BatchNorm1d(dec.W[i].shape[0], eps=dec.eps).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(dec.W[i]))
            lin.bias.copy_(torch.from_numpy(dec.b[i]))
            bn.weight.copy_(torch.from_numpy(dec.gamma[i]))
            bn.bias.copy_(torch.from_numpy(dec.beta[i]))
            bn.running_mean.copy_(torch.from_numpy(dec.mean[i]))
            bn.running_var.copy_(torch.from_numpy(dec.var[i]))
        layers += [lin, bn, torch.nn.ReLU()]
    out = torch.nn.Linear(256, 8).double()
    with torch.no_grad():
        out.weight.copy_(torch.from_numpy(dec.W[5]))
        out.bias.copy_(torch.from_numpy(dec.b[5]))
    net = torch.nn.Sequential(*layers, out).eval()
    return torch, net


@pytest.mark.parametrize("behaviour", [0, 1])
def test_decoder_matches_torch_layers(orc, behaviour):
    """The decoder MLP equals torch.nn Linear / BatchNorm1d (eval) / ReLU
    blocks in FP64 on the same weights and inputs."""
    dec = workload.decoder_weights(3, behaviour)
    s = workload.scene(2, 7, 10)
    o = workload.observation(s)
    z = orc.decoder_latent(s.seed, 64)
    torch, net = torch_decoder(dec)
    x = torch.from_numpy(np.concatenate([np.tile(o, (64, 1)), z], axis=1))
    with torch.no_grad():
        want = net(x).numpy()
    got = orc.decoder_forward(dec, o, z, behaviour)
    if behaviour:
        assert np.all(got[:, 2:] == 0)
        want[:, 2:] = 0.0
    assert np.abs(got - want).max() <= 1e-12 * max(1.0, np.abs(want).max())


def test_decoder_with_zero_weights_is_its_biases(orc):
    """All weights 0: every block outputs relu(beta + gamma (b - mean) /
    sqrt(var + eps)), and p = W6 that + b6, the same for every z."""
    dec = workload.decoder_weights(1)
    for i in range(5):
        dec.W[i] = np.zeros_like(dec.W[i])
    h = None
    for i in range(5):
        h = np.maximum(dec.beta[i] + dec.gamma[i] * (dec.b[i] - dec.mean[i]) / np.sqrt(dec.var[i] + dec.eps), 0.0)
    want = dec.W[5] @ h + dec.b[5]
    p = orc.decoder_forward(dec, np.ones(55), orc.decoder_latent(9, 5))
    assert np.allclose(p, want[None, :], rtol=1e-12, atol=1e-12)


def test_latent_draws_are_the_structured_samplers_normals(orc):
    """z_j is the first Box-Muller pair of Philox block (j, 0, 0, 0): the
    structured sampler's lateral set-points 0 and 1 of sample j are
    lane + sigma z_j."""
    par = orc.default_params()
    N = 300
    z = orc.decoder_latent(4242, N)
    p = orc.sample(par, 4242, 0, N, True)
    lanes = np.array(list(par.lane_c))
    # lanes are 3.5 m apart and sigma is 0.3 m: the nearest centre is the lane
    lane = lanes[np.argmin(np.abs(p[:, :1] - lanes[None, :]), axis=1)]
    resid = (p[:, :2] - lane[:, None]) / par.lane_sigma
    assert np.allclose(resid, z, atol=1e-9)


def test_latent_draws_are_standard_normal(orc):
    N = 40000
    z = orc.decoder_latent(77, N)
    se = 1.0 / np.sqrt(N)
    assert np.all(np.abs(z.mean(axis=0)) < 5 * se)
    assert np.allclose(z.var(axis=0), 1.0, atol=0.03)
    assert abs(np.corrcoef(z.T)[0, 1]) < 5 * se
    assert not np.array_equal(orc.decoder_latent(78, 10), z[:10])


def test_sample_moments_match_numpy(orc):
    rng = np.random.default_rng(5)
    p = rng.standard_normal((500, 8)) * np.arange(1, 9) + np.arange(8)
    mu, S = orc.sample_moments(p)
    assert np.allclose(mu, p.mean(axis=0), rtol=1e-13, atol=1e-13)
    assert np.allclose(S, np.cov(p.T, bias=True), rtol=1e-12, atol=1e-12)


def test_plan_from_samples_uses_their_moments_as_prior(orc):
    """Started from the very samples the structured sampler would draw, the
    plan evaluates the same first iteration; only the prior of the first
    update differs (sample moments instead of the exact ones). The first mean
    differs by (1 - eta) (mean(p0) - mu_exact). The covariance is centred on
    the new mean: with m the EliteSet's weighted mean, it differs by
    (1 - eta) (cov(p0) - Sigma_exact) + eta ((m - mu_b)(m - mu_b)^T -
    (m - mu_a)(m - mu_a)^T)."""
    par = orc.default_params(T=50, M=4, K=10, L=1)
    s = workload.scene(1, 2, 4)
    sc = orc.Scene(s.ego, s.obstacles)
    N = 64
    p0 = orc.sample(par, s.seed, 0, N, True)
    a = orc.plan(par, sc, s.seed, N, trace=True)
    b = orc.plan(par, sc, s.seed, N, trace=True, p0=p0)
    assert np.array_equal(b.trace["p"][0], p0)
    for k in ("r", "cu", "ces", "es"):
        assert np.array_equal(a.trace[k][0], b.trace[k][0]), k
    mu_e, S_e = orc.initial_moments(par)
    mu_s, S_s = orc.sample_moments(p0)
    assert np.allclose(b.mu - a.mu, (1 - par.eta) * (mu_s - mu_e), atol=1e-12)
    m = (a.mu - (1 - par.eta) * mu_e) / par.eta
    want = ((1 - par.eta) * (S_s - S_e)
            + par.eta * (np.outer(m - b.mu, m - b.mu) - np.outer(m - a.mu, m - a.mu)))
    assert np.allclose(b.Sigma - a.Sigma, want, atol=1e-10)


def test_decoder_plan_runs_and_meets_its_samples(orc):
    """Alg. 1 from decoder samples: the first iteration's samples are the
    decoder's and the returned trajectory is one of a later iteration's."""
    par = orc.default_params(T=50, M=4, K=10, L=3)
    s = workload.scene(1, 3, 4)
    sc = orc.Scene(s.ego, s.obstacles)
    dec = workload.decoder_weights(0)
    p0 = orc.decoder_sample(par, dec, workload.observation(s), s.seed, 64)
    res = orc.plan(par, sc, s.seed, 64, trace=True, p0=p0)
    assert np.array_equal(res.trace["p"][0], p0)
    assert np.all(np.isfinite(res.xi_best)) and res.best_index == res.trace["es"][-1][0]

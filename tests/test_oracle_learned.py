"""Pins for the learned-proposal oracle (CPU): BF16 rounding against an
independent implementation, descriptor and height-map closed forms,
rigid-motion invariance, finite-difference gradients, AdamW closed form,
top-k tie rule, and bin bookkeeping of proposal poses."""
import math

import numpy as np
import pytest
import torch

from oracle import bruteforce as bf
from oracle import learned as ol
from paper_2512_16896_amd import scenegen as sg


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 65504.0]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ol.bf16(x), want)
    assert ol.bf16(1.0 + 2 ** -8) == 1.0              # tie -> even
    assert ol.bf16(1.0 + 3 * 2 ** -9) == 1.0 + 2 ** -7


def test_descriptor_single_sphere_closed_form():
    a, b, c, r = 0.01, -0.02, 0.03, 0.04
    d = ol.descriptor(np.array([[a, b, c, r]]))
    assert d[0] == 1 / 256
    np.testing.assert_allclose(d[1:5], [10 * r, 10 * r, 10 * r, 0.0], atol=1e-15)
    assert d[5] == pytest.approx(1e3 * r ** 3)
    np.testing.assert_allclose(d[6:9], [10 * a, 10 * b, 10 * c], atol=1e-15)
    np.testing.assert_allclose(d[9:15], 0.0, atol=1e-15)
    np.testing.assert_allclose(d[15:18], 10 * r, atol=1e-15)
    assert d[18] == pytest.approx(10 * (r - c))
    assert d[19] == pytest.approx(20 * r)                  # rests on the plane: top = 2r
    assert d[20] == pytest.approx(10 * (math.hypot(a, b) + r))
    assert np.all(d[21:] == 0)


def test_descriptor_two_spheres():
    t = np.array([[-0.1, 0.0, 0.0, 0.02], [0.1, 0.0, 0.0, 0.02]])
    d = ol.descriptor(t)
    np.testing.assert_allclose(d[6:9], 0.0, atol=1e-15)           # symmetric centroid
    assert d[9] == pytest.approx(100 * 0.01)                      # var x = 0.1^2
    np.testing.assert_allclose(d[10:15], 0.0, atol=1e-15)
    assert d[15] == pytest.approx(10 * 0.12)                      # half extent x


def _one_scene(boxes=(), sup_R=np.eye(3), sup_t=(0.0, 0.0, 0.0), hx=0.64, hy=0.32):
    tm = np.array([[0.0, 0.0, 0.0, 0.05]] * 2, np.float32)
    sup = np.zeros((1, 16), np.float32)
    sup[0, :9] = np.asarray(sup_R).reshape(9)
    sup[0, 9:12] = sup_t
    sup[0, 12], sup[0, 13] = hx, hy
    bx = np.zeros((len(boxes), 16), np.float32)
    for i, (R, c, h) in enumerate(boxes):
        bx[i, :9], bx[i, 9:12], bx[i, 12:15] = np.asarray(R).reshape(9), c, h
    return sg.SceneBatch(obj_off=np.array([0, 2], np.int32), sph_off=np.array([0, 1, 2], np.int32),
                         tmpl=tm, obj_sup=np.zeros(2, np.int32), obj_ncand=np.full(2, 8, np.int32),
                         sup=sup, box_off=np.array([0, len(boxes)], np.int32), box=bx)


def test_heightmap_box_and_sphere_closed_forms():
    # upright box resting on the support: height 2 h_z over its footprint
    b = _one_scene(boxes=[(np.eye(3), (0.1, 0.05, 0.08), (0.2, 0.1, 0.08))])
    H = ol.heightmap(b, np.zeros((2, 4)), 0, 0)
    hx, hy = 0.64, 0.32
    cx = -hx + (np.arange(64) + 0.5) * (2 * hx / 64)
    cy = -hy + (np.arange(64) + 0.5) * (2 * hy / 64)
    X, Y = np.meshgrid(cx, cy, indexing="ij")
    inside = (np.abs(X - 0.1) <= 0.2) & (np.abs(Y - 0.05) <= 0.1)
    np.testing.assert_allclose(H[inside], float(np.float32(0.08)) * 2, atol=1e-7)
    assert np.all(H[~inside] == 0)
    # one placed sphere: z + sqrt(r^2 - d^2) above the cells it covers
    placed = np.array([[0.0, 0.0, 0.05, 0.05], [0.3, -0.1, 0.03, 0.03]])
    b2 = _one_scene()
    H2 = ol.heightmap(b2, placed, 0, 1)
    d2 = X ** 2 + Y ** 2
    want = np.where(d2 < 0.05 ** 2, 0.05 + np.sqrt(np.maximum(0.05 ** 2 - d2, 0)), 0.0)
    np.testing.assert_allclose(H2, want, atol=1e-12)
    # only the first n_state objects count
    assert np.all(ol.heightmap(b2, placed, 0, 0) == 0)


def test_heightmap_rigid_motion_invariance():
    rng = np.random.default_rng(3)
    Rz = lambda a: np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    boxes_l = [(Rz(0.4), np.array([0.1, 0.05, 0.08]), (0.15, 0.1, 0.08)),
               (Rz(-1.1), np.array([-0.3, -0.1, 0.12]), (0.05, 0.2, 0.12))]
    placed_l = np.array([[0.2, 0.1, 0.04, 0.04], [-0.1, 0.05, 0.2, 0.03]])
    H0 = ol.heightmap(_one_scene(boxes=boxes_l), np.concatenate([placed_l]), 0, 2)
    for _ in range(3):
        R, t = Rz(rng.uniform(0, 6)), rng.uniform(-1, 1, 3)
        boxes_w = [(R @ Rb, R @ c + t, h) for Rb, c, h in boxes_l]
        placed_w = np.concatenate([placed_l[:, :3] @ R.T + t, placed_l[:, 3:]], 1)
        b = _one_scene(boxes=boxes_w, sup_R=R, sup_t=t)
        H1 = ol.heightmap(b, placed_w, 0, 2)
        # box rows and support rows are FP32 in the batch: compare loosely, and
        # only away from footprint edges (a cell centre on an edge may flip)
        assert np.mean(np.abs(H1 - H0) > 1e-5) < 0.01


def _tiny_net(rng, dims=(32, 16, 16, 16, 24)):
    W = [rng.standard_normal((dims[l + 1], dims[l])) / math.sqrt(dims[l]) for l in range(4)]
    b = [rng.standard_normal(dims[l + 1]) * 0.1 for l in range(4)]
    return W, b


def test_forward_single_layer_is_a_matmul():
    rng = np.random.default_rng(4)
    W, b = _tiny_net(rng)
    x = rng.standard_normal((5, 32))
    z, ins = ol.forward(x, W, b, round_bf16=False)
    h = x
    for l in range(3):
        h = np.maximum(h @ W[l].T + b[l], 0)
    np.testing.assert_allclose(z, h @ W[3].T + b[3], rtol=1e-13)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(5)
    W, b = _tiny_net(rng)
    x = rng.standard_normal((4, 32))
    bins = rng.integers(0, 24, size=(4, 3))
    bins[0, 2] = -1
    tgt = rng.integers(0, 2, size=(4, 3)).astype(np.float64)
    loss, gW, gb = ol.backward(x, W, b, bins, tgt, round_bf16=False)
    f = lambda W_, b_: ol.bce_loss(ol.forward(x, W_, b_, round_bf16=False)[0], bins, tgt)[0]
    eps = 1e-6
    for l in range(4):
        for (i, j) in [(0, 0), (3, 5), (W[l].shape[0] - 1, W[l].shape[1] - 1)]:
            Wp = [w.copy() for w in W]; Wp[l][i, j] += eps
            Wm = [w.copy() for w in W]; Wm[l][i, j] -= eps
            fd = (f(Wp, b) - f(Wm, b)) / (2 * eps)
            assert gW[l][i, j] == pytest.approx(fd, rel=1e-6, abs=1e-9)
        bp = [v.copy() for v in b]; bp[l][1] += eps
        bm = [v.copy() for v in b]; bm[l][1] -= eps
        assert gb[l][1] == pytest.approx((f(W, bp) - f(W, bm)) / (2 * eps), rel=1e-6, abs=1e-9)
    assert loss == pytest.approx(f(W, b))


def test_adamw_first_step_closed_form():
    w = np.array([0.5, -0.2, 0.0])
    g = np.array([0.3, -0.01, 0.0])
    nw, m, v = ol.adamw_step(w, g, np.zeros(3), np.zeros(3), 0, 1e-3, 0.9, 0.999, 1e-8, 1e-4)
    # bias-corrected moments equal g and g^2 on the first step
    want = w - 1e-3 * (g / (np.abs(g) + 1e-8) + 1e-4 * w)
    np.testing.assert_allclose(nw, want, rtol=1e-12)


def test_topk_tie_rule():
    z = np.array([0.5, 2.0, 2.0, -1.0, 2.0, 0.5])
    assert ol.topk(z, 6).tolist() == [1, 2, 4, 0, 5, 3]


def test_proposal_pose_stays_in_its_bin():
    rng = np.random.default_rng(6)
    for _ in range(200):
        bin_ = int(rng.integers(0, 4096))
        x, y, z, yaw = ol.proposal_pose(int(rng.integers(0, 2 ** 63)), 3, 2, int(rng.integers(0, 64)),
                                        bin_, 1.0, 0.5, 0.1)
        u0, u1, u2 = (x / 1.0 + 1) / 2, (y / 0.5 + 1) / 2, yaw / (2 * math.pi)
        assert ol.bin_of(u0, u1, u2) == bin_
        assert z == 0.1


def test_label_bins_come_from_the_uniforms():
    # bin of a uniform candidate = (floor(32 u0) * 16 + floor(16 u1)) * 8 + floor(8 u2)
    w = bf.philox(np.array([[5, 0x20000, 1, 7]]), (1, 2))
    u = bf.unit(w)[0]
    assert ol.bin_of(u[0], u[1], u[2]) == (int(32 * u[0]) * 16 + int(16 * u[1])) * 8 + int(8 * u[2])

"""CPU pins of the forward-kinematics oracle (oracle/fk.c): closed forms of
prismatic and revolute joints, an independent rotation-vector construction,
chains against 4 x 4 homogeneous products, rigid motion of the base, and the
sampled joint values against the Philox generator pinned by its published
known answers."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle


def _T(R=None, t=(0, 0, 0)):
    R = np.eye(3) if R is None else np.asarray(R, float)
    return np.concatenate([R.ravel(), np.asarray(t, float)])


def _joint(kind, parent, lo, hi, axis, Tj):
    row = np.zeros(24)
    row[0], row[1], row[2], row[3] = kind, parent, lo, hi
    row[4:7] = axis
    row[8:20] = Tj
    return row


def _h(T):
    H = np.eye(4)
    H[:3, :3] = T[:9].reshape(3, 3)
    H[:3, 3] = T[9:12]
    return H


def test_prismatic_moves_by_q_along_the_axis():
    base = _T(t=(1.0, -2.0, 0.5))
    J = _joint(0, -1, 0.0, 0.4, (1, 0, 0), _T(t=(0.25, 0.0, 0.0)))
    q, link, (rows,) = oracle.forward_kinematics(
        [0, 1], [J], [base], q=[0.3],
        rows=[(np.zeros((1, 16)), [0], [_T(t=(0.0, 0.1, 0.2))])])
    assert np.array_equal(link[0][:9], np.eye(3).ravel())
    np.testing.assert_allclose(link[0][9:], [1.0 + 0.25 + 0.3, -2.0, 0.5], rtol=0, atol=1e-15)
    np.testing.assert_allclose(rows[0][9:12], [1.55, -1.9, 0.7], rtol=0, atol=1e-15)


def test_revolute_quarter_turn_about_z_is_the_exact_rational_rotation():
    J = _joint(1, -1, -np.pi, np.pi, (0, 0, 1), _T())
    q, link, (rows,) = oracle.forward_kinematics(
        [0, 1], [J], [_T()], q=[np.pi / 2],
        rows=[(np.zeros((1, 16)), [0], [_T(t=(1.0, 0.0, 0.3))])])
    np.testing.assert_allclose(link[0][:9].reshape(3, 3), [[0, -1, 0], [1, 0, 0], [0, 0, 1]],
                               rtol=0, atol=1e-15)
    np.testing.assert_allclose(rows[0][9:12], [0.0, 1.0, 0.3], rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_revolute_matches_rotation_vector(seed):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    q = rng.uniform(-3, 3)
    J = _joint(1, -1, -4, 4, a, _T())
    _, link, _ = oracle.forward_kinematics([0, 1], [J], [_T()], q=[q])
    want = Rotation.from_rotvec(q * a).as_matrix()
    np.testing.assert_allclose(link[0][:9].reshape(3, 3), want, rtol=0, atol=1e-14)
    # a point on the axis does not move; the radial distance is kept
    p = rng.normal(size=3)
    Rq = link[0][:9].reshape(3, 3)
    assert abs(np.linalg.norm(Rq @ p - np.dot(p, a) * a) - np.linalg.norm(p - np.dot(p, a) * a)) < 1e-14
    np.testing.assert_allclose(Rq @ a, a, rtol=0, atol=1e-14)


def test_chain_equals_homogeneous_product():
    rng = np.random.default_rng(4)
    base = _T(Rotation.random(random_state=1).as_matrix(), rng.normal(size=3))
    Ts = [_T(Rotation.random(random_state=10 + i).as_matrix(), rng.normal(size=3)) for i in range(3)]
    axes = [rng.normal(size=3) for _ in range(3)]
    axes = [a / np.linalg.norm(a) for a in axes]
    kinds, qs = [0, 1, 1], [0.2, 0.7, -1.1]
    joints = [_joint(kinds[i], i - 1, -2, 2, axes[i], Ts[i]) for i in range(3)]
    _, link, _ = oracle.forward_kinematics([0, 3], joints, [base], q=qs)
    H = _h(base)
    for i in range(3):
        M = np.eye(4)
        if kinds[i] == 0:
            M[:3, 3] = qs[i] * axes[i]
        else:
            M[:3, :3] = Rotation.from_rotvec(qs[i] * axes[i]).as_matrix()
        H = H @ _h(Ts[i]) @ M
        np.testing.assert_allclose(_h(link[i]), H, rtol=0, atol=1e-12)


def test_rigid_motion_of_the_base_moves_every_link():
    rng = np.random.default_rng(6)
    joints = [_joint(0, -1, 0, 0.3, (1, 0, 0), _T(t=(0.2, 0, 0))),
              _joint(1, 0, -1, 1, (0, 0, 1), _T(t=(0, 0.1, 0)))]
    base = _T(Rotation.random(random_state=3).as_matrix(), rng.normal(size=3))
    G = _T(Rotation.random(random_state=4).as_matrix(), rng.normal(size=3))
    q = [0.17, 0.4]
    _, l1, _ = oracle.forward_kinematics([0, 2], joints, [base], q=q)
    moved = (_h(G) @ _h(base))
    base2 = np.concatenate([moved[:3, :3].ravel(), moved[:3, 3]])
    _, l2, _ = oracle.forward_kinematics([0, 2], joints, [base2], q=q)
    for i in range(2):
        np.testing.assert_allclose(_h(l2[i]), _h(G) @ _h(l1[i]), rtol=0, atol=1e-13)


def test_sampled_values_follow_the_counter_based_generator():
    joints = [_joint(0, -1, 0.05, 0.35, (1, 0, 0), _T()), _joint(1, -1, -1.0, 2.0, (0, 0, 1), _T()),
              _joint(0, -1, 0.0, 0.0, (0, 1, 0), _T())]
    joint_off = [0, 2, 3]
    seed = 0x1234_5678_9ABC
    q, _, _ = oracle.forward_kinematics(joint_off, joints, [_T(), _T()], seed=seed,
                                        scene_id=[7, 9])
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for i, (s, local) in enumerate([(7, 0), (7, 1), (9, 0)]):
        w = oracle.philox4x32_10([local, 0x30000, 0, s], key)
        u = oracle.u01(int(w[0]))
        lo, hi = joints[i][2], joints[i][3]
        assert q[i] == lo + u * (hi - lo)
        assert lo <= q[i] <= hi
    # rows not linked to a joint are left as they are
    rows = np.arange(32, dtype=float).reshape(2, 16)
    _, _, (moved,) = oracle.forward_kinematics(joint_off, joints, [_T(), _T()], q=[0.1, 0.2, 0.0],
                                               rows=[(rows, [-1, 2], np.zeros((2, 12)))])
    assert np.array_equal(moved[0], rows[0])
    assert np.array_equal(moved[1][12:], rows[1][12:])

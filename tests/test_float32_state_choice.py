"""Why the scan state is a 3x4 affine: a float32 emulation (numpy) of one
1000-residue chain built transform by transform, with the lane aggregate of
each residue composed into a running prefix, in two representations:

* 3x4 affine, one polar step R <- R (3I - R^T R) / 2 per residue aggregate
  (what the kernels do);
* unit quaternion + translation (7 floats), the residue aggregate converted
  by Shepperd's method and normalised.

Against the FP64 oracle the affine chain stays within the 1e-3 A bound at
L = 1000, while the quaternion chain drifts by about 5e-2 A: the rotation a
float32 quaternion represents carries a larger rounding error, and a run of
similar residues repeats it coherently.  A quaternion state would save about
a tenth of the scan's instructions; the accuracy bound rules it out."""
import numpy as np

import oracle
from workloads import BACKBONE_GEOMETRY as G, make_angles

f32 = np.float32


def _transforms(ang):
    pi = np.pi
    bond = [G["bond_C_N"], G["bond_N_CA"], G["bond_CA_C"]]
    angle = [G["angle_CA_C_N"], G["angle_C_N_CA"], G["angle_N_CA_C"]]
    plane = [2, 0, 1]
    out = []
    for j in range(ang.shape[1]):
        res = []
        for s in range(3):
            th, a, d = pi - angle[s] * pi / 180, float(ang[plane[s], j]), bond[s]
            ry = np.array([[np.cos(th), 0, np.sin(th)], [0, 1, 0], [-np.sin(th), 0, np.cos(th)]])
            rx = np.array([[1, 0, 0], [0, np.cos(a), -np.sin(a)], [0, np.sin(a), np.cos(a)]])
            m = np.eye(4)
            m[:3, :3] = ry @ rx
            m[:3, 3] = ry @ np.array([d, 0, 0])
            res.append(m.astype(f32))
        out.append(res)
    return out


def _residue_aggregates(ts):
    for res in ts:
        m = np.eye(4, dtype=f32)
        local = []
        for t in res:
            m = (m @ t).astype(f32)
            local.append(m[:3, 3].copy())
        yield m, local


def _affine_chain(ts):
    prefix = np.eye(4, dtype=f32)
    pos = []
    for m, local in _residue_aggregates(ts):
        pos += [(prefix[:3, :3] @ p + prefix[:3, 3]).astype(f32) for p in local]
        r = m[:3, :3]
        m[:3, :3] = (r + r @ ((np.eye(3, dtype=f32) - r.T @ r) / 2)).astype(f32)
        prefix = (prefix @ m).astype(f32)
    return np.array(pos).T


def _qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2],
                    dtype=f32)


def _qrot(q, v):
    u = q[1:]
    t = (f32(2) * np.cross(u, v)).astype(f32)
    return (v + q[0] * t + np.cross(u, t)).astype(f32)


def _to_quat(m):
    r = m[:3, :3]
    d = [1 + r[0, 0] + r[1, 1] + r[2, 2], 1 + r[0, 0] - r[1, 1] - r[2, 2],
         1 - r[0, 0] + r[1, 1] - r[2, 2], 1 - r[0, 0] - r[1, 1] + r[2, 2]]
    k = int(np.argmax(d))
    s = f32(2) * np.sqrt(f32(d[k]))
    h, inv = f32(0.25) * s, f32(1) / s
    a, b, c = r[2, 1] - r[1, 2], r[0, 2] - r[2, 0], r[1, 0] - r[0, 1]
    p, q, rr = r[0, 1] + r[1, 0], r[0, 2] + r[2, 0], r[1, 2] + r[2, 1]
    rows = [[h, a * inv, b * inv, c * inv], [a * inv, h, p * inv, q * inv],
            [b * inv, p * inv, h, rr * inv], [c * inv, q * inv, rr * inv, h]]
    qv = np.array(rows[k], dtype=f32)
    return (qv / np.sqrt(np.sum(qv * qv, dtype=f32))).astype(f32)


def _quaternion_chain(ts):
    pq, pt = np.array([1, 0, 0, 0], dtype=f32), np.zeros(3, dtype=f32)
    pos = []
    for m, local in _residue_aggregates(ts):
        pos += [(_qrot(pq, p) + pt).astype(f32) for p in local]
        pt = (pt + _qrot(pq, m[:3, 3])).astype(f32)
        pq = _qmul(pq, _to_quat(m))
    return np.array(pos).T


def test_affine_state_meets_the_bound_and_quaternion_state_does_not():
    rng = np.random.Generator(np.random.PCG64(5))
    L = 1000
    ang = make_angles(rng, L, "mixture", 3)
    ref = oracle.backbone_forward(np.array([0, L]), ang, G)
    ts = _transforms(ang)
    e_aff = float(np.max(np.abs(_affine_chain(ts) - ref)))
    e_quat = float(np.max(np.abs(_quaternion_chain(ts) - ref)))
    print(f"float32 chain, L = 1000: 3x4 + polar {e_aff:.2e} A, quaternion {e_quat:.2e} A")
    assert e_aff < 1e-3
    assert e_quat > 10 * e_aff

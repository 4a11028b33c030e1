"""Oracle of the discrete adjoint: the explicit step of the C oracle written
again with plain PyTorch CPU float64 operations, differentiated by torch's
autograd. Test infrastructure, like the rest of `oracle/`: only the tests may
use it.

The adjoint is that of the gauge misfit of an inverse analysis (sec. 1: the
solver serves calibration and inverse problems): with the time-step schedule
dt_0 .. dt_{N-1} frozen (taken from a forward run and held fixed),

    L(m, z) = sum over gauge cells g of (h_g(t_N) - h_target_g)^2,

and its gradients with respect to the per-cell Manning coefficient m and bed
elevation z. The step follows the C oracle's functions operation for
operation (sec. 3.1 geometry from the C oracle's own mesh arrays; HLLC of
sec. 3.2, eqs. 17-26; reconstruction and bed-slope terms, eqs. 28-30; the
semi-implicit friction update, eqs. 31-37; positivity and the wet/dry
threshold as read in the C oracle). The derivative is that of the branches
taken at the evaluation point: comparisons (wet/dry, wave-speed cases, the
star region, the reconstruction's max and the positivity fix) select a
branch and carry no derivative. Branches not taken are evaluated on
harmless stand-in operands so that their zero weights never meet an
infinite or undefined derivative.
"""
import math

import numpy as np
import torch

from . import Oracle

K_WALL, K_TRANSMISSIVE, K_INFLOW, K_FIXED_DEPTH, K_FIXED_STAGE = range(5)


def _w(mask, a, b):
    return torch.where(mask, a, b)


def hllc(g, h_dry, hL, uL, vL, hR, uR, vR):
    """HLLC flux (G0, G1, G2) of eqs. 17-26 for tensors of edges."""
    one = torch.ones_like(hL)
    wetL, wetR = hL > h_dry, hR > h_dry
    hL, uL, vL = _w(wetL, hL, 0 * hL), _w(wetL, uL, 0 * uL), _w(wetL, vL, 0 * vL)
    hR, uR, vR = _w(wetR, hR, 0 * hR), _w(wetR, uR, 0 * uR), _w(wetR, vR, 0 * vR)
    any_wet = wetL | wetR
    both = wetL & wetR
    aL = _w(wetL, torch.sqrt(g * _w(wetL, hL, one)), 0 * hL)
    aR = _w(wetR, torch.sqrt(g * _w(wetR, hR, one)), 0 * hR)
    # both wet: star depth (eqs. 21-23) on stand-ins elsewhere
    hLb, hRb = _w(both, hL, one), _w(both, hR, one)
    aLb, aRb = _w(both, aL, one), _w(both, aR, one)
    h0 = 0.5 * (hLb + hRb) - (uR - uL) * (hLb + hRb) / (4.0 * (aLb + aRb))
    trrs = h0 <= torch.minimum(hLb, hRb)
    b = 0.5 * (aLb + aRb) + 0.25 * (uL - uR)
    b = _w(b < 0.0, 0 * b, b)
    hs_r = b * b / g
    ts = both & ~trrs
    h0t = _w(ts, h0, one)
    gL = torch.sqrt(g * (h0t + hLb) / (2.0 * h0t * hLb))
    gR = torch.sqrt(g * (h0t + hRb) / (2.0 * h0t * hRb))
    hs_t = (hLb * gL + hRb * gR + uL - uR) / (gL + gR)
    hs = _w(trrs, hs_r, hs_t)
    shL, shR = both & (hs > hLb), both & (hs > hRb)
    wL = _w(shL, hs * (hs + hLb) / 2.0, one)
    wR = _w(shR, hs * (hs + hRb) / 2.0, one)
    pL = _w(shL, torch.sqrt(wL) / hLb, one)
    pR = _w(shR, torch.sqrt(wR) / hRb, one)
    SL_b, SR_b = uL - aL * pL, uR + aR * pR
    # dry sides (eq. 26)
    SL = _w(both, SL_b, _w(wetL, uL - aL, uR - 2.0 * aR))
    SR = _w(both, SR_b, _w(wetL, uL + 2.0 * aL, uR + aR))
    with torch.no_grad():        # the contact speed only selects a branch
        den = hR * (uR - SR) - hL * (uL - SL)
        den = torch.where(den == 0, torch.ones_like(den), den)
        Ss_b = (SL * hR * (uR - SR) - SR * hL * (uL - SL)) / den
        Ss = torch.where(both, Ss_b, torch.where(wetL, SR, SL))
    FL0, FL1, FL2 = hL * uL, hL * uL * uL + 0.5 * g * hL * hL, hL * uL * vL
    FR0, FR1, FR2 = hR * uR, hR * uR * uR + 0.5 * g * hR * hR, hR * uR * vR
    star = any_wet & (SL < 0.0) & (SR > 0.0)
    D = _w(star, SR - SL, one)
    rD = 1.0 / D          # one reciprocal, as in the C oracle
    S0 = (SR * FL0 - SL * FR0 + SR * SL * (hR - hL)) * rD
    S1 = (SR * FL1 - SL * FR1 + SR * SL * (hR * uR - hL * uL)) * rD
    S2 = S0 * _w(Ss >= 0.0, vL, vR)
    left = SL >= 0.0
    G0 = _w(left, FL0, _w(SR <= 0.0, FR0, S0))
    G1 = _w(left, FL1, _w(SR <= 0.0, FR1, S1))
    G2 = _w(left, FL2, _w(SR <= 0.0, FR2, S2))
    zero = 0 * hL
    return _w(any_wet, G0, zero), _w(any_wet, G1, zero), _w(any_wet, G2, zero)


class TorchScheme:
    """The step of the C oracle on the C oracle's mesh, in torch float64."""

    def __init__(self, case, threads=1):
        o = Oracle(case, threads=threads)
        e = o.edges()
        area, _, _ = o.geometry()
        self.g, self.h_dry = float(case.g), float(case.h_dry)
        t = lambda a: torch.as_tensor(np.asarray(a))
        self.left = t(e["left"]).long()
        self.right = t(e["right"]).long()
        self.nx, self.ny, self.len = t(e["nx"]), t(e["ny"]), t(e["len"])
        inner = self.right >= 0
        self.ii = torch.nonzero(inner).flatten()
        self.bi = torch.nonzero(~inner).flatten()
        self.area = t(area)
        self.c_edge = t(e["c_edge"]).long()
        self.c_right = t(e["c_right"]).bool()
        tag = np.asarray(e["tag"])
        bnd = np.asarray(e["right"]) < 0
        lsum = {}
        for k in np.unique(tag[bnd]):
            lsum[int(k)] = math.fsum(np.asarray(e["len"])[bnd & (tag == k)])
        kind = np.zeros(tag.size, np.int64)
        value = np.zeros(tag.size)
        q = np.zeros(tag.size)
        for k, (kd, val) in case.bc.items():
            sel = bnd & (tag == k)
            kind[sel] = kd
            value[sel] = val
            if kd == K_INFLOW and lsum.get(int(k), 0.0) > 0.0:
                q[sel] = val / lsum[int(k)]
        bi = self.bi.numpy()
        self.bkind = torch.as_tensor(kind[bi])
        self.bvalue = torch.as_tensor(value[bi])
        self.bq = torch.as_tensor(q[bi])
        self.n_edges = tag.size

    def _velocity(self, h, hu, hv):
        wet = h > self.h_dry
        hs = _w(wet, h, torch.ones_like(h))
        r = 1.0 / hs
        return _w(wet, hu * r, 0 * hu), _w(wet, hv * r, 0 * hv)

    def step(self, h, hu, hv, z, m, dt):
        g, h_dry = self.g, self.h_dry
        u, v = self._velocity(h, hu, hv)
        cl = [torch.zeros(self.n_edges, dtype=h.dtype) for _ in range(3)]
        cr = [torch.zeros(self.n_edges, dtype=h.dtype) for _ in range(3)]
        # interior edges (eqs. 12, 28-30)
        ii = self.ii
        i, j = self.left[ii], self.right[ii]
        nx, ny, L = self.nx[ii], self.ny[ii], self.len[ii]
        zi, zj = z[i], z[j]
        zs = _w(zi > zj, zi, zj)
        hLs = h[i] - (zs - zi)
        hRs = h[j] - (zs - zj)
        hLs = _w(hLs <= h_dry, 0 * hLs, hLs)
        hRs = _w(hRs <= h_dry, 0 * hRs, hRs)
        ui, vi, uj, vj = u[i], v[i], u[j], v[j]
        G0, G1, G2 = hllc(g, h_dry, hLs, ui * nx + vi * ny, -ui * ny + vi * nx,
                          hRs, uj * nx + vj * ny, -uj * ny + vj * nx)
        F1 = G1 * nx - G2 * ny
        F2 = G1 * ny + G2 * nx
        pL = 0.5 * g * (hLs * hLs - h[i] * h[i])
        pR = 0.5 * g * (hRs * hRs - h[j] * h[j])
        vals_l = [L * (-G0), L * (pL * nx - F1), L * (pL * ny - F2)]
        vals_r = [L * G0, L * (F1 - pR * nx), L * (F2 - pR * ny)]
        for k in range(3):
            cl[k] = cl[k].index_put((ii,), vals_l[k])
            cr[k] = cr[k].index_put((ii,), vals_r[k])
        # boundary edges (sec. 3.1 and the fixed-level conditions)
        bi = self.bi
        if bi.numel():
            i = self.left[bi]
            nx, ny, L = self.nx[bi], self.ny[bi], self.len[bi]
            hi, ui, vi, zi = h[i], u[i], v[i], z[i]
            un, ut = ui * nx + vi * ny, -ui * ny + vi * nx
            kind, val, q = self.bkind, self.bvalue, self.bq
            # transmissive: the physical flux of the cell
            T0 = hi * un
            T1 = hi * un * un + 0.5 * g * hi * hi
            T2 = hi * un * ut
            # inflow
            wet = hi > h_dry
            hs_ = _w(wet, hi, torch.ones_like(hi))
            I1 = _w(wet, q * q / hs_, 0 * hi) + 0.5 * g * hi * hi
            # fixed depth / fixed stage: HLLC against a ghost
            hb = _w(kind == K_FIXED_STAGE, val - zi, val)
            hb = _w(hb < 0.0, 0 * hb, hb)
            H0, H1, H2 = hllc(g, h_dry, hi, un, ut, hb, un, ut)
            W1 = 0.5 * g * hi * hi
            ghost = (kind == K_FIXED_DEPTH) | (kind == K_FIXED_STAGE)
            G0 = _w(kind == K_TRANSMISSIVE, T0,
                    _w(kind == K_INFLOW, -q, _w(ghost, H0, 0 * hi)))
            G1 = _w(kind == K_TRANSMISSIVE, T1,
                    _w(kind == K_INFLOW, I1, _w(ghost, H1, W1)))
            G2 = _w(kind == K_TRANSMISSIVE, T2,
                    _w(kind == K_INFLOW, 0 * hi, _w(ghost, H2, 0 * hi)))
            F1 = G1 * nx - G2 * ny
            F2 = G1 * ny + G2 * nx
            for k, val_k in enumerate((L * (-G0), L * (-F1), L * (-F2))):
                cl[k] = cl[k].index_put((bi,), val_k)
        # cell update (eqs. 31-37) with the positivity fix
        R = []
        for k in range(3):
            acc = torch.zeros_like(h)
            for s in range(3):
                e = self.c_edge[:, s]
                acc = acc + _w(self.c_right[:, s], cr[k][e], cl[k][e])
            R.append(acc)
        A = self.area
        rA = 1.0 / A
        bh, bx, by = R[0] * rA, R[1] * rA, R[2] * rA
        dh = dt * bh
        with torch.no_grad():
            qn_raw = torch.sqrt(hu * hu + hv * hv)
        fric = (h > h_dry) & (qn_raw > 0.0)
        one = torch.ones_like(h)
        hf = _w(fric, h, one)
        qn = torch.sqrt(_w(fric, hu * hu + hv * hv, one))
        c = g * m * m / (hf * hf * torch.pow(hf, 1.0 / 3.0))
        sfx, sfy = -c * qn * hu, -c * qn * hv
        rh, rq = 1.0 / hf, 1.0 / qn
        jhx = (7.0 / 3.0) * c * qn * hu * rh
        jhy = (7.0 / 3.0) * c * qn * hv * rh
        jxx = -c * (qn + hu * hu * rq)
        jxy = -c * hu * hv * rq
        jyy = -c * (qn + hv * hv * rq)
        m11 = 1.0 - 0.5 * dt * jxx
        m12 = -0.5 * dt * jxy
        m22 = 1.0 - 0.5 * dt * jyy
        rx = dt * (bx + sfx) + 0.5 * dt * jhx * dh
        ry = dt * (by + sfy) + 0.5 * dt * jhy * dh
        det = m11 * m22 - m12 * m12
        rd = 1.0 / det
        dqx = _w(fric, (rx * m22 - m12 * ry) * rd, dt * bx)
        dqy = _w(fric, (m11 * ry - m12 * rx) * rd, dt * by)
        hn, hun, hvn = h + dh, hu + dqx, hv + dqy
        hn = _w(hn < 0.0, 0 * hn, hn)
        dry = hn <= h_dry
        return hn, _w(dry, 0 * hun, hun), _w(dry, 0 * hvn, hvn)


def gauge_misfit(case, dts, gauges, h_target, manning=None, z=None,
                 grad=True):
    """Loss after len(dts) frozen steps from the case's state and, with
    grad, its gradients with respect to the Manning field and the bed."""
    sch = TorchScheme(case)
    m = torch.tensor(case.manning if manning is None else manning,
                     dtype=torch.float64, requires_grad=grad)
    zz = torch.tensor(case.z if z is None else z, dtype=torch.float64,
                      requires_grad=grad)
    h = torch.tensor(case.h, dtype=torch.float64)
    hu = torch.tensor(case.hu, dtype=torch.float64)
    hv = torch.tensor(case.hv, dtype=torch.float64)
    for dt in dts:
        h, hu, hv = sch.step(h, hu, hv, zz, m, float(dt))
    gi = torch.as_tensor(np.asarray(gauges), dtype=torch.long)
    tgt = torch.as_tensor(np.asarray(h_target), dtype=torch.float64)
    loss = torch.sum((h[gi] - tgt) ** 2)
    if not grad:
        return float(loss), h.detach().numpy()
    loss.backward()
    return float(loss.detach()), m.grad.numpy().copy(), zz.grad.numpy().copy()

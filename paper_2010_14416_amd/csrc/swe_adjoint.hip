// Discrete adjoint of one explicit step with a frozen time step (gfx950).
//
// The step maps U^k to U^{k+1} = F(U^k; z, g m^2, dt_k). Given the adjoint
// lambda^{k+1} = dL/dU^{k+1}, one reverse step produces
//   lambda^k = (dF/dU^k)^T lambda^{k+1},
// and adds (dF/dz)^T lambda^{k+1} and (dF/d(g m^2))^T lambda^{k+1} to the
// bed and friction gradients. The derivative is that of the branches the
// forward step takes at U^k (wet/dry, wave-speed cases, star region,
// reconstruction maximum, positivity fix: they select and do not
// differentiate); idle edges (both sides holding no water) and dry cells
// on the quiet path have the derivatives of their exact-zero
// contributions.
//
// Two launches per reverse step, one workgroup per mesh block as in the
// forward step:
//   adj_cell_kernel: recomputes the block's edge contributions into LDS
//     (the forward's arithmetic, swe_scheme.hpp), then for each cell the
//     reverse of the cell update: the adjoint of the cell's summed
//     contribution R (lr), the direct part of lambda^k, and the friction
//     gradient;
//   adj_edge_kernel: for every edge of the block, the reverse of the edge's
//     contributions, weighted by the lr of its two cells (a neighbour in
//     another block is read from HBM), kept in LDS slots of the block's own
//     cells; each cell then sums its three sides in side order. Edges on a
//     block border are reversed by both blocks, each keeping its own side,
//     so no atomics are needed and the sums are order-fixed.
#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

#include <cmath>

#include "swe_adjoint.hpp"
#include "swe_scheme.hpp"

namespace swe {
namespace {

// Reverse of hllc(): from the adjoints Gb of (G0, G1, G2), the adjoints of
// the six inputs. The contact speed S* only selects v_L or v_R and carries
// no derivative.
__device__ void hllc_rev(double g, double h_dry, double hL, double uL,
                         double vL, double hR, double uR, double vR,
                         double Gb0, double Gb1, double Gb2, double &hLb,
                         double &uLb, double &vLb, double &hRb, double &uRb,
                         double &vRb)
{
    hLb = uLb = vLb = hRb = uRb = vRb = 0.0;
    const bool wetL = hL > h_dry, wetR = hR > h_dry;
    if (!wetL && !wetR) return;
    if (!wetL) { hL = 0.0; uL = 0.0; vL = 0.0; }
    if (!wetR) { hR = 0.0; uR = 0.0; vR = 0.0; }
    // forward, keeping what the reverse needs
    const double aL = sqrt(g * hL), aR = sqrt(g * hR);
    double SL, SR, Ss;
    double hsum = 0.0, c4 = 0.0, h0 = 0.0, hs = 0.0, b = 0.0;
    double yL = 0.0, yR = 0.0, gL = 0.0, gR = 0.0;
    double pL = 1.0, pR = 1.0, wL = 0.0, wR = 0.0, sL = 0.0, sR = 0.0;
    bool trrs = false, shL = false, shR = false;
    if (!wetL) {
        SL = uR - 2.0 * aR;
        SR = uR + aR;
        Ss = SL;
    } else if (!wetR) {
        SL = uL - aL;
        SR = uL + 2.0 * aL;
        Ss = SR;
    } else {
        hsum = hL + hR;
        c4 = 4.0 * (aL + aR);
        h0 = 0.5 * hsum - (uR - uL) * hsum / c4;
        if (h0 <= fmin(hL, hR)) {
            trrs = true;
            b = fmax(0.5 * (aL + aR) + 0.25 * (uL - uR), 0.0);
            hs = b * b / g;
        } else {
            yL = g * (h0 + hL) / (2.0 * h0 * hL);
            yR = g * (h0 + hR) / (2.0 * h0 * hR);
            gL = sqrt(yL);
            gR = sqrt(yR);
            hs = (hL * gL + hR * gR + uL - uR) / (gL + gR);
        }
        shL = hs > hL;
        shR = hs > hR;
        if (shL) {
            wL = hs * (hs + hL) / 2.0;
            sL = sqrt(wL);
            pL = sL / hL;
        }
        if (shR) {
            wR = hs * (hs + hR) / 2.0;
            sR = sqrt(wR);
            pR = sR / hR;
        }
        SL = uL - aL * pL;
        SR = uR + aR * pR;
        Ss = (SL * hR * (uR - SR) - SR * hL * (uL - SL)) /
             (hR * (uR - SR) - hL * (uL - SL));
    }
    const double qL = hL * uL, qR = hR * uR;
    double qLb = 0.0, qRb = 0.0, SLb = 0.0, SRb = 0.0;
    if (SL >= 0.0) {
        // G = (qL, qL uL + g hL^2 / 2, qL vL)
        qLb += Gb0 + Gb1 * uL + Gb2 * vL;
        uLb += Gb1 * qL;
        hLb += Gb1 * g * hL;
        vLb += Gb2 * qL;
    } else if (SR <= 0.0) {
        qRb += Gb0 + Gb1 * uR + Gb2 * vR;
        uRb += Gb1 * qR;
        hRb += Gb1 * g * hR;
        vRb += Gb2 * qR;
    } else {
        const double FL1 = qL * uL + 0.5 * g * hL * hL;
        const double FR1 = qR * uR + 0.5 * g * hR * hR;
        const double D = SR - SL;
        const double rD = 1.0 / D;   // as the forward step
        const double G0 = (SR * qL - SL * qR + SR * SL * (hR - hL)) * rD;
        const double G1 = (SR * FL1 - SL * FR1 + SR * SL * (qR - qL)) * rD;
        // G2 = G0 v*, v* = vL if S* >= 0 else vR
        const bool up = Ss >= 0.0;
        const double G0b = Gb0 + Gb2 * (up ? vL : vR);
        if (up) vLb += Gb2 * G0; else vRb += Gb2 * G0;
        const double N0b = G0b * rD, N1b = Gb1 * rD;
        const double Db = -(G0b * G0 + Gb1 * G1) * rD;
        SRb += Db;
        SLb -= Db;
        SRb += N0b * (qL + SL * (hR - hL));
        SLb += N0b * (-qR + SR * (hR - hL));
        qLb += N0b * SR;
        qRb -= N0b * SL;
        hRb += N0b * SR * SL;
        hLb -= N0b * SR * SL;
        SRb += N1b * (FL1 + SL * (qR - qL));
        SLb += N1b * (-FR1 + SR * (qR - qL));
        const double FL1b = N1b * SR, FR1b = -N1b * SL;
        qRb += N1b * SR * SL;
        qLb -= N1b * SR * SL;
        qLb += FL1b * uL;
        uLb += FL1b * qL;
        hLb += FL1b * g * hL;
        qRb += FR1b * uR;
        uRb += FR1b * qR;
        hRb += FR1b * g * hR;
    }
    hLb += qLb * uL;
    uLb += qLb * hL;
    hRb += qRb * uR;
    uRb += qRb * hR;
    // wave speeds
    double aLb = 0.0, aRb = 0.0;
    if (!wetL) {
        uRb += SLb + SRb;
        aRb += -2.0 * SLb + SRb;
    } else if (!wetR) {
        uLb += SLb + SRb;
        aLb += -SLb + 2.0 * SRb;
    } else {
        uLb += SLb;
        aLb -= SLb * pL;
        const double pLb = -SLb * aL;
        uRb += SRb;
        aRb += SRb * pR;
        const double pRb = SRb * aR;
        double hsb = 0.0;
        if (shL) {   // pL = sqrt(wL) / hL, wL = hs (hs + hL) / 2
            const double rL = 1.0 / hL;
            const double sLb = pLb * rL;
            hLb -= pLb * pL * rL;
            const double wLb = sLb / (2.0 * sL);
            hsb += wLb * (2.0 * hs + hL) / 2.0;
            hLb += wLb * hs / 2.0;
        }
        if (shR) {
            const double rR = 1.0 / hR;
            const double sRb = pRb * rR;
            hRb -= pRb * pR * rR;
            const double wRb = sRb / (2.0 * sR);
            hsb += wRb * (2.0 * hs + hR) / 2.0;
            hRb += wRb * hs / 2.0;
        }
        if (trrs) {  // hs = b^2 / g, b = max(0, (aL + aR)/2 + (uL - uR)/4)
            const double bb = hsb * 2.0 * b / g;
            if (b > 0.0) {
                aLb += 0.5 * bb;
                aRb += 0.5 * bb;
                uLb += 0.25 * bb;
                uRb -= 0.25 * bb;
            }
        } else {     // hs = (hL gL + hR gR + uL - uR) / (gL + gR)
            const double den = gL + gR;
            const double rden = 1.0 / den;
            const double nb = hsb * rden, denb = -hsb * hs * rden;
            hLb += nb * gL;
            hRb += nb * gR;
            uLb += nb;
            uRb -= nb;
            const double gLb = nb * hL + denb, gRb = nb * hR + denb;
            // g_k = sqrt(y_k), y_k = g (h0 + h_k) / (2 h0 h_k)
            const double yLb = gLb / (2.0 * gL), yRb = gRb / (2.0 * gR);
            const double dL = 2.0 * h0 * hL, dR = 2.0 * h0 * hR;
            const double rdL = 1.0 / dL, rdR = 1.0 / dR;
            double h0b = yLb * (g - yL * 2.0 * hL) * rdL +
                         yRb * (g - yR * 2.0 * hR) * rdR;
            hLb += yLb * (g - yL * 2.0 * h0) * rdL;
            hRb += yRb * (g - yR * 2.0 * h0) * rdR;
            // h0 = hsum / 2 - (uR - uL) hsum / c4, c4 = 4 (aL + aR)
            const double du = uR - uL;
            const double rc4 = 1.0 / c4;
            const double hsumb = h0b * (0.5 - du * rc4);
            const double dub = -h0b * hsum * rc4;
            const double c4b = h0b * du * hsum * rc4 * rc4;
            hLb += hsumb;
            hRb += hsumb;
            uRb += dub;
            uLb -= dub;
            aLb += 4.0 * c4b;
            aRb += 4.0 * c4b;
        }
    }
    if (wetL) hLb += aLb * g / (2.0 * aL);
    if (wetR) hRb += aRb * g / (2.0 * aR);
    if (!wetL) { hLb = 0.0; uLb = 0.0; vLb = 0.0; }
    if (!wetR) { hRb = 0.0; uRb = 0.0; vRb = 0.0; }
}

// Adjoint of a side's (h, u, v, z), as (h, hu, hv, z) through u = hu / h.
struct SideAdj {
    double h, hu, hv, z;
};

__device__ __forceinline__ SideAdj to_conservative(double h_dry,
                                                   const CellState &s,
                                                   double hb, double ub,
                                                   double vb, double zb)
{
    SideAdj r;
    r.h = hb;
    r.hu = 0.0;
    r.hv = 0.0;
    r.z = zb;
    if (s.h > h_dry) {
        const double rh = 1.0 / s.h;
        r.hu = ub * rh;
        r.hv = vb * rh;
        r.h -= (ub * s.u + vb * s.v) * rh;
    }
    return r;
}

// Reverse of edge_contrib() for an interior edge: clb, crb are the
// adjoints of the two cells' contributions (their lr).
__device__ void interior_edge_rev(double g, double h_dry, const CellState &L,
                                  const CellState &R, double nx, double ny,
                                  double len, const double clb[3],
                                  const double crb[3], SideAdj &La,
                                  SideAdj &Ra)
{
    const double unl = L.u * nx + L.v * ny, utl = -L.u * ny + L.v * nx;
    const double unr = R.u * nx + R.v * ny, utr = -R.u * ny + R.v * nx;
    const double zs = fmax(L.z, R.z);
    double hl = L.h - (zs - L.z);
    double hr = R.h - (zs - R.z);
    const bool hlp = hl > h_dry, hrp = hr > h_dry;
    if (!hlp) hl = 0.0;
    if (!hrp) hr = 0.0;
    // cl = (-len G0, len (pl nx - F1), len (pl ny - F2))
    // cr = ( len G0, len (F1 - pr nx), len (F2 - pr ny))
    const double G0b = len * (crb[0] - clb[0]);
    const double F1b = len * (crb[1] - clb[1]);
    const double F2b = len * (crb[2] - clb[2]);
    const double plb = len * (clb[1] * nx + clb[2] * ny);
    const double prb = -len * (crb[1] * nx + crb[2] * ny);
    const double G1b = F1b * nx + F2b * ny;
    const double G2b = -F1b * ny + F2b * nx;
    double hlb, unlb, utlb, hrb, unrb, utrb;
    hllc_rev(g, h_dry, hl, unl, utl, hr, unr, utr, G0b, G1b, G2b, hlb, unlb,
             utlb, hrb, unrb, utrb);
    // pl = g/2 (hl^2 - L.h^2), pr likewise
    hlb += plb * g * hl;
    hrb += prb * g * hr;
    double Lhb = -plb * g * L.h, Rhb = -prb * g * R.h;
    double Lzb = 0.0, Rzb = 0.0, zsb = 0.0;
    if (hlp) { Lhb += hlb; zsb -= hlb; Lzb += hlb; }
    if (hrp) { Rhb += hrb; zsb -= hrb; Rzb += hrb; }
    if (L.z > R.z) Lzb += zsb; else Rzb += zsb;
    const double Lub = unlb * nx - utlb * ny, Lvb = unlb * ny + utlb * nx;
    const double Rub = unrb * nx - utrb * ny, Rvb = unrb * ny + utrb * nx;
    La = to_conservative(h_dry, L, Lhb, Lub, Lvb, Lzb);
    Ra = to_conservative(h_dry, R, Rhb, Rub, Rvb, Rzb);
}

// Reverse of edge_contrib() for a boundary edge of cell L.
__device__ void boundary_edge_rev(double g, double h_dry, const BcEntry &bc,
                                  const CellState &L, double nx, double ny,
                                  double len, const double clb[3],
                                  SideAdj &La)
{
    const double unl = L.u * nx + L.v * ny, utl = -L.u * ny + L.v * nx;
    // cl = -len F, F = (G0, G1 nx - G2 ny, G1 ny + G2 nx)
    const double G0b = -len * clb[0];
    const double F1b = -len * clb[1], F2b = -len * clb[2];
    const double G1b = F1b * nx + F2b * ny;
    const double G2b = -F1b * ny + F2b * nx;
    double hb = 0.0, unb = 0.0, utb = 0.0, zb = 0.0;
    switch (bc.kind) {
    case 1: {  // transmissive: G0 = h un, G1 = G0 un + g h^2/2, G2 = G0 ut
        const double G0 = L.h * unl;
        const double G0t = G0b + G1b * unl + G2b * utl;
        unb += G1b * G0 + G0t * L.h;
        utb += G2b * G0;
        hb += G0t * unl + G1b * g * L.h;
        break;
    }
    case 2:    // inflow: G1 = q^2 / h (wet) + g h^2 / 2
        if (L.h > h_dry) hb += G1b * (-(bc.q * bc.q) / (L.h * L.h));
        hb += G1b * g * L.h;
        break;
    case 3:
    case 4: {  // ghost of fixed depth / fixed stage through HLLC
        double hr = bc.value;
        bool hrp = true;
        if (bc.kind == 4) {
            hr = bc.value - L.z;
            hrp = hr > 0.0;
            if (!hrp) hr = 0.0;
        }
        double hLb, uLb, vLb, hRb, uRb, vRb;
        hllc_rev(g, h_dry, L.h, unl, utl, hr, unl, utl, G0b, G1b, G2b, hLb,
                 uLb, vLb, hRb, uRb, vRb);
        hb += hLb;
        unb += uLb + uRb;
        utb += vLb + vRb;
        if (bc.kind == 4 && hrp) zb -= hRb;
        break;
    }
    default:   // wall: G1 = g h^2 / 2
        hb += G1b * g * L.h;
        break;
    }
    La = to_conservative(h_dry, L, hb, unb * nx - utb * ny,
                         unb * ny + utb * nx, zb);
}

// Reverse of cell_update() (without the positivity ledger, which the
// state does not depend on).
__device__ void cell_update_rev(double h_dry, double dt, double A,
                                double gm2, double h, double hu, double hv,
                                double R0, double R1, double R2, double hnb,
                                double hunb, double hvnb, double &hb,
                                double &hub, double &hvb, double &R0b,
                                double &R1b, double &R2b, double &gm2b)
{
    // the forward values as the step computes them (one reciprocal per
    // repeated denominator)
    const double rA = 1.0 / A;
    const double bh = R0 * rA, bx = R1 * rA, by = R2 * rA;
    const double dh = dt * bh;
    const double qn = sqrt(hu * hu + hv * hv);
    const bool fric = h > h_dry && qn > 0.0;
    double dqx, dqy;
    double c = 0.0, K = 0.0, jhx = 0.0, jhy = 0.0, m11 = 0.0, m12 = 0.0;
    double m22 = 0.0, rx = 0.0, ry = 0.0, det = 0.0;
    double rh = 0.0, rq = 0.0, rd = 0.0;   // 1/h, 1/|q|, 1/det
    if (fric) {
        K = h * h * cbrt(h);
        c = gm2 / K;
        const double sfx = -c * qn * hu, sfy = -c * qn * hv;
        rh = 1.0 / h;
        rq = 1.0 / qn;
        jhx = (7.0 / 3.0) * c * qn * hu * rh;
        jhy = (7.0 / 3.0) * c * qn * hv * rh;
        const double jxx = -c * (qn + hu * hu * rq);
        const double jxy = -c * hu * hv * rq;
        const double jyy = -c * (qn + hv * hv * rq);
        m11 = 1.0 - 0.5 * dt * jxx;
        m12 = -0.5 * dt * jxy;
        m22 = 1.0 - 0.5 * dt * jyy;
        rx = dt * (bx + sfx) + 0.5 * dt * jhx * dh;
        ry = dt * (by + sfy) + 0.5 * dt * jhy * dh;
        det = m11 * m22 - m12 * m12;
        rd = 1.0 / det;
        dqx = (rx * m22 - m12 * ry) * rd;
        dqy = (m11 * ry - m12 * rx) * rd;
    } else {
        dqx = dt * bx;
        dqy = dt * by;
    }
    const double hn = h + dh;
    // positivity: a clamped depth and the discharges of a dry result are
    // constants
    if (hn < 0.0) hnb = 0.0;
    if (!(hn > h_dry)) {   // h_{n+1} <= h_dry after the clamp as well
        hunb = 0.0;
        hvnb = 0.0;
    }
    hb = hnb;
    double dhb = hnb;
    hub = hunb;
    hvb = hvnb;
    const double dqxb = hunb, dqyb = hvnb;
    double bxb, byb;
    gm2b = 0.0;
    if (fric) {
        const double rxb = (dqxb * m22 - dqyb * m12) * rd;
        const double ryb = (-dqxb * m12 + dqyb * m11) * rd;
        double m22b = dqxb * rx * rd, m11b = dqyb * ry * rd;
        double m12b = -(dqxb * ry + dqyb * rx) * rd;
        const double detb = -(dqxb * dqx + dqyb * dqy) * rd;
        m11b += detb * m22;
        m22b += detb * m11;
        m12b += -2.0 * detb * m12;
        bxb = rxb * dt;
        const double sfxb = rxb * dt;
        const double jhxb = rxb * 0.5 * dt * dh;
        dhb += rxb * 0.5 * dt * jhx;
        byb = ryb * dt;
        const double sfyb = ryb * dt;
        const double jhyb = ryb * 0.5 * dt * dh;
        dhb += ryb * 0.5 * dt * jhy;
        const double jxxb = -0.5 * dt * m11b;
        const double jxyb = -0.5 * dt * m12b;
        const double jyyb = -0.5 * dt * m22b;
        double cb = 0.0, qnb = 0.0;
        const double rq2 = rq * rq;
        cb += -jxxb * (qn + hu * hu * rq);
        qnb += -jxxb * c * (1.0 - hu * hu * rq2);
        hub += -jxxb * c * 2.0 * hu * rq;
        cb += -jxyb * hu * hv * rq;
        hub += -jxyb * c * hv * rq;
        hvb += -jxyb * c * hu * rq;
        qnb += jxyb * c * hu * hv * rq2;
        cb += -jyyb * (qn + hv * hv * rq);
        qnb += -jyyb * c * (1.0 - hv * hv * rq2);
        hvb += -jyyb * c * 2.0 * hv * rq;
        cb += jhxb * (7.0 / 3.0) * qn * hu * rh;
        qnb += jhxb * (7.0 / 3.0) * c * hu * rh;
        hub += jhxb * (7.0 / 3.0) * c * qn * rh;
        hb -= jhxb * jhx * rh;
        cb += jhyb * (7.0 / 3.0) * qn * hv * rh;
        qnb += jhyb * (7.0 / 3.0) * c * hv * rh;
        hvb += jhyb * (7.0 / 3.0) * c * qn * rh;
        hb -= jhyb * jhy * rh;
        cb -= sfxb * qn * hu;
        qnb -= sfxb * c * hu;
        hub -= sfxb * c * qn;
        cb -= sfyb * qn * hv;
        qnb -= sfyb * c * hv;
        hvb -= sfyb * c * qn;
        // c = gm2 / (h^2 cbrt(h)): dc/dgm2 = 1 / K, dc/dh = -(7/3) c / h
        gm2b = cb / K;
        hb += cb * (-(7.0 / 3.0) * c * rh);
        hub += qnb * hu * rq;
        hvb += qnb * hv * rq;
    } else {
        bxb = dt * dqxb;
        byb = dt * dqyb;
    }
    const double bhb = dt * dhb;
    R0b = bhb * rA;
    R1b = bxb * rA;
    R2b = byb * rA;
}

__device__ __forceinline__ CellState cell_at(const AdjArgs &a, int c)
{
    CellState s;
    s.h = at(a.h, c);
    s.z = at(a.z, c);
    s.u = 0.0;
    s.v = 0.0;
    if (s.h > a.h_dry) {
        const double r = 1.0 / s.h;
        s.u = at(a.hu, c) * r;
        s.v = at(a.hv, c) * r;
    }
    return s;
}

// A block dormant in the forward step whose cells all hold no water
// (h == 0): its cells took the quiet dry path, every edge touching them
// added exact zeros, so the reverse step reduces to lambda_h passing
// through (lambda_hu = lambda_hv = 0) with no gradient. The check of h
// keeps the shortcut exact even for a quiet cell with a film of water.
template <int NC>
__device__ __forceinline__ bool dormant_dry(const AdjArgs &a, int blk,
                                           bool owner, int i)
{
    if (!a.ran || a.ran[blk] != 0) return false;
    const bool dry = !owner || at(a.h, i) == 0.0;
    return __syncthreads_and(dry) != 0;
}

template <int NC>
__global__ __launch_bounds__(NC) void adj_cell_kernel(AdjArgs a)
{
    __shared__ double s_h[NC], s_u[NC], s_v[NC], s_z[NC];
    __shared__ double s_c[9 * NC];   // [component][side][cell]
    const int tid = threadIdx.x, blk = blockIdx.x;
    const int c0 = blk * NC, nc = min(NC, a.n_cells - c0);
    const bool owner = tid < nc;
    const int i = c0 + tid;
    if (dormant_dry<NC>(a, blk, owner, i)) {
        // what the cell reverse gives for h = 0 and R = 0 (hn = 0 <= h_dry)
        if (owner) {
            const double lh = at(a.lam_h, i);
            at(a.ld_h, i) = lh;
            at(a.ld_hu, i) = 0.0;
            at(a.ld_hv, i) = 0.0;
            at(a.lr_h, i) = a.dt * lh / at(a.area, i);
            at(a.lr_hu, i) = 0.0;
            at(a.lr_hv, i) = 0.0;
        }
        return;
    }
    const int e0 = a.blk_edge[blk], ne = a.blk_edge[blk + 1] - e0;
    const double g = a.g, h_dry = a.h_dry;
    // the block's records first (edges to other blocks come first in the
    // list), then the neighbour of the first edge, as in the forward step
    int32_t ea = 0, eb = 0, ea2 = 0, eb2 = 0;
    if (tid < ne) {
        ea = at(a.be_a, e0 + tid);
        eb = at(a.be_b, e0 + tid);
    }
    if (tid + NC < ne) {
        ea2 = at(a.be_a, e0 + tid + NC);
        eb2 = at(a.be_b, e0 + tid + NC);
    }
    if (owner) {
        const CellState s = cell_at(a, i);
        s_h[tid] = s.h;
        s_u[tid] = s.u;
        s_v[tid] = s.v;
        s_z[tid] = s.z;
    }
    CellState X;
    X.h = 0.0; X.u = 0.0; X.v = 0.0; X.z = 0.0;
    {
        const bool xa = uint32_t(ea) < kSideBoundary;
        const bool xb = uint32_t(eb) < kSideBoundary;
        if (tid < ne && (xa || xb)) X = cell_at(a, xa ? ea : eb);
    }
    __syncthreads();
    auto edge = [&](int k, int32_t va, int32_t vb, const CellState &Y) {
        const Side pa = decode_side(va), pb = decode_side(vb);
        CellState Lc, Rc;
        Rc.h = 0.0; Rc.u = 0.0; Rc.v = 0.0; Rc.z = 0.0;
        if (pa.kind == 0) {
            Lc.h = s_h[pa.local]; Lc.u = s_u[pa.local];
            Lc.v = s_v[pa.local]; Lc.z = s_z[pa.local];
        } else {
            Lc = Y;
        }
        BcEntry bc{};
        bool idle;
        if (pb.kind == 2) {
            bc = a.bc[pb.global];
            idle = Lc.h == 0.0 && (bc.kind == 0 || bc.kind == 1);
        } else {
            if (pb.kind == 0) {
                Rc.h = s_h[pb.local]; Rc.u = s_u[pb.local];
                Rc.v = s_v[pb.local]; Rc.z = s_z[pb.local];
            } else {
                Rc = Y;
            }
            idle = Lc.h == 0.0 && Rc.h == 0.0;
        }
        double cl0 = 0.0, cl1 = 0.0, cl2 = 0.0, cr0 = 0.0, cr1 = 0.0,
               cr2 = 0.0;
        if (!idle)
            edge_contrib(g, h_dry, pb.kind == 2, bc, Lc, Rc,
                         at(a.be_nx + e0, k), at(a.be_ny + e0, k),
                         at(a.be_len + e0, k), cl0, cl1, cl2, cr0, cr1, cr2);
        if (pa.kind == 0) {
            double *d = s_c + pa.k * NC + pa.local;
            d[0] = cl0;
            d[3 * NC] = cl1;
            d[6 * NC] = cl2;
        }
        if (pb.kind == 0) {
            double *d = s_c + pb.k * NC + pb.local;
            d[0] = cr0;
            d[3 * NC] = cr1;
            d[6 * NC] = cr2;
        }
    };
    if (tid < ne) edge(tid, ea, eb, X);
    for (int k = tid + NC; k < ne; k += NC) {
        int32_t va = ea2, vb = eb2;
        if (k != tid + NC) {
            va = at(a.be_a, e0 + k);
            vb = at(a.be_b, e0 + k);
        }
        CellState Y;
        Y.h = 0.0; Y.u = 0.0; Y.v = 0.0; Y.z = 0.0;
        if (uint32_t(va) < kSideBoundary) Y = cell_at(a, va);
        if (uint32_t(vb) < kSideBoundary) Y = cell_at(a, vb);
        edge(k, va, vb, Y);
    }
    __syncthreads();
    if (!owner) return;
    double R0 = 0.0, R1 = 0.0, R2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        R0 += s_c[k * NC + tid];
        R1 += s_c[(3 + k) * NC + tid];
        R2 += s_c[(6 + k) * NC + tid];
    }
    const double h = at(a.h, i);
    double hb, hub, hvb, R0b, R1b, R2b, gm2b;
    cell_update_rev(h_dry, a.dt, at(a.area, i),
                    h > h_dry ? at(a.gm2, i) : 0.0, h, at(a.hu, i),
                    at(a.hv, i), R0, R1, R2, at(a.lam_h, i), at(a.lam_hu, i),
                    at(a.lam_hv, i), hb, hub, hvb, R0b, R1b, R2b, gm2b);
    at(a.ld_h, i) = hb;
    at(a.ld_hu, i) = hub;
    at(a.ld_hv, i) = hvb;
    at(a.lr_h, i) = R0b;
    at(a.lr_hu, i) = R1b;
    at(a.lr_hv, i) = R2b;
    if (gm2b != 0.0) at(a.grad_gm2, i) += gm2b;
}

// The cell pass when the forward step stored its summed contributions R:
// the reverse of the cell update from the stored R (the same values the
// edge evaluation of adj_cell_kernel gives), one thread per cell.
template <int NC>
__global__ __launch_bounds__(NC) void adj_cell_stored_kernel(AdjArgs a)
{
    const int tid = threadIdx.x, blk = blockIdx.x;
    const int c0 = blk * NC, nc = min(NC, a.n_cells - c0);
    const bool owner = tid < nc;
    const int i = c0 + tid;
    const bool skip = dormant_dry<NC>(a, blk, owner, i);
    if (!owner) return;
    if (skip) {
        const double lh = at(a.lam_h, i);
        at(a.ld_h, i) = lh;
        at(a.ld_hu, i) = 0.0;
        at(a.ld_hv, i) = 0.0;
        at(a.lr_h, i) = a.dt * lh / at(a.area, i);
        at(a.lr_hu, i) = 0.0;
        at(a.lr_hv, i) = 0.0;
        return;
    }
    const double R0 = a.R[i], R1 = a.R[a.n_cells + i],
                 R2 = a.R[2 * a.n_cells + i];
    const double h = at(a.h, i), h_dry = a.h_dry;
    double hb, hub, hvb, R0b, R1b, R2b, gm2b;
    cell_update_rev(h_dry, a.dt, at(a.area, i),
                    h > h_dry ? at(a.gm2, i) : 0.0, h, at(a.hu, i),
                    at(a.hv, i), R0, R1, R2, at(a.lam_h, i), at(a.lam_hu, i),
                    at(a.lam_hv, i), hb, hub, hvb, R0b, R1b, R2b, gm2b);
    at(a.ld_h, i) = hb;
    at(a.ld_hu, i) = hub;
    at(a.ld_hv, i) = hvb;
    at(a.lr_h, i) = R0b;
    at(a.lr_hu, i) = R1b;
    at(a.lr_hv, i) = R2b;
    if (gm2b != 0.0) at(a.grad_gm2, i) += gm2b;
}

template <int NC>
__global__ __launch_bounds__(NC) void adj_edge_kernel(AdjArgs a)
{
    __shared__ double s_h[NC], s_u[NC], s_v[NC], s_z[NC];
    __shared__ double s_r[3 * NC];    // lr of the block's cells
    __shared__ double s_a[12 * NC];   // [h, hu, hv, z][side][cell]
    const int tid = threadIdx.x, blk = blockIdx.x;
    const int c0 = blk * NC, nc = min(NC, a.n_cells - c0);
    const bool owner = tid < nc;
    const int i = c0 + tid;
    if (dormant_dry<NC>(a, blk, owner, i)) {
        if (owner) {
            at(a.lam_out_h, i) = at(a.lam_h, i) + 0.0;
            at(a.lam_out_hu, i) = 0.0;
            at(a.lam_out_hv, i) = 0.0;
        }
        return;
    }
    const int e0 = a.blk_edge[blk], ne = a.blk_edge[blk + 1] - e0;
    const double g = a.g, h_dry = a.h_dry;
    if (owner) {
        const CellState s = cell_at(a, i);
        s_h[tid] = s.h;
        s_u[tid] = s.u;
        s_v[tid] = s.v;
        s_z[tid] = s.z;
        s_r[tid] = at(a.lr_h, i);
        s_r[NC + tid] = at(a.lr_hu, i);
        s_r[2 * NC + tid] = at(a.lr_hv, i);
    }
    __syncthreads();
    for (int k = tid; k < ne; k += NC) {
        const Side pa = decode_side(at(a.be_a, e0 + k));
        const Side pb = decode_side(at(a.be_b, e0 + k));
        CellState Lc, Rc;
        double lb[3], rb[3] = {0.0, 0.0, 0.0};
        if (pa.kind == 0) {
            Lc.h = s_h[pa.local]; Lc.u = s_u[pa.local];
            Lc.v = s_v[pa.local]; Lc.z = s_z[pa.local];
            lb[0] = s_r[pa.local];
            lb[1] = s_r[NC + pa.local];
            lb[2] = s_r[2 * NC + pa.local];
        } else {
            Lc = cell_at(a, pa.global);
            lb[0] = at(a.lr_h, pa.global);
            lb[1] = at(a.lr_hu, pa.global);
            lb[2] = at(a.lr_hv, pa.global);
        }
        SideAdj La{0.0, 0.0, 0.0, 0.0}, Ra{0.0, 0.0, 0.0, 0.0};
        if (pb.kind == 2) {
            const BcEntry bc = a.bc[pb.global];
            if (!(Lc.h == 0.0 && (bc.kind == 0 || bc.kind == 1)))
                boundary_edge_rev(g, h_dry, bc, Lc, at(a.be_nx + e0, k),
                                  at(a.be_ny + e0, k), at(a.be_len + e0, k),
                                  lb, La);
        } else {
            if (pb.kind == 0) {
                Rc.h = s_h[pb.local]; Rc.u = s_u[pb.local];
                Rc.v = s_v[pb.local]; Rc.z = s_z[pb.local];
                rb[0] = s_r[pb.local];
                rb[1] = s_r[NC + pb.local];
                rb[2] = s_r[2 * NC + pb.local];
            } else {
                Rc = cell_at(a, pb.global);
                rb[0] = at(a.lr_h, pb.global);
                rb[1] = at(a.lr_hu, pb.global);
                rb[2] = at(a.lr_hv, pb.global);
            }
            if (!(Lc.h == 0.0 && Rc.h == 0.0))
                interior_edge_rev(g, h_dry, Lc, Rc, at(a.be_nx + e0, k),
                                  at(a.be_ny + e0, k), at(a.be_len + e0, k),
                                  lb, rb, La, Ra);
        }
        if (pa.kind == 0) {
            double *d = s_a + pa.k * NC + pa.local;
            d[0] = La.h;
            d[3 * NC] = La.hu;
            d[6 * NC] = La.hv;
            d[9 * NC] = La.z;
        }
        if (pb.kind == 0) {
            double *d = s_a + pb.k * NC + pb.local;
            d[0] = Ra.h;
            d[3 * NC] = Ra.hu;
            d[6 * NC] = Ra.hv;
            d[9 * NC] = Ra.z;
        }
    }
    __syncthreads();
    if (!owner) return;
    double lh = at(a.ld_h, i), lhu = at(a.ld_hu, i), lhv = at(a.ld_hv, i);
    double lz = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        lh += s_a[k * NC + tid];
        lhu += s_a[(3 + k) * NC + tid];
        lhv += s_a[(6 + k) * NC + tid];
        lz += s_a[(9 + k) * NC + tid];
    }
    at(a.lam_out_h, i) = lh;
    at(a.lam_out_hu, i) = lhu;
    at(a.lam_out_hv, i) = lhv;
    if (lz != 0.0) at(a.grad_z, i) += lz;
}

__global__ __launch_bounds__(256) void gm2_to_manning_kernel(
    const double *gm2_grad, const double *man, double g, int64_t n,
    double *out)
{
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < n;
         k += int64_t(gridDim.x) * blockDim.x)
        out[k] = gm2_grad[k] * (2.0 * g * man[k]);   // d(g m m)/dm = 2 g m
}

}  // namespace

hipError_t launch_adjoint_step(const AdjArgs &a, int block_cells,
                               hipStream_t s)
{
    if (block_cells != 256) return hipErrorInvalidValue;
    if (a.R)
        hipLaunchKernelGGL(adj_cell_stored_kernel<256>, dim3(a.n_blocks),
                           dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(adj_cell_kernel<256>, dim3(a.n_blocks), dim3(256),
                           0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(adj_edge_kernel<256>, dim3(a.n_blocks), dim3(256), 0,
                       s, a);
    return hipGetLastError();
}

hipError_t launch_manning_gradient(const double *gm2_grad, const double *man,
                                   double g, int64_t n, double *out,
                                   hipStream_t s)
{
    int64_t b = (n + 255) / 256;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    hipLaunchKernelGGL(gm2_to_manning_kernel, dim3(unsigned(b)), dim3(256),
                       0, s, gm2_grad, man, g, n, out);
    return hipGetLastError();
}

}  // namespace swe

"""Exact solution of the 1D Riemann problem for an ideal gas (TEST INFRASTRUCTURE).

Used to pin the oracle: the paper checks its Sod shock tube (section 3.1)
against the analytic solution with the L1 metric of section 3 (equation
"l1_error"), cell averages taken by 10-node Gauss-Legendre quadrature.

The solver follows the textbook construction (Toro, "Riemann Solvers and
Numerical Methods for Fluid Dynamics", 3rd ed., chapter 4): the star pressure
is the root of f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock
(Rankine-Hugoniot) branch for p > p_K and the rarefaction (isentropic) branch
otherwise; Newton's method starts from the primitive-variable guess and runs
to a relative change below 1e-15.  The self-similar solution is then sampled
at xi = (x - x0)/t.
"""
import numpy as np


class RiemannSolution:
    def __init__(self, rhoL, uL, pL, rhoR, uR, pR, gamma=1.4):
        self.g = float(gamma)
        self.L = (float(rhoL), float(uL), float(pL))
        self.R = (float(rhoR), float(uR), float(pR))
        g = self.g
        self.cL = np.sqrt(g * pL / rhoL)
        self.cR = np.sqrt(g * pR / rhoR)
        if 2.0 / (g - 1.0) * (self.cL + self.cR) <= uR - uL:
            raise ValueError("initial data generate vacuum")
        self.pstar, self.ustar = self._star()

    # f_K(p) and its derivative for one side
    def _f(self, p, rhoK, pK, cK):
        g = self.g
        if p > pK:
            A = 2.0 / ((g + 1.0) * rhoK)
            B = (g - 1.0) / (g + 1.0) * pK
            q = np.sqrt(A / (p + B))
            return (p - pK) * q, q * (1.0 - 0.5 * (p - pK) / (B + p))
        r = p / pK
        f = 2.0 * cK / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rhoK * cK) * r ** (-(g + 1.0) / (2.0 * g))
        return f, df

    def _star(self):
        rhoL, uL, pL = self.L
        rhoR, uR, pR = self.R
        cL, cR = self.cL, self.cR
        du = uR - uL
        p = 0.5 * (pL + pR) - 0.125 * du * (rhoL + rhoR) * (cL + cR)
        p = max(p, 1e-12 * min(pL, pR))
        for _ in range(200):
            fL, dfL = self._f(p, rhoL, pL, cL)
            fR, dfR = self._f(p, rhoR, pR, cR)
            pn = p - (fL + fR + du) / (dfL + dfR)
            if pn <= 0.0:
                pn = 0.5 * p
            change = abs(pn - p) / (0.5 * (pn + p))
            p = pn
            if change < 1e-15:
                break
        fL, _ = self._f(p, rhoL, pL, cL)
        fR, _ = self._f(p, rhoR, pR, cR)
        u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
        return p, u

    def star_densities(self):
        """(rho*_L, rho*_R)."""
        g = self.g
        out = []
        for (rhoK, _, pK) in (self.L, self.R):
            r = self.pstar / pK
            if r > 1.0:
                gr = (g - 1.0) / (g + 1.0)
                out.append(rhoK * (r + gr) / (gr * r + 1.0))
            else:
                out.append(rhoK * r ** (1.0 / g))
        return tuple(out)

    def wave_speeds(self):
        """Dictionary of the left/right wave edges (shock speed or fan head/tail)."""
        g = self.g
        rhoL, uL, pL = self.L
        rhoR, uR, pR = self.R
        ps, us = self.pstar, self.ustar
        w = {"contact": us}
        if ps > pL:
            w["left_shock"] = uL - self.cL * np.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
        else:
            w["left_head"] = uL - self.cL
            w["left_tail"] = us - self.cL * (ps / pL) ** ((g - 1) / (2 * g))
        if ps > pR:
            w["right_shock"] = uR + self.cR * np.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
        else:
            w["right_head"] = uR + self.cR
            w["right_tail"] = us + self.cR * (ps / pR) ** ((g - 1) / (2 * g))
        return w

    def sample(self, xi):
        """(rho, u, p) at similarity coordinate(s) xi = (x - x0)/t."""
        xi = np.asarray(xi, dtype=np.float64)
        g = self.g
        rhoL, uL, pL = self.L
        rhoR, uR, pR = self.R
        cL, cR = self.cL, self.cR
        ps, us = self.pstar, self.ustar
        rsL, rsR = self.star_densities()
        rho = np.empty_like(xi)
        u = np.empty_like(xi)
        p = np.empty_like(xi)

        left = xi <= us
        # ---- left of the contact
        if ps > pL:
            SL = uL - cL * np.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
            a = left & (xi <= SL)
            b = left & (xi > SL)
            rho[a], u[a], p[a] = rhoL, uL, pL
            rho[b], u[b], p[b] = rsL, us, ps
        else:
            SH = uL - cL
            ST = us - cL * (ps / pL) ** ((g - 1) / (2 * g))
            a = left & (xi <= SH)
            b = left & (xi > ST)
            f = left & (xi > SH) & (xi <= ST)
            rho[a], u[a], p[a] = rhoL, uL, pL
            rho[b], u[b], p[b] = rsL, us, ps
            c = 2.0 / (g + 1) * (cL + 0.5 * (g - 1) * (uL - xi[f]))
            u[f] = 2.0 / (g + 1) * (cL + 0.5 * (g - 1) * uL + xi[f])
            rho[f] = rhoL * (c / cL) ** (2.0 / (g - 1))
            p[f] = pL * (c / cL) ** (2.0 * g / (g - 1))
        # ---- right of the contact
        right = ~left
        if ps > pR:
            SR = uR + cR * np.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
            a = right & (xi >= SR)
            b = right & (xi < SR)
            rho[a], u[a], p[a] = rhoR, uR, pR
            rho[b], u[b], p[b] = rsR, us, ps
        else:
            SH = uR + cR
            ST = us + cR * (ps / pR) ** ((g - 1) / (2 * g))
            a = right & (xi >= SH)
            b = right & (xi <= ST)
            f = right & (xi < SH) & (xi > ST)
            rho[a], u[a], p[a] = rhoR, uR, pR
            rho[b], u[b], p[b] = rsR, us, ps
            c = 2.0 / (g + 1) * (cR - 0.5 * (g - 1) * (uR - xi[f]))
            u[f] = 2.0 / (g + 1) * (-cR + 0.5 * (g - 1) * uR + xi[f])
            rho[f] = rhoR * (c / cR) ** (2.0 / (g - 1))
            p[f] = pR * (c / cR) ** (2.0 * g / (g - 1))
        return rho, u, p

    def cell_averages(self, n, t, x0=0.5, xlo=0.0, xhi=1.0, nodes=10):
        """Gauss-Legendre cell averages of (rho, u, p) on n uniform cells."""
        xg, wg = np.polynomial.legendre.leggauss(nodes)
        dx = (xhi - xlo) / n
        centres = xlo + (np.arange(n) + 0.5) * dx
        x = centres[:, None] + 0.5 * dx * xg[None, :]
        rho, u, p = self.sample((x - x0) / t)
        avg = lambda q: 0.5 * (q * wg[None, :]).sum(axis=1)
        return avg(rho), avg(u), avg(p)

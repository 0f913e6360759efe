"""Nondimensional parameters from physical inputs (oracle; test infrastructure only).

One layer (Sec. 2.1): Sverdrup velocity V = pi tau0/(rho H beta L) (not needed
when V is given), Ro = V/(beta L^2) = (delta_I/L)^2, Munk scale
delta_M/L = (nu/(beta L^3))^(1/3) = (Ro/Re)^(1/3), so Re = Ro/(delta_M/L)^3,
Re_B = Re delta_I/L.

Two layers (Sec. 2.2): V = 2 pi tau0/(rho1 H1 beta L), Ro = V/(beta L^2),
Fr = f0^2 V/(g' beta H), A = nu/(beta L^3), sigma = gamma/(beta L),
delta = H1/H, length scales delta_M = (nu/beta)^(1/3), delta_S = gamma/beta,
delta_I = (V/beta)^(1/2), R_d = (g' H1 H2/(f0^2 H))^(1/2); Re = Ro/A.

Vorticity-form coefficients used by the step: 1/Ro, 1/Re, F1 = Fr/(Ro delta),
F2 = Fr/(Ro (1 - delta)), bottom drag sigma/Ro.
"""
from __future__ import annotations

import math

SECONDS_PER_YEAR = 365.25 * 86400.0


def one_layer(L, beta, nu, V):
    Ro = V / (beta * L * L)
    dM = (nu / (beta * L ** 3)) ** (1.0 / 3.0)
    dI = math.sqrt(Ro)
    Re = Ro / dM ** 3
    return dict(Ro=Ro, Re=Re, delta_M_over_L=dM, delta_I_over_L=dI, Re_B=Re * dI,
                L_over_V_years=L / V / SECONDS_PER_YEAR)


def two_layer(L, H1, H2, f0, beta, rho1, gprime, tau0, gamma, nu):
    H = H1 + H2
    V = 2.0 * math.pi * tau0 / (rho1 * H1 * beta * L)
    Ro = V / (beta * L * L)
    Fr = f0 * f0 * V / (gprime * beta * H)
    A = nu / (beta * L ** 3)
    sigma = gamma / (beta * L)
    delta = H1 / H
    Rd = math.sqrt(gprime * H1 * H2 / (f0 * f0 * H))
    out = dict(V=V, Ro=Ro, Fr=Fr, A=A, sigma=sigma, delta=delta, Re=Ro / A,
               delta_M=(nu / beta) ** (1.0 / 3.0), delta_S=gamma / beta,
               delta_I=math.sqrt(V / beta), Rd=Rd, L_over_V_years=L / V / SECONDS_PER_YEAR,
               L_over_Rd=L / Rd)
    out.update(vorticity_form_two_layer(Ro, Fr, delta, sigma, A))
    return out


def vorticity_form_two_layer(Ro, Fr, delta, sigma, A):
    return dict(f1=Fr / (Ro * delta), f2=Fr / (Ro * (1.0 - delta)), drag=sigma / Ro,
                inv_re=A / Ro, inv_ro=1.0 / Ro)

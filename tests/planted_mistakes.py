"""Planted mistakes: each entry below puts one plausible mistake (a dropped term, a wrong
sign, coefficient or index, a swapped operand) into a copy of the oracle, and the CPU pins
(tests/test_oracle_*.py) are run against that copy: every mistake must fail at least one
pin.  The oracle under oracle/ is never modified.

Not collected by pytest (about half an hour on 8 cores).  Usage, from the repository root:

    python tests/planted_mistakes.py [ids...]

The copies live under _build/planted/.  Exit status 1 if any mistake passes every pin.
"""
import json
import os
import shutil
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WORK = os.path.join(ROOT, "_build", "planted")
C = "oracle/aq_oracle.c"
D = "oracle/diagnostics.py"

M = [  # id, file, description, old, new
 ("S_quad", C, "eq. 8 quadratic coefficient 9/2 -> 3", "4.5 * eu * eu", "3.0 * eu * eu"),
 ("S_uu_sign", C, "eq. 8 |u|^2 term sign", "- 1.5 * uu", "+ 1.5 * uu"),
 ("S_lin", C, "eq. 8 linear coefficient 3 -> 1", "(3.0 * eu + 4.5", "(1.0 * eu + 4.5"),
 ("w_diag", C, "diagonal weight 1/36 -> 1/18", "1.0 / 9.0 : 1.0 / 36.0", "1.0 / 9.0 : 1.0 / 18.0"),
 ("w_rest", C, "rest weight 4/9 -> 1/3", "i == 0 ? 4.0 / 9.0", "i == 0 ? 1.0 / 3.0"),
 ("sigma", C, "sigma 5/12 -> 1/2", "sigma_ = 5.0 / 12.0", "sigma_ = 0.5"),
 ("gamma", C, "gamma 1/12 -> 1/9", "1.0 / 3.0 : 1.0 / 12.0", "1.0 / 3.0 : 1.0 / 9.0"),
 ("mom_uy_index", C, "u_y summed with e_x", "uy += ey[i] * h8[i - 1];", "uy += ex[i] * h8[i - 1];"),
 ("mom_S0", C, "eq. 9 S_0(u) dropped", "(sum + S(0, ux, uy))", "(sum)"),
 ("mom_T_ref", C, "T without T_ref", "m.T = s->P.T_ref + T;", "m.T = T;"),
 ("buoy_T0", C, "buoyancy about T_ref instead of T0", "double Bx = P->gbeta * (m.T - P->T0)", "double Bx = P->gbeta * (m.T - P->T_ref)"),
 ("buoy_axes", C, "gravity components swapped", "(m.T - P->T0) * s->gx_hat;", "(m.T - P->T0) * s->gy_hat;"),
 ("buoy_sign", C, "buoyancy sign", "double By = P->gbeta * (m.T - P->T0) * s->gy_hat;", "double By = -P->gbeta * (m.T - P->T0) * s->gy_hat;"),
 ("darcy_mid", C, "Darcy mid-step denominator 1 + nu/K", "/ (1.0 + 0.5 * nuK);\n        double uDy", "/ (1.0 + nuK);\n        double uDy"),
 ("darcy_u", C, "Darcy drag on u instead of u_D", "Dx = -nuK * uDx;", "Dx = -nuK * m.ux;"),
 ("darcy_w", C, "Darcy link weights w_i instead of 3 w_i", "Fi += 3.0 * w_flow(i)", "Fi += 1.0 * w_flow(i)"),
 ("force_half", C, "eq. 17 factor 1/2 -> 1", "? 0.5 * (ex[i] * Bx + ey[i] * By)", "? 1.0 * (ex[i] * Bx + ey[i] * By)"),
 ("force_diag", C, "eq. 17 force on the diagonals too", "double Fi = (i <= 4) ?", "double Fi = (i <= 8) ?"),
 ("bgk_sign", C, "eq. 6 relaxation sign", "h8[i - 1] - omega * (h8[i - 1] - heq) + Fi", "h8[i - 1] - omega * (heq - h8[i - 1]) + Fi"),
 ("heq_lambda", C, "eq. 7 lambda_i dp dropped", "double heq = lambda_i(i) * m.dp + S(i, m.ux, m.uy);", "double heq = S(i, m.ux, m.uy);"),
 ("geq_dev", C, "eq. 12 advective term on the deviation T - T_ref", "((m.T - P->T_ref) + m.T * eu / cs2T)", "((m.T - P->T_ref) + (m.T - P->T_ref) * eu / cs2T)"),
 ("cs2T", C, "thermal c_s^2 (1-w0)/2 -> (1-w0)/3", "double omegaT = 1.0 / P->tau_t;\n    double cs2T = (1.0 - P->w0) / 2.0;", "double omegaT = 1.0 / P->tau_t;\n    double cs2T = (1.0 - P->w0) / 3.0;"),
 ("omegaT", C, "thermal relaxation uses tau_f", "double omegaT = 1.0 / P->tau_t;", "double omegaT = 1.0 / P->tau_f;"),
 ("nu", C, "eq. 10 viscosity (2tau-1)/3", "return (2.0 * P->tau_f - 1.0) / 6.0;", "return (2.0 * P->tau_f - 1.0) / 3.0;"),
 ("bz_hi", C, "Bouzidi q>=1/2 second weight", "(2.0 * q - 1.0) / (2.0 * q) * s->hs", "(2.0 * q - 1.0) / q * s->hs"),
 ("bz_lo", C, "Bouzidi q<1/2 second weight", "(1.0 - 2.0 * q) * s->hs", "(1.0 - q) * s->hs"),
 ("bz_lo_idx", C, "Bouzidi q<1/2 reads the opposite population", "(1.0 - 2.0 * q) * s->hs[(size_t)(i - 1) * n + kb]", "(1.0 - 2.0 * q) * s->hs[(size_t)(ib - 1) * n + kb]"),
 ("inlet_coef", C, "moving-wall inlet 6 w_i -> 3 w_i", "*back = hout - 6.0 * w_flow(i) * eu;                /* moving wall u_in */", "*back = hout - 3.0 * w_flow(i) * eu;                /* moving wall u_in */"),
 ("inlet_sign", C, "moving-wall inlet sign", "*back = hout - 6.0 * w_flow(i) * eu;                /* moving wall u_in */", "*back = hout + 6.0 * w_flow(i) * eu;                /* moving wall u_in */"),
 ("abb_coef", C, "pressure ABB 2 lambda_i -> lambda_i", "*back = -hout + 2.0 * lambda_i(i) * (P->p_out - P->p_ref);", "*back = -hout + 1.0 * lambda_i(i) * (P->p_out - P->p_ref);"),
 ("abb_sign", C, "pressure ABB as bounce-back", "*back = -hout + 2.0 * lambda_i(i)", "*back = hout + 2.0 * lambda_i(i)"),
 ("abb_pref", C, "pressure ABB without p_ref", "2.0 * lambda_i(i) * (P->p_out - P->p_ref); /* pressure ABB */", "2.0 * lambda_i(i) * (P->p_out); /* pressure ABB */"),
 ("lumped_dir", C, "lumped outlet direction off by one", "int d = s->wall[kk] + 1;                            /* outward axis link */", "int d = s->wall[kk];                            /* outward axis link */"),
 ("lumped_coef", C, "lumped moving wall 6 w_i -> 3 w_i", "*back = hout - 6.0 * w_flow(i) * eu;                /* moving wall u_s n */", "*back = hout - 3.0 * w_flow(i) * eu;                /* moving wall u_s n */"),
 ("seep_nu", C, "seepage K*mu instead of K/mu", "return P->K_tm / nu_of(P) *", "return P->K_tm * nu_of(P) *"),
 ("seep_psc", C, "seepage without p_sc", "((p_iop - P->p_sc) / P->h_tm)", "((p_iop) / P->h_tm)"),
 ("seep_pref", C, "seepage against p_ref instead of p_sc", "((p_iop - P->p_sc) / P->h_tm)", "((p_iop - P->p_ref) / P->h_tm)"),
 ("dir_coef", C, "thermal Dirichlet ABB 2 w -> w", "*back = -gout + 2.0 * w_heat(P, i) * (Tw - P->T_ref);", "*back = -gout + 1.0 * w_heat(P, i) * (Tw - P->T_ref);"),
 ("dir_sign", C, "thermal Dirichlet as adiabatic", "*back = -gout + 2.0 * w_heat(P, i) * (Tw - P->T_ref);", "*back = gout + 2.0 * w_heat(P, i) * (Tw - P->T_ref);"),
 ("inlet_T", C, "INLET temperature taken from the wall", "double Tw = (c == OR_INLET) ? P->T_inlet : wall_temperature(s, wall);\n                    *back = -gout", "double Tw = wall_temperature(s, wall);\n                    *back = -gout"),
 ("walls_swapped", C, "cornea and iris temperatures swapped", "wall == OR_WALL_CORNEA ? s->P.T_cornea : s->P.T_iris", "wall == OR_WALL_CORNEA ? s->P.T_iris : s->P.T_cornea"),
 ("box_dirichlet", C, "BOX wall treated as Dirichlet", "} else if ((c == OR_SOLID && wall != OR_WALL_BOX) || c == OR_INLET) {\n                    double Tw", "} else if ((c == OR_SOLID) || c == OR_INLET) {\n                    double Tw"),
 ("rest_pop", C, "rest thermal population not collided", "s->gn[k] = s->gs[k];   /* rest population stays */", "s->gn[k] = s->g[k];   /* rest population stays */"),
 ("ext_neq", C, "extrapolation without the non-equilibrium part", "*back = heq_of(ib, dpb, uxb, uyb) + (s->hs[(size_t)(ib - 1) * n + k] - heq_of(ib, ms.dp, ms.ux, ms.uy));\n                    if (c == OR_INLET) q_in", "*back = heq_of(ib, dpb, uxb, uyb);\n                    if (c == OR_INLET) q_in"),
 ("ext_inlet_u", C, "extrapolated inlet at rest", "if (c == OR_INLET) {\n                        uxb = P->u_in_x;\n                        uyb = P->u_in_y;\n                    } else if (P->outlet_mode == OR_OUTLET_LUMPED) {\n                        int d = s->wall[kk] + 1;\n                        uxb = ex[d] * s->u_seep;\n                        uyb = ey[d] * s->u_seep;\n                    } else {\n                        dpb = P->p_out - P->p_ref;\n                    }\n                    *back", "if (c == OR_INLET) {\n                        uxb = 0.0;\n                        uyb = 0.0;\n                    } else if (P->outlet_mode == OR_OUTLET_LUMPED) {\n                        int d = s->wall[kk] + 1;\n                        uxb = ex[d] * s->u_seep;\n                        uyb = ey[d] * s->u_seep;\n                    } else {\n                        dpb = P->p_out - P->p_ref;\n                    }\n                    *back"),
 ("ext_outlet_p", C, "extrapolated outlet pressure without p_ref", "} else {\n                        dpb = P->p_out - P->p_ref;\n                    }\n                    *back", "} else {\n                        dpb = P->p_out;\n                    }\n                    *back"),
 ("ext_T_idx", C, "thermal extrapolation equilibrium index", "*back = geq_of(P, ib, Tw, uxb, uyb) + (s->gs[(size_t)ib * n + k] - geq_of(P, ib, ms.T, ms.ux, ms.uy));", "*back = geq_of(P, i, Tw, uxb, uyb) + (s->gs[(size_t)ib * n + k] - geq_of(P, ib, ms.T, ms.ux, ms.uy));"),
 ("wss_factor", C, "WSS factor 1 - 1/tau", "double f = -(1.0 - 0.5 / P->tau_f);", "double f = -(1.0 - 1.0 / P->tau_f);"),
 ("wss_pxy", C, "WSS Pi_xy index", "pxy += ex[i] * ey[i] * neq;", "pxy += ex[i] * ex[i] * neq;"),
 ("wss_normal", C, "WSS keeps the normal part", "double tau_w = sqrt((tx - tn * nx_) * (tx - tn * nx_) + (ty - tn * ny_) * (ty - tn * ny_));", "double tau_w = sqrt(tx * tx + ty * ty);"),
 ("iop_gauge", C, "IOP gauge against p_ref", "o->iop_gauge = o->p_mean_fluid - P->p_out;", "o->iop_gauge = o->p_mean_fluid - P->p_ref;"),
 ("iop_porous", C, "IOP averaged over porous nodes too", "if (s->cls[k] == OR_FLUID) { sum_dp += m.dp; cnt += 1.0; }", "if (1) { sum_dp += m.dp; cnt += 1.0; }"),
 ("resid_D", C, "residual not per step", "o->resid_u = u2 > 0 ? sqrt(du2) / (D * sqrt(u2))", "o->resid_u = u2 > 0 ? sqrt(du2) / (sqrt(u2))"),
 ("q_in_sign", C, "inflow sign", "q_in += *back - hout;\n                } else if (P->outlet_mode", "q_in += hout - *back;\n                } else if (P->outlet_mode"),
 ("opposite", C, "opposite of the diagonals permuted", "{0, 3, 4, 1, 2, 7, 8, 5, 6}", "{0, 3, 4, 1, 2, 8, 7, 6, 5}"),
 ("init_p", C, "initial pressure at p_ref", "lambda_i(i) * (P->p_init - P->p_ref) + S(i, 0.0, 0.0)", "lambda_i(i) * 0.0 + S(i, 0.0, 0.0)"),
 ("init_T", C, "initial temperature weights", "G(s, i, k) = act ? w_heat(P, i) * (P->T_init - P->T_ref) : NAN;", "G(s, i, k) = act ? 0.2 * (P->T_init - P->T_ref) : NAN;"),
 ("porous_all", C, "Darcy drag on every node", "collide_node(s, s->cls[k] == OR_POROUS, h8, g5, h8s, g5s);", "collide_node(s, 1, h8, g5, h8s, g5s);"),
 ("grav_angle", C, "gravity angle components swapped", "s->gx_hat = sin(P->gravity_angle);\n    s->gy_hat = cos(P->gravity_angle);", "s->gx_hat = cos(P->gravity_angle);\n    s->gy_hat = sin(P->gravity_angle);"),
 ("vort_sign", D, "vorticity as a sum of the cross derivatives", "0.5 * (_derivative(uy, act, x, y, 1, 0) - _derivative(ux, act, x, y, 0, 1))", "0.5 * (_derivative(uy, act, x, y, 1, 0) + _derivative(ux, act, x, y, 0, 1))"),
 ("vort_half", D, "vorticity without the factor 1/2", "w[y, x] = 0.5 * (", "w[y, x] = 1.0 * ("),
 ("central", D, "central difference without the 1/2", "(f[y + dy, x + dx] - f[y - dy, x - dx]) / 2.0", "(f[y + dy, x + dx] - f[y - dy, x - dx]) / 1.0"),
 ("one_sided", D, "forward one-sided difference sign", "return f[y + dy, x + dx] - f[y, x]", "return f[y, x] - f[y + dy, x + dx]"),
 ("intensity", D, "intensity without the factor 2", "float(2.0 * np.sum(np.abs(w[fluid])))", "float(1.0 * np.sum(np.abs(w[fluid])))"),
 ("psi_axis", D, "stream function summed along x", "np.cumsum(np.where(act, ux, 0.0), axis=0)", "np.cumsum(np.where(act, ux, 0.0), axis=1)"),
 ("psi_uy", D, "stream function sign", "def stream_function(ux, mask):\n    act = _active(mask)\n    return np.cumsum(np.where(act, ux, 0.0), axis=0)", "def stream_function(ux, mask):\n    act = _active(mask)\n    return np.cumsum(np.where(act, -ux, 0.0), axis=0)"),
 ("ext_lumped_dir", C, "extrapolated lumped outlet direction off by one",
  "} else if (P->outlet_mode == OR_OUTLET_LUMPED) {\n                        int d = s->wall[kk] + 1;\n                        uxb = ex[d] * s->u_seep;\n                        uyb = ey[d] * s->u_seep;\n                    } else {\n                        dpb = P->p_out - P->p_ref;\n                    }\n                    *back",
  "} else if (P->outlet_mode == OR_OUTLET_LUMPED) {\n                        int d = s->wall[kk];\n                        uxb = ex[d] * s->u_seep;\n                        uyb = ey[d] * s->u_seep;\n                    } else {\n                        dpb = P->p_out - P->p_ref;\n                    }\n                    *back"),
 ("ext_q_out", C, "outflow of the extrapolated outlet with the wrong sign",
  "if (c == OR_INLET) q_in += *back - hout;\n                    else q_out += hout - *back;",
  "if (c == OR_INLET) q_in += *back - hout;\n                    else q_out += *back - hout;"),
 ("abb_q_out", C, "outflow of the pressure outlet with the wrong sign",
  "*back = -hout + 2.0 * lambda_i(i) * (P->p_out - P->p_ref); /* pressure ABB */\n                    q_out += hout - *back;",
  "*back = -hout + 2.0 * lambda_i(i) * (P->p_out - P->p_ref); /* pressure ABB */\n                    q_out += *back - hout;"),
 ("ext_T_inlet_u", C, "thermal extrapolation at the inlet with the fluid at rest",
  "double uxb = c == OR_INLET ? P->u_in_x : 0.0, uyb = c == OR_INLET ? P->u_in_y : 0.0;\n                    moments ms = post_moments(s, k);                        /* extrapolation */",
  "double uxb = 0.0, uyb = 0.0;\n                    moments ms = post_moments(s, k);                        /* extrapolation */"),
 ("bz_fallback", C, "interpolation for q < 1/2 without an active node behind",
  "} else if (q > 0.0 && kb >= 0 && is_active(s, (size_t)kb)) {",
  "} else if (q > 0.0 && kb >= 0) {"),
 ("bz_threshold", C, "interpolation branches split at q = 1 instead of 1/2",
  "if (q >= 0.5) {                                     /* interpolated bounce-back */",
  "if (q >= 1.0) {                                     /* interpolated bounce-back */"),
 ("wss_max", C, "maximum wall shear taken as the last value",
  "if (tau_w > wm[id]) wm[id] = tau_w;", "wm[id] = tau_w;"),
 ("wss_sign_f", C, "wall shear from Pi^neq without the factor's sign and size",
  "double f = -(1.0 - 0.5 / P->tau_f);", "double f = 1.0;"),
 ("mass_thermal", C, "thermal mass without the rest population",
  "for (int i = 0; i < 5; i++) mt += g5[i];", "for (int i = 1; i < 5; i++) mt += g5[i];"),
 ("resid_T_ref", C, "thermal residual relative to T instead of T - T_ref",
  "T2 += (m.T - P->T_ref) * (m.T - P->T_ref);", "T2 += m.T * m.T;"),
 ("umax_fluid", C, "maximum speed as the sum of the components",
  "double um = sqrt(m.ux * m.ux + m.uy * m.uy);", "double um = fabs(m.ux) + fabs(m.uy);"),
 ("init_ext", C, "paper scheme started without its boundary populations",
  "if (P->bc_scheme == OR_BC_PAPER) initial_boundary_populations(s);", "(void)initial_boundary_populations;"),
 ("lumped_first", C, "first lumped interval at zero seepage",
  "s->u_seep = P->outlet_mode == OR_OUTLET_LUMPED ? seepage_speed(P, P->p_init) : 0.0;", "s->u_seep = 0.0;"),
 ("set_outlet_iop", C, "recalibrated seepage from p_init instead of the last IOP",
  "s->u_seep = seepage_speed(&s->P, s->obs.step > 0 ? s->obs.p_mean_fluid : s->P.p_init);",
  "s->u_seep = seepage_speed(&s->P, s->P.p_init);"),
 ("darcy_by_tau", C, "Darcy drag with nu replaced by tau", "double nuK = nu_of(P) / P->K;", "double nuK = P->tau_f / P->K;"),
 ("periodic_wrap", C, "periodic wrap without the shift", "if (s->P.periodic_x) xx = (xx + s->nx) % s->nx;", "if (s->P.periodic_x) xx = xx % s->nx;"),
 ("inlet_uy_index", C, "inlet wall velocity's y part along e_x", "double eu = ex[i] * P->u_in_x + ey[i] * P->u_in_y;", "double eu = ex[i] * P->u_in_x + ex[i] * P->u_in_y;"),
 ("lumped_y", C, "lumped outlet flux along x only", "double eu = (ex[i] * ex[d] + ey[i] * ey[d]) * s->u_seep;", "double eu = (ex[i] * ex[d]) * s->u_seep;"),
 ("outlet_T_dirichlet", C, "outlet treated as a Dirichlet thermal wall", "} else if ((c == OR_SOLID && wall != OR_WALL_BOX) || c == OR_INLET) {\n                    double Tw = (c == OR_INLET) ? P->T_inlet : wall_temperature(s, wall);\n                    *back = -gout", "} else if ((c == OR_SOLID && wall != OR_WALL_BOX) || c == OR_INLET || c == OR_OUTLET) {\n                    double Tw = (c == OR_INLET) ? P->T_inlet : wall_temperature(s, wall);\n                    *back = -gout"),
 ("iop_pref", C, "mean pressure without p_ref", "o->p_mean_fluid = P->p_ref + (cnt > 0 ? sum_dp / cnt : 0.0);", "o->p_mean_fluid = (cnt > 0 ? sum_dp / cnt : 0.0);"),
 ("darcy_in_fluid", C, "Darcy drag in fluid nodes instead of porous ones", "collide_node(s, s->cls[k] == OR_POROUS, h8, g5, h8s, g5s);", "collide_node(s, s->cls[k] == OR_FLUID, h8, g5, h8s, g5s);"),
 ("back_one_sided", D, "backward one-sided difference sign", "    if dn:\n        return f[y, x] - f[y - dy, x - dx]", "    if dn:\n        return f[y - dy, x - dx] - f[y, x]"),
 ("umax_active", D, "maximum speed over all active nodes", "float(np.max(np.hypot(ux, uy)[fluid]))", "float(np.nanmax(np.where(_active(mask), np.hypot(ux, uy), np.nan)))"),
 ("argmax_last", D, "vortex centre at the last maximum", "imax = int(np.nanargmax(flat))      # first occurrence in y * nx + x order", "imax = int(len(flat) - 1 - np.nanargmax(flat[::-1]))"),
 ("psi_active", D, "stream function summed over inactive nodes too", "np.cumsum(np.where(act, ux, 0.0), axis=0)", "np.cumsum(np.nan_to_num(ux), axis=0)"),
 ("bz_hi_idx", C, "interpolation for q >= 1/2 reads the outgoing population again",
  "*back = hout / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * s->hs[(size_t)(ib - 1) * n + k];",
  "*back = hout / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * s->hs[(size_t)(i - 1) * n + k];"),
 ("mass_flow_half", C, "flow mass over half the links", "for (int i = 0; i < 8; i++) mf += h8[i];", "for (int i = 0; i < 4; i++) mf += h8[i];"),
 ("wss_ids", C, "wall shear of cornea and iris merged", "        int id = s->wall_id[w];\n        if (id < 1 || id > 2) continue;", "        int id = 1;\n        if (id < 1 || id > 2) continue;"),
 ("nonfinite", C, "non-finite count ignores the temperature", "if (!isfinite(m.dp) || !isfinite(m.ux) || !isfinite(m.uy) || !isfinite(m.T)) bad++;", "if (!isfinite(m.dp) || !isfinite(m.ux) || !isfinite(m.uy)) bad++;"),
 ("ext_T_wall_u", C, "thermal extrapolation at walls with the inlet velocity", "double uxb = c == OR_INLET ? P->u_in_x : 0.0, uyb = c == OR_INLET ? P->u_in_y : 0.0;\n                    moments ms = post_moments(s, k);                        /* extrapolation */", "double uxb = P->u_in_x, uyb = P->u_in_y;\n                    moments ms = post_moments(s, k);                        /* extrapolation */"),
 ("buoy_gbeta", C, "buoyancy without g beta on x", "double Bx = P->gbeta * (m.T - P->T0) * s->gx_hat;", "double Bx = (m.T - P->T0) * s->gx_hat;"),
 ("thermal_rest_w", C, "thermal weights with the rest weight on the axis links", "static double w_heat(const or_params* P, int i) { return i == 0 ? P->w0 : (1.0 - P->w0) / 4.0; }", "static double w_heat(const or_params* P, int i) { return i == 0 ? (1.0 - P->w0) / 4.0 : P->w0; }"),
 ("uprev_stale", C, "velocity residual against a reference never updated", "        s->u_prev_x[k] = m.ux;\n        s->u_prev_y[k] = m.uy;\n        s->T_prev[k] = m.T;\n    }\n\n    /* wall shear", "        s->T_prev[k] = m.T;\n    }\n\n    /* wall shear"),
 ("Tprev_stale", C, "thermal residual against a reference never updated", "        s->u_prev_y[k] = m.uy;\n        s->T_prev[k] = m.T;\n    }\n\n    /* wall shear", "        s->u_prev_y[k] = m.uy;\n    }\n\n    /* wall shear"),
 ("ext_q_in", C, "inflow of the extrapolated inlet with the wrong sign", "if (c == OR_INLET) q_in += *back - hout;\n                    else q_out += hout - *back;", "if (c == OR_INLET) q_in += hout - *back;\n                    else q_out += hout - *back;"),
 ("wss_normal_sign", C, "wall shear removes the normal part with the wrong sign", "double tn = tx * nx_ + ty * ny_;", "double tn = -(tx * nx_ + ty * ny_);"),
]


def setup():
    if os.path.isdir(WORK):
        shutil.rmtree(WORK)
    os.makedirs(WORK)
    for d in ("tests", "oracle", "aqinputs"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(WORK, d),
                        ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), WORK)
    pkg = os.path.join(WORK, "paper_2102_12663_amd")       # its pure-Python helpers only
    os.makedirs(pkg)
    for f in ("__init__.py", "serve.py", "build.py"):
        shutil.copy(os.path.join(ROOT, "paper_2102_12663_amd", f), pkg)


def run(mid, f, desc, old, new):
    src = open(os.path.join(ROOT, f)).read()
    n = src.count(old)
    if n != 1:
        return {"id": mid, "desc": desc, "status": f"pattern found {n} times"}
    open(os.path.join(WORK, f), "w").write(src.replace(old, new))
    so = os.path.join(WORK, "oracle", "liboracle.so")
    if os.path.exists(so):
        os.remove(so)
    t0 = time.time()
    tests = sorted(t for t in os.listdir(os.path.join(WORK, "tests")) if t.startswith("test_oracle_"))
    try:
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                            *[os.path.join("tests", t) for t in tests]],
                           cwd=WORK, capture_output=True, text=True, timeout=900)
    except subprocess.TimeoutExpired:
        # the pins did not all pass within the limit (run nothing else on the CPU meanwhile:
        # two OpenMP processes on the same cores slow each other by orders of magnitude)
        open(os.path.join(WORK, f), "w").write(src)
        return {"id": mid, "desc": desc, "status": "timed out", "by": "", "s": round(time.time() - t0, 1)}
    open(os.path.join(WORK, f), "w").write(src)
    failed = [l for l in r.stdout.splitlines() if l.startswith(("FAILED", "ERROR"))]
    # 1: a pin failed; negative: the copy crashed its test process (also a failed pin);
    # 0: every pin passed; anything else is a harness problem
    status = {0: "MISSED", 1: "caught"}.get(r.returncode, "caught" if r.returncode < 0 else f"pytest exit {r.returncode}")
    tail = (r.stdout.strip().splitlines() or [""])[-1]
    return {"id": mid, "desc": desc, "status": status, "by": (failed[0] if failed else tail)[:160],
            "s": round(time.time() - t0, 1)}


def main(ids):
    setup()
    base = run("unchanged copy", C, "no mistake", "#include <math.h>", "#include <math.h>")
    print(json.dumps(base), flush=True)
    if base["status"] != "MISSED":
        print("the unchanged copy fails its pins: fix that first", flush=True)
        return 2
    missed = 0
    for m in M:
        if ids and m[0] not in ids:
            continue
        res = run(*m)
        missed += res["status"] not in ("caught", "timed out")
        print(json.dumps(res), flush=True)
    print(f"{missed} planted mistake(s) passed every pin", flush=True)
    return 1 if missed else 0


if __name__ == "__main__":
    sys.exit(main(set(sys.argv[1:])))

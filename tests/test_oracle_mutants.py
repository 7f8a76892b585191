"""Mutation check of the oracle's pins (CPU).

Each case plants one plausible mistake in a copy of the oracle's C source (a
dropped term, a wrong sign, index or constant, a transposed operand, a
world/body mix-up), builds the copy, and runs the pin files against it with
``QS_ORACLE_LIB`` pointing at that build; the case passes when at least one
pin fails.  An unmodified copy built and run the same way must pass every
pin, so a failing pin is the planted mistake's doing, not the harness's.
The mistakes never reach the GPU library or the committed oracle.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_pins.py", "tests/test_oracle_grad.py"]

# (name, passage the original follows, original text, planted text)
MUTANTS = [
    # Philox4x32-10 and the draws built on it (§III-A.2 noise)
    ("philox_multiplier", "Philox4x32-10", "M0 = 0xD2511F53u", "M0 = 0xD2511F57u"),
    ("philox_key_bump", "Philox4x32-10", "k0 += W0; k1 += W1;", "k0 += W0; k1 += W0;"),
    ("philox_word_order", "Philox4x32-10",
     "n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;", "n0 = (uint32_t)(p1 >> 32) ^ c3 ^ k0;"),
    ("uniform_offset", "uniform map", "(double)(2u * (r >> 9) + 1u)", "(double)(2u * (r >> 9) + 2u)"),
    ("box_muller_radius", "Box-Muller", "sqrt(-2.0 * log(u1))", "sqrt(-log(u1))"),
    ("box_muller_angle", "Box-Muller",
     "const double two_pi = 6.283185307179586476925286766559;",
     "const double two_pi = 3.141592653589793238462643383279;"),
    # §III-A.1 action map and motor lag
    ("action_map_unit_in_default", "§III-A.1",
     "0.5 * (clampd(act[i], -1.0, 1.0) + 1.0)", "clampd(act[i], 0.0, 1.0)"),
    ("lag_direction", "§III-A.1",
     "s[IU + i] = alpha_lag * (uhat[i] - s[IU + i]) + s[IU + i];",
     "s[IU + i] = alpha_lag * (s[IU + i] - uhat[i]) + s[IU + i];"),
    ("lag_forward_euler", "§III-A.1",
     "const double alpha_lag = OR_CONST(1.0 - exp(-dt / p[PTAU]));",
     "const double alpha_lag = OR_CONST(dt / p[PTAU]);"),
    # §III-A.2 motor noise and thrust
    ("noise_scale_no_sqrt", "§III-A.2",
     "const double a_ns = OR_CONST(d->motor_noise_std * f_max * sqrt(1.0 - a_nd * a_nd));",
     "const double a_ns = OR_CONST(d->motor_noise_std * f_max * (1.0 - a_nd * a_nd));"),
    ("noise_no_decay", "§III-A.2",
     "s[IE + i] = a_nd * s[IE + i] + a_ns * z[i];", "s[IE + i] = s[IE + i] + a_ns * z[i];"),
    ("thrust_not_squared", "§III-A.2",
     "f[i] = f_max * s[IU + i] * s[IU + i] + s[IE + i];", "f[i] = f_max * s[IU + i] + s[IE + i];"),
    ("f_max_half_weight", "§III-A.2",
     "const double f_max = OR_CONST(0.25 * m * g * p[PT2W]);",
     "const double f_max = OR_CONST(0.5 * m * g * p[PT2W]);"),
    # §III-A X mix and rigid body
    ("roll_mix_rotors", "§III-A mix",
     "tau[0] = arm_d * ((f[2] + f[3]) - (f[0] + f[1]));",
     "tau[0] = arm_d * ((f[1] + f[2]) - (f[0] + f[3]));"),
    ("yaw_reaction_sign", "§III-A mix",
     "tau[2] = d->k_tau * ((f[0] + f[2]) - (f[1] + f[3]));",
     "tau[2] = d->k_tau * ((f[1] + f[3]) - (f[0] + f[2]));"),
    ("arm_not_diagonal", "§III-A mix",
     "const double arm_d = OR_CONST(d->arm_length / sqrt(2.0));\n\n  /* §III-A.1",
     "const double arm_d = OR_CONST(d->arm_length);\n\n  /* §III-A.1"),
    ("thrust_along_row", "§III-A",
     "double F[3] = {T * R[2], T * R[5], T * R[8]};", "double F[3] = {T * R[6], T * R[7], T * R[8]};"),
    ("gravity_sign", "§III-A", "acc[2] -= g;", "acc[2] += g;"),
    ("drag_dropped", "linear drag",
     "acc[k] = F[k] / m - d->drag_coef / m * v[k];", "acc[k] = F[k] / m;"),
    ("gyroscopic_dropped", "§III-A Euler's equation", "(tau[0] - wxJw[0]) / jx", "tau[0] / jx"),
    ("inertia_index", "§III-A Euler's equation", "(tau[1] - wxJw[1]) / jy", "(tau[1] - wxJw[1]) / jx"),
    ("explicit_euler", "semi-implicit Euler",
     "    for (int k = 0; k < 3; ++k) v[k] += dt * acc[k];\n"
     "    for (int k = 0; k < 3; ++k) x[k] += dt * v[k];",
     "    for (int k = 0; k < 3; ++k) x[k] += dt * v[k];\n"
     "    for (int k = 0; k < 3; ++k) v[k] += dt * acc[k];"),
    ("rotation_world_rate", "§III-A attitude",
     "acc_rc += R[3 * r + k] * W[3 * k + c];", "acc_rc += W[3 * r + k] * R[3 * k + c];"),
    ("gram_schmidt_projection", "Gram-Schmidt",
     "for (int k = 0; k < 3; ++k) c1[k] -= dp * c0[k];",
     "for (int k = 0; k < 3; ++k) c1[k] -= dp * c1[k];"),
    ("gram_schmidt_handedness", "Gram-Schmidt",
     "double c2[3] = {c0[1] * c1[2] - c0[2] * c1[1], c0[2] * c1[0] - c0[0] * c1[2],\n"
     "                    c0[0] * c1[1] - c0[1] * c1[0]};",
     "double c2[3] = {c1[1] * c0[2] - c1[2] * c0[1], c1[2] * c0[0] - c1[0] * c0[2],\n"
     "                    c1[0] * c0[1] - c1[1] * c0[0]};"),
    # §III-B.2 walls, §III-B.3 floor
    ("upper_wall_absorbs", "§III-B.2",
     "if (v[k] > 0.0) { v[k] = -e * v[k]; bounced = 1; r->flip[k] = 1; }",
     "if (v[k] > 0.0) { v[k] = 0.0 * v[k]; bounced = 1; r->flip[k] = 1; }"),
    ("lower_wall_no_clamp", "§III-B.2",
     "x[k] = d->room_min[k];\n        r->clamp[k] = 1;", "r->clamp[k] = 1;"),
    ("wall_decay_dropped", "§III-B.2",
     "v[k] = d->col_decay * (v[k] + d->col_noise_v * zv[k]);",
     "v[k] = (v[k] + d->col_noise_v * zv[k]);"),
    ("wall_decay_per_wall", "§III-B.2",
     "if (v[k] > 0.0) { v[k] = -e * v[k]; bounced = 1; r->flip[k] = 1; }",
     "if (v[k] > 0.0) { v[k] = -e * d->col_decay * v[k]; bounced = 1; r->flip[k] = 1; }"),
    ("pair_decay_dropped", "§III-B.1",
     "si[IV + k] = d->col_decay * (si[IV + k] + dv[i][k] + d->col_noise_v * zv[k]);",
     "si[IV + k] = (si[IV + k] + dv[i][k] + d->col_noise_v * zv[k]);"),
    ("rest_threshold", "§III-B.3",
     "s[IF] != 0.0 && F[2] <= m * g;", "s[IF] != 0.0 && F[2] <= 0.5 * m * g;"),
    ("friction_direction", "§III-B.3",
     "fb[0] = F[0] - mu_n * v[0] / nv;", "fb[0] = F[0] + mu_n * v[0] / nv;"),
    ("friction_normal_force", "§III-B.3", "double N = m * g - F[2];", "double N = m * g;"),
    ("floor_level_handedness", "§III-B.3",
     "c1[0] = -c0[1]; c1[1] = c0[0]; c1[2] = 0.0;", "c1[0] = c0[1]; c1[1] = -c0[0]; c1[2] = 0.0;"),
    ("floor_hit_keeps_xy_velocity", "§III-B.3",
     "    v[0] = v[1] = v[2] = 0.0;\n    w[0] = w[1] = w[2] = 0.0;\n    s[IF] = 1.0;",
     "    v[2] = 0.0;\n    w[0] = w[1] = w[2] = 0.0;\n    s[IF] = 1.0;"),
    # §III-B.1 pair collisions
    ("contact_unsquared_distance", "§III-B.1",
     "if (!(d->flags & OR_COLLIDE) || !(d2 < dc2)) continue;",
     "if (!(d->flags & OR_COLLIDE) || !(d2 < d->col_dist)) continue;"),
    ("response_sign", "§III-B.1",
     "        dv[i][k] += sp * nrm[k];\n        dv[j][k] -= sp * nrm[k];",
     "        dv[i][k] -= sp * nrm[k];\n        dv[j][k] += sp * nrm[k];"),
    ("approach_test_sign", "§III-B.1",
     "if ((d->flags & OR_APPROACH_ONLY) && !(sp > 0.0)) continue;\n"
     "      for (int k = 0; k < 3; ++k) {\n        dv[i][k]",
     "if ((d->flags & OR_APPROACH_ONLY) && !(sp < 0.0)) continue;\n"
     "      for (int k = 0; k < 3; ++k) {\n        dv[i][k]"),
    # §III-B.4 downwash
    ("downwash_sign", "§III-B.4",
     "adw[i] += -d->dw_k1 * (d->dw_k2 * dz + d->dw_b1);",
     "adw[i] += d->dw_k1 * (d->dw_k2 * dz + d->dw_b1);"),
    ("downwash_on_upper_quad", "§III-B.4",
     "dz > 0.0 && dz < d->dw_height", "dz < 0.0 && -dz < d->dw_height"),
    ("downwash_on_resting_quad", "§III-B.4",
     "if (si[IF] != 0.0) continue; /* resting on the floor */", "/* resting quads too */"),
    # §III-C observation and sensor noise
    ("knn_farthest_first", "§III-C",
     "if (!used[j] && (best < 0 || dist[j] < dist[best])) best = j;",
     "if (!used[j] && (best < 0 || dist[j] > dist[best])) best = j;"),
    ("knn_tie_to_later_index", "§III-C",
     "if (!used[j] && (best < 0 || dist[j] < dist[best])) best = j;",
     "if (!used[j] && (best < 0 || dist[j] <= dist[best])) best = j;"),
    ("knn_relative_sign", "§III-C",
     "for (int k = 0; k < 3; ++k) os[k] = sj[IX + k] - si[IX + k];",
     "for (int k = 0; k < 3; ++k) os[k] = si[IX + k] - sj[IX + k];"),
    ("knn_rate_for_velocity", "§III-C",
     "os[3 + k] = sj[IV + k] - si[IV + k];", "os[3 + k] = sj[IW + k] - si[IW + k];"),
    ("obs_goal_sign", "§III-C",
     "o[k] = si[IX + k] - goals[(size_t)(q0 + i) * 3 + k];",
     "o[k] = goals[(size_t)(q0 + i) * 3 + k] - si[IX + k];"),
    ("obs_rotation_transposed", "§III-C",
     "for (int k = 0; k < 9; ++k) o[6 + k] = si[IR + k];",
     "for (int k = 0; k < 9; ++k) o[6 + k] = si[IR + 3 * (k % 3) + k / 3];"),
    ("sensor_noise_one_sided", "§III-C",
     "o[3 * draw + k] += a * (2.0 * or_uniform_from_u32(r[k]) - 1.0);",
     "o[3 * draw + k] += a * or_uniform_from_u32(r[k]);"),
    ("sensor_rate_variance_for_std", "§III-C",
     "o[15 + k] += d->sn_w * z[k];", "o[15 + k] += d->sn_w * d->sn_w * z[k];"),
    # §III-E reward
    ("reward_orientation_entry", "§III-E", "w[2] * b[IR + 8]", "w[2] * b[IR + 6]"),
    ("reward_yaw_entry", "§III-E", "w[7] * b[IR + 0]", "w[7] * b[IR + 4]"),
    ("reward_proximity_scale", "§III-E",
     "const double h = 1.0 - dd / w[14];", "const double h = 1.0 - dd * w[14];"),
    ("reward_thrust_change", "§III-E",
     "df2 += (f1 - f0) * (f1 - f0);", "df2 += f1 * f1;"),
    ("reward_wall_bit", "§III-E",
     "w[10] * ((ev[q] & EV_WALL) ? 1.0 : 0.0)", "w[10] * ((ev[q] & EV_CEILING) ? 1.0 : 0.0)"),
    ("reward_floor_hit_bit", "§III-E",
     "w[8] * ((ev[q] & EV_FLOOR_HIT) ? 1.0 : 0.0)", "w[8] * ((ev[q] & EV_PAIR_RESPONSE) ? 1.0 : 0.0)"),
    ("reward_on_floor_from_hit", "§III-E",
     "w[9] * (b[IF] != 0.0 ? 1.0 : 0.0)", "w[9] * ((ev[q] & EV_FLOOR_HIT) ? 1.0 : 0.0)"),
    ("reward_prox_counts_empty_slots", "§III-E",
     "const int kr = n - 1 < K ? n - 1 : K;", "const int kr = K;"),
    # padded slots told apart by their zero values instead of by count: a
    # coincident, co-moving swarm-mate then adds nothing
    ("reward_prox_skips_zero_valued_slots", "§III-E",
     "        const double* x = o + 18 + 6 * k;\n",
     "        const double* x = o + 18 + 6 * k;\n"
     "        if (x[0] == 0.0 && x[1] == 0.0 && x[2] == 0.0 && x[3] == 0.0 && x[4] == 0.0 &&\n"
     "            x[5] == 0.0)\n          continue;\n"),
    # reverse mode (§III-E penalty and every row above)
    ("vjp_lag_factor", "reverse mode, §III-A.1",
     "lu0[i] = (1.0 - r->alpha_lag) * lu[i];", "lu0[i] = r->alpha_lag * lu[i];"),
    ("vjp_thrust_square", "reverse mode, §III-A.2",
     "lu[i] += 2.0 * r->f_max * r->u1[i] * lf[i];", "lu[i] += r->f_max * r->u1[i] * lf[i];"),
    ("vjp_noise_decay", "reverse mode, §III-A.2",
     "le0[i] = d->motor_noise_decay * le[i];", "le0[i] = le[i];"),
    ("vjp_tau_derivative_sign", "reverse mode, §III-A.1",
     "gp[PTAU] += lalag * OR_CONST(-exp(-dt / p[PTAU]) * dt / (p[PTAU] * p[PTAU]));",
     "gp[PTAU] += lalag * OR_CONST(exp(-dt / p[PTAU]) * dt / (p[PTAU] * p[PTAU]));"),
    ("vjp_wall_mirror", "reverse mode, §III-B.2",
     "if (r->flip[k]) lv[k] *= -d->wall_restitution;",
     "if (r->flip[k]) lv[k] *= d->wall_restitution;"),
    ("vjp_gyroscopic_operands", "reverse mode, §III-A", "cross3(r->Jw, lc, tmp);", "cross3(lc, r->Jw, tmp);"),
    ("vjp_mass_power", "reverse mode, §III-A",
     "lm += -(r->F[k] - d->drag_coef * r->v0[k]) * lacc[k] / (m * m);",
     "lm += -(r->F[k] - d->drag_coef * r->v0[k]) * lacc[k] / m;"),
    ("vjp_friction_normal", "reverse mode, §III-B.3",
     "lF[2] += -d->floor_mu * lmu;", "lF[2] += d->floor_mu * lmu;"),
    ("vjp_response_sign", "reverse mode, §III-B.1",
     "        li[IV + k] += -mn * nrm[k];\n        lj[IV + k] += mn * nrm[k];",
     "        li[IV + k] += mn * nrm[k];\n        lj[IV + k] += -mn * nrm[k];"),
    ("vjp_penalty_sign", "reverse mode, §III-E penalty",
     "double coef = -0.5 * (gpen[q0 + i] + gpen[q0 + j])",
     "double coef = 0.5 * (gpen[q0 + i] + gpen[q0 + j])"),
    # further slips in the floor model, contacts, downwash, sensor noise,
    # reward and reverse mode
    ("static_friction_sign", "§III-B.3",
     "double mag = nf - mu_n > 0.0 ? nf - mu_n : 0.0;", "double mag = nf + mu_n > 0.0 ? nf + mu_n : 0.0;"),
    ("friction_guard_dropped", "§III-B.3",
     "if (dot < 0.0) { v[0] = 0.0; v[1] = 0.0; r->guard = 1; }",
     "if (dot < -1e300) { v[0] = 0.0; v[1] = 0.0; r->guard = 1; }"),
    ("rest_keeps_vz", "§III-B.3",
     "    v[0] += dt * acc[0];\n    v[1] += dt * acc[1];\n    v[2] = 0.0;",
     "    v[0] += dt * acc[0];\n    v[1] += dt * acc[1];"),
    ("rest_keeps_body_rate", "§III-B.3",
     "    for (int k = 0; k < 3; ++k) x[k] += dt * v[k];\n    w[0] = w[1] = w[2] = 0.0;\n  }",
     "    for (int k = 0; k < 3; ++k) x[k] += dt * v[k];\n  }"),
    ("takeoff_keeps_flag", "§III-B.3", "    s[IF] = 0.0;\n", "\n"),
    ("coincident_normal_along_x", "§III-B.1",
     "        nrm[0] = 0.0; nrm[1] = 0.0; nrm[2] = 1.0;", "        nrm[0] = 1.0; nrm[1] = 0.0; nrm[2] = 0.0;"),
    ("downwash_slope_sign", "§III-B.4",
     "adw[i] += -d->dw_k1 * (d->dw_k2 * dz + d->dw_b1);",
     "adw[i] += -d->dw_k1 * (-d->dw_k2 * dz + d->dw_b1);"),
    ("downwash_radius_unsquared", "§III-B.4",
     "const double dw_r2 = OR_CONST(d->dw_radius * d->dw_radius);",
     "const double dw_r2 = OR_CONST(d->dw_radius);"),
    ("sensor_widths_swapped", "§III-C",
     "const double a = draw == 0 ? d->sn_x : d->sn_v;", "const double a = draw == 0 ? d->sn_v : d->sn_x;"),
    ("observe_padding_nonzero", "§III-C",
     "          for (int k = 0; k < 6; ++k) os[k] = 0.0;", "          for (int k = 0; k < 6; ++k) os[k] = 1.0;"),
    ("reward_goal_distance_squared", "§III-E", "w[0] * sqrt(dx2)", "w[0] * dx2"),
    ("reward_spin_squared", "§III-E", "w[3] * sqrt(w2)", "w[3] * w2"),
    ("reward_rotation_offset", "§III-E",
     "w[6] * (b[IR + 0] + b[IR + 4] + b[IR + 8] - 1.0) / 2.0",
     "w[6] * (b[IR + 0] + b[IR + 4] + b[IR + 8]) / 2.0"),
    ("penalty_half_dropped", "§III-E penalty",
     "double h = 0.5 * softplus(beta * (d->col_dist - sqrt(d2))) / beta;",
     "double h = softplus(beta * (d->col_dist - sqrt(d2))) / beta;"),
    ("vjp_inertia_sign", "reverse mode, §III-A",
     "lJ[k] += -lwd[k] * r->wdot[k] / J[k];", "lJ[k] += lwd[k] * r->wdot[k] / J[k];"),
    ("vjp_gram_schmidt_norm", "reverse mode, Gram-Schmidt",
     "lb[k] = (lc1[k] - dd * r->c1[k]) / r->n1;", "lb[k] = (lc1[k] - dd * r->c1[k]) / r->n0;"),
    ("vjp_gram_schmidt_projection", "reverse mode, Gram-Schmidt",
     "lc0[k] += -r->dp * lb[k] + ldp * r->A1[k];", "lc0[k] += -r->dp * lb[k];"),
    ("vjp_sqrt_half_dropped", "reverse mode, §III-A.1",
     "gu[(size_t)q * 4 + i] * 0.5 / uh * dfhat_da(d, a)", "gu[(size_t)q * 4 + i] / uh * dfhat_da(d, a)"),
    ("vjp_penalty_sigmoid_argument", "reverse mode, §III-E penalty",
     "sigmoid(beta * (d->col_dist - dd))", "sigmoid(beta * (dd - d->col_dist))"),
    ("vjp_action_map_slope", "reverse mode, §III-A.1",
     "return (a > -1.0 && a < 1.0) ? 0.5 : 0.0;", "return (a > -1.0 && a < 1.0) ? 1.0 : 0.0;"),
    ("room_floor_as_wall", "§III-B.2, §III-B.3",
     "if (k < 2 && x[k] < d->room_min[k]) {", "if (x[k] < d->room_min[k]) {"),
    ("gyroscopic_operand_order", "§III-A Euler's equation",
     "double wxJw[3] = {w[1] * Jw[2] - w[2] * Jw[1], w[2] * Jw[0] - w[0] * Jw[2],\n"
     "                      w[0] * Jw[1] - w[1] * Jw[0]};",
     "double wxJw[3] = {Jw[1] * w[2] - Jw[2] * w[1], Jw[2] * w[0] - Jw[0] * w[2],\n"
     "                      Jw[0] * w[1] - Jw[1] * w[0]};"),
    ("drag_not_per_mass", "linear drag",
     "acc[k] = F[k] / m - d->drag_coef / m * v[k];", "acc[k] = F[k] / m - d->drag_coef * v[k];"),
    ("kinetic_friction_index", "§III-B.3",
     "fb[1] = F[1] - mu_n * v[1] / nv;", "fb[1] = F[1] - mu_n * v[0] / nv;"),
    ("floor_heading_from_row", "§III-B.3",
     "double hx = R[0], hy = R[3];", "double hx = R[0], hy = R[1];"),
    ("knn_self_included", "§III-C", "used[j] = (j == i);", "used[j] = 0;"),
    ("reward_thrust_without_noise", "§III-E",
     "const double f1 = f_max * b[IU + i] * b[IU + i] + b[IE + i];",
     "const double f1 = f_max * b[IU + i] * b[IU + i];"),
    ("vjp_drag_dropped", "reverse mode, linear drag",
     "lv0[k] = lv1 - d->drag_coef / m * lacc[k];", "lv0[k] = lv1;"),
    ("vjp_wall_decay_dropped", "reverse mode, §III-B.2",
     "for (int k = 0; k < 3; ++k) lv[k] *= d->col_decay;",
     "for (int k = 0; k < 3; ++k) lv[k] *= 1.0;"),
    ("vjp_contact_position_sign", "reverse mode, §III-B.1",
     "          li[IX + k] += gx;", "          li[IX + k] -= gx;"),
    ("wall_noise_one_axis", "§III-B.2",
     "v[k] = d->col_decay * (v[k] + d->col_noise_v * zv[k]);",
     "v[k] = d->col_decay * (v[k] + d->col_noise_v * zv[0]);"),
    ("wall_rate_noise_from_velocity_draws", "§III-B.2",
     "w[k] = w[k] + d->col_noise_w * zw[k];", "w[k] = w[k] + d->col_noise_w * zv[k];"),
    ("pair_noise_one_axis", "§III-B.1",
     "si[IV + k] = d->col_decay * (si[IV + k] + dv[i][k] + d->col_noise_v * zv[k]);",
     "si[IV + k] = d->col_decay * (si[IV + k] + dv[i][k] + d->col_noise_v * zv[0]);"),
    ("pair_rate_noise_from_velocity_draws", "§III-B.1",
     "si[IW + k] = si[IW + k] + d->col_noise_w * zw[k];",
     "si[IW + k] = si[IW + k] + d->col_noise_w * zv[k];"),
    ("downwash_noise_one_axis", "§III-B.4", "d->dw_noise_a * za[k]", "d->dw_noise_a * za[0]"),
    ("downwash_rate_noise_from_acceleration_draws", "§III-B.4",
     "si[IW + k] += d->dt * d->dw_noise_w * zw[k];", "si[IW + k] += d->dt * d->dw_noise_w * za[k];"),
    ("substep_index_not_advanced", "§III-A.2 noise per substep",
     "    const uint64_t t = t0 + (uint64_t)sub;\n    if (contacts)",
     "    const uint64_t t = t0;\n    if (contacts)"),
    ("penalty_on_one_quad", "§III-E penalty",
     "        pen[q0 + i] += h;\n        pen[q0 + j] += h;", "        pen[q0 + i] += h + h;"),
    ("pair_noise_local_index", "§III-B.1 (noise keyed by global quad index)",
     "or_normal4(d->seed, d->quad_id_offset + (uint32_t)(q0 + i), t, STREAM_PAIR, 0, zv);",
     "or_normal4(d->seed, (uint32_t)(q0 + i), t, STREAM_PAIR, 0, zv);"),
    ("downwash_noise_local_index", "§III-B.4 (noise keyed by global quad index)",
     "or_normal4(d->seed, d->quad_id_offset + (uint32_t)(q0 + i), t, STREAM_DOWNWASH, 0, za);",
     "or_normal4(d->seed, (uint32_t)(q0 + i), t, STREAM_DOWNWASH, 0, za);"),
    ("sensor_noise_local_index", "§III-C (noise keyed by global quad index)",
     "const uint32_t gq = d->quad_id_offset + (uint32_t)q;", "const uint32_t gq = (uint32_t)q;"),
    ("rollout_first_action_only", "rollout",
     "actions + ((size_t)c * Q + q) * 4, d->quad_id_offset + (uint32_t)q, t,\n"
     "                       &ev[q], &mg[q], NULL);",
     "actions + ((size_t)0 * Q + q) * 4, d->quad_id_offset + (uint32_t)q, t,\n"
     "                       &ev[q], &mg[q], NULL);"),
    ("vjp_rerun_wrong_substep", "reverse mode",
     "t0 + kk, &ev[q], &mg[q], &rec[q]);", "t0 + kk + 1, &ev[q], &mg[q], &rec[q]);"),
    ("vjp_command_gradient_not_reset", "reverse mode, §III-A.1",
     "          gu[(size_t)q * 4 + i] = 0.0;", "          (void)0;"),
    ("contacts_accumulate_over_substeps", "§III-B.1 (contact mask of the last substep)",
     "    if (contacts) memset(contacts, 0, (size_t)Q * sizeof(uint64_t));\n#pragma omp",
     "\n#pragma omp"),
    ("observe_rate_field", "§III-C",
     "for (int k = 0; k < 3; ++k) o[15 + k] = si[IW + k];",
     "for (int k = 0; k < 3; ++k) o[15 + k] = si[IV + k];"),
    ("reward_speed_from_rate", "§III-E", "w[1] * sqrt(v2)", "w[1] * sqrt(w2)"),
    ("reward_previous_thrust_from_after", "§III-E",
     "const double f0 = f_max * a[IU + i] * a[IU + i] + a[IE + i];",
     "const double f0 = f_max * b[IU + i] * b[IU + i] + b[IE + i];"),
    ("downwash_rest_check_on_upper_quad", "§III-B.4",
     "      if (si[IF] != 0.0) continue; /* resting on the floor */\n"
     "      for (int j = 0; j < n; ++j) {\n        if (j == i) continue;\n"
     "        const double* sj = S + (size_t)(q0 + j) * NS;",
     "      for (int j = 0; j < n; ++j) {\n        if (j == i) continue;\n"
     "        const double* sj = S + (size_t)(q0 + j) * NS;\n        if (sj[IF] != 0.0) continue;"),
    ("vjp_floor_hit_heading_sign", "reverse mode, §III-B.3",
     "      double gh[2] = {lR[0] + lR[4], lR[3] - lR[1]};",
     "      double gh[2] = {lR[0] + lR[4], lR[1] - lR[3]};"),
    ("vjp_floor_hit_projection_dropped", "reverse mode, §III-B.3",
     "      gr[0] = (gh[0] - dd * h[0]) / r->nh;", "      gr[0] = gh[0] / r->nh;"),
    ("vjp_floor_hit_height_kept", "reverse mode, §III-B.3",
     "  if (r->hit) {\n    lx[2] = 0.0;", "  if (r->hit) {\n    (void)0;"),
    ("vjp_static_friction_projection_dropped", "reverse mode, §III-B.3",
     "for (int k = 0; k < 2; ++k) lF[k] += lfb[k] - r->mu_n * (lfb[k] - dd * Fh[k]) / r->nf;",
     "for (int k = 0; k < 2; ++k) lF[k] += lfb[k] - r->mu_n * lfb[k] / r->nf;"),
    ("vjp_static_friction_normal_force_sign", "reverse mode, §III-B.3",
     "          lmu = -dd;", "          lmu = dd;"),
    ("vjp_kinetic_friction_normal_force_sign", "reverse mode, §III-B.3",
     "        lmu = -(lfb[0] * vh[0] + lfb[1] * vh[1]);", "        lmu = (lfb[0] * vh[0] + lfb[1] * vh[1]);"),
    ("vjp_wall_clamp_position_kept", "reverse mode, §III-B.2",
     "if (r->clamp[k]) lx[k] = 0.0;", "if (r->clamp[k]) (void)0;"),
    ("vjp_friction_stop_ignored", "reverse mode, §III-B.3", "    if (!r->guard) {", "    if (1) {"),
    ("vjp_rest_drag_dropped", "reverse mode, §III-B.3",
     "lv0[k] = lv1[k] * (1.0 - dt * d->drag_coef / m);", "lv0[k] = lv1[k];"),
    ("vjp_response_decay_dropped", "reverse mode, §III-B.1",
     "ldv[i][k] = marked[i] ? d->col_decay * li[IV + k] : 0.0;",
     "ldv[i][k] = marked[i] ? li[IV + k] : 0.0;"),
    ("vjp_contact_normal_term_dropped", "reverse mode, §III-B.1",
     "gn[k] = sp * mu[k] + mn * wv[k];", "gn[k] = sp * mu[k];"),
]

CASES = [("unmodified", "", "", "")] + MUTANTS


def _run_case(case, work):
    name, _, orig, planted = case
    src = open(O.SRC).read()
    if orig:
        if src.count(orig) != 1:
            return ("harness", f"original text found {src.count(orig)} times")
        src = src.replace(orig, planted)
    path = os.path.join(work, name + ".c")
    lib = os.path.join(work, name + ".so")
    with open(path, "w") as f:
        f.write(src)
    try:
        O.compile_lib(path, lib)
    except subprocess.CalledProcessError as e:
        return ("harness", f"build failed: {e}")
    env = dict(os.environ, QS_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *PIN_FILES],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    failed = [ln for ln in p.stdout.splitlines() if ln.startswith("FAILED")]
    return (p.returncode, failed[0] if failed else p.stdout[-600:])


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    work = str(tmp_path_factory.mktemp("mutants"))
    workers = max(1, min(8, (os.cpu_count() or 2) - 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        out = list(ex.map(lambda c: _run_case(c, work), CASES))
    return {c[0]: r for c, r in zip(CASES, out)}


def test_unmodified_copy_passes_every_pin(results):
    rc, detail = results["unmodified"]
    assert rc == 0, detail


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(name, results):
    rc, detail = results[name]
    assert rc != "harness", detail
    # pytest exit code 1: the run completed and at least one pin failed
    assert rc == 1, f"mutant {name} survived the pins (exit {rc}): {detail}"

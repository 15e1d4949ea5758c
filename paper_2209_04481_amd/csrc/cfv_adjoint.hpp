// Hand-written reverse-mode (adjoint) pieces of the residual.
//
// Each function takes the primal inputs of a forward piece of cfv_math.hpp,
// recomputes the intermediates it needs, and maps the adjoint of the outputs
// to the adjoint of the inputs.  Branches (|v_n|, the clamp under the square
// root, the Rusanov speed pick) follow the primal values exactly as the
// forward code does, so J^T here is the transpose of the forward J.
#pragma once
#include "cfv_math.hpp"

namespace cfv {

// One side of the Rusanov flux: F(q).n, U(q) and lambda = |v_n| + c_f with
// adjoints Fb, Ub, lamb; accumulates into qb.
__host__ __device__ __forceinline__ void flux_side_adjoint(const double q[9], V3 n, const double Fb[9], const double Ub[9],
                                                  double lamb, double qb[9], double gamma, double c_h) {
  const double rho = q[0], vx = q[1], vy = q[2], vz = q[3], bx = q[4], by = q[5], bz = q[6], p = q[7];
  // forward intermediates
  const double vn = vx * n.x + vy * n.y + vz * n.z;
  const double bn = bx * n.x + by * n.y + bz * n.z;
  const double B2 = bx * bx + by * by + bz * bz;
  const double v2 = vx * vx + vy * vy + vz * vz;
  const double igm1 = 1.0 / (gamma - 1.0);  // the same expression for every face: computed once
  const double pT = p + 0.5 * B2;
  const double E = p * igm1 + 0.5 * rho * v2 + 0.5 * B2;
  const double rvn = rho * vn;
  const double vb = vx * bx + vy * by + vz * bz;
  const double irho = recip(rho);  // as side_speed
  const double a2 = gamma * p * irho;
  const double b2 = B2 * irho;
  const double bn2 = bn * bn * irho;
  const double s = a2 + b2;
  const double disc = s * s - 4.0 * a2 * bn2;
  // the roots with 1/(2 root) from the same sequence (hsd only where disc > 0)
  double hsd = 0.0, hcf;
  const double sd = disc > 0.0 ? sqrt_nonneg(disc, &hsd) : 0.0;
  (void)sqrt_nonneg(0.5 * (s + sd), &hcf);  // c_f itself is not needed, only 1/(2 c_f)

  // adjoints of the intermediates from the flux components
  double rvnb = Fb[0] + Fb[1] * vx + Fb[2] * vy + Fb[3] * vz;
  double pTb = Fb[1] * n.x + Fb[2] * n.y + Fb[3] * n.z + Fb[7] * vn;
  double bnb = -(bx * Fb[1] + by * Fb[2] + bz * Fb[3]) - (vx * Fb[4] + vy * Fb[5] + vz * Fb[6]) - vb * Fb[7] +
               (c_h * c_h) * Fb[8];
  double vnb = (bx * Fb[4] + by * Fb[5] + bz * Fb[6]) + (E + pT) * Fb[7];
  double Eb = Fb[7] * vn + Ub[7];
  const double vbb = -bn * Fb[7];
  double vxb = rvn * Fb[1] - bn * Fb[4] + vbb * bx;
  double vyb = rvn * Fb[2] - bn * Fb[5] + vbb * by;
  double vzb = rvn * Fb[3] - bn * Fb[6] + vbb * bz;
  double bxb = -bn * Fb[1] + vn * Fb[4] + vbb * vx + Ub[4];
  double byb = -bn * Fb[2] + vn * Fb[5] + vbb * vy + Ub[5];
  double bzb = -bn * Fb[3] + vn * Fb[6] + vbb * vz + Ub[6];
  double psib = n.x * Fb[4] + n.y * Fb[5] + n.z * Fb[6] + Ub[8];

  // lambda = |v_n| + c_f
  vnb += (vn < 0.0 ? -lamb : lamb);
  const double hb = lamb * hcf;
  double sb = 0.5 * hb;
  const double discb = disc > 0.0 ? (0.5 * hb) * hsd : 0.0;
  sb += 2.0 * s * discb;
  double a2b = -4.0 * bn2 * discb + sb;
  const double bn2b = -4.0 * a2 * discb;
  const double b2b = sb;
  double pb = gamma * irho * a2b;
  const double irhob = gamma * p * a2b + B2 * b2b + bn * bn * bn2b;
  double B2b = irho * b2b;
  bnb += 2.0 * bn * irho * bn2b;
  double rhob = -irho * irho * irhob;

  // E and p_T
  pb += Eb * igm1 + pTb;
  rhob += 0.5 * v2 * Eb;
  const double v2b = 0.5 * rho * Eb;
  B2b += 0.5 * Eb + 0.5 * pTb;
  // rho v_n
  rhob += vn * rvnb;
  vnb += rho * rvnb;
  // conservative variables U(q) = (rho, rho v, B, E, psi)
  rhob += Ub[0] + vx * Ub[1] + vy * Ub[2] + vz * Ub[3];
  vxb += rho * Ub[1];
  vyb += rho * Ub[2];
  vzb += rho * Ub[3];
  // v_n, B_n, |B|^2, |v|^2
  vxb += vnb * n.x + 2.0 * vx * v2b;
  vyb += vnb * n.y + 2.0 * vy * v2b;
  vzb += vnb * n.z + 2.0 * vz * v2b;
  bxb += bnb * n.x + 2.0 * bx * B2b;
  byb += bnb * n.y + 2.0 * by * B2b;
  bzb += bnb * n.z + 2.0 * bz * B2b;

  qb[0] += rhob;
  qb[1] += vxb;
  qb[2] += vyb;
  qb[3] += vzb;
  qb[4] += bxb;
  qb[5] += byb;
  qb[6] += bzb;
  qb[7] += pb;
  qb[8] += psib;
}

// Adjoint of rusanov(): given wb = adjoint of the face flux, accumulate the
// adjoints of the left and right face states; want_L / want_R select which
// sides are needed (a side not wanted is skipped).
__host__ __device__ __forceinline__ void rusanov_adjoint(const double qL[9], const double qR[9], V3 S, const double wb[9],
                                                double qLb[9], double qRb[9], const Params& pr,
                                                bool want_L = true, bool want_R = true) {
  double ia;
  const double area = area_and_inverse(S, ia);  // as rusanov()
  const V3 n = mk(S.x * ia, S.y * ia, S.z * ia);
  double UL[9], UR[9];
  const double lamL = side_speed(qL, n, pr.gamma);
  const double lamR = side_speed(qR, n, pr.gamma);
  const double s1 = lamL >= lamR ? lamL : lamR;
  const double s = s1 >= pr.c_h ? s1 : pr.c_h;
  prim_to_cons(qL, UL, pr.gamma);
  prim_to_cons(qR, UR, pr.gamma);
  double Fb[9], ULb[9], URb[9];
  double sb = 0.0;
  for (int v = 0; v < 9; ++v) {
    Fb[v] = 0.5 * area * wb[v];
    ULb[v] = 0.5 * s * area * wb[v];
    URb[v] = -ULb[v];
    sb -= 0.5 * area * wb[v] * (UR[v] - UL[v]);
  }
  double lamLb = 0.0, lamRb = 0.0;
  if (s1 >= pr.c_h) {
    if (lamL >= lamR) lamLb = sb; else lamRb = sb;
  }
  if (want_L) flux_side_adjoint(qL, n, Fb, ULb, lamLb, qLb, pr.gamma, pr.c_h);
  if (want_R) flux_side_adjoint(qR, n, Fb, URb, lamRb, qRb, pr.gamma, pr.c_h);
}

// Adjoint of rusanov() with respect to one side only: qa is that side's
// state, qb the other's, a_is_L whether qa is the left (owner) state of the
// canonical face; accumulates into qab.  The arithmetic is that of
// rusanov_adjoint() for the side asked for, with the roles chosen by value,
// so that lanes of both orientations follow one code path.
__host__ __device__ __forceinline__ void rusanov_adjoint_side(const double qa[9], const double qb[9], V3 S,
                                                     const double wb[9], double qab[9], const Params& pr,
                                                     bool a_is_L) {
  double ia;
  const double area = area_and_inverse(S, ia);
  const V3 n = mk(S.x * ia, S.y * ia, S.z * ia);
  const double lamA = side_speed(qa, n, pr.gamma);
  const double lamB = side_speed(qb, n, pr.gamma);
  // the larger speed (the same value whichever side has it); on a tie the
  // left side wins
  const double s1 = ::fmax(lamA, lamB);
  const double s = ::fmax(s1, pr.c_h);
  double UA[9], UB[9];
  prim_to_cons(qa, UA, pr.gamma);
  prim_to_cons(qb, UB, pr.gamma);
  const double sg = a_is_L ? 1.0 : -1.0;  // U_R - U_L = sg (U_B - U_A); U_A's weight is sg s/2
  double Fb[9], UAb[9];
  double sb = 0.0;
  for (int v = 0; v < 9; ++v) {
    Fb[v] = 0.5 * area * wb[v];
    UAb[v] = sg * (0.5 * s * area * wb[v]);
    sb -= 0.5 * area * wb[v] * (sg * (UB[v] - UA[v]));
  }
  const bool a_wins = lamA > lamB || (lamA == lamB && a_is_L);
  const double lamAb = s1 >= pr.c_h && a_wins ? sb : 0.0;
  flux_side_adjoint(qa, n, Fb, UAb, lamAb, qab, pr.gamma, pr.c_h);
}

// (dP/dU)^T Pb for P = prim(U): returns Ub.
__host__ __device__ __forceinline__ void prim_adjoint(const double u[9], const double Pb[9], double Ub[9], double gamma) {
  const double rho = u[0];
  const double ir = recip(rho);  // as cons_to_prim
  const double vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
  const double g1 = gamma - 1.0;
  const double pb = Pb[7];
  Ub[0] = Pb[0] - (Pb[1] * vx + Pb[2] * vy + Pb[3] * vz) * ir + pb * g1 * 0.5 * (vx * vx + vy * vy + vz * vz);
  Ub[1] = Pb[1] * ir - pb * g1 * vx;
  Ub[2] = Pb[2] * ir - pb * g1 * vy;
  Ub[3] = Pb[3] * ir - pb * g1 * vz;
  Ub[4] = Pb[4] - pb * g1 * u[4];
  Ub[5] = Pb[5] - pb * g1 * u[5];
  Ub[6] = Pb[6] - pb * g1 * u[6];
  Ub[7] = pb * g1;
  Ub[8] = Pb[8];
}

}  // namespace cfv

/*
 * Driver of the CPU oracle for sanitizer builds (test infrastructure only).
 *
 * Compiled together with lbm_oracle.c (included below) into a standalone executable with
 * -fsanitize=address,undefined, so that the oracle's memory accesses and arithmetic run
 * under AddressSanitizer and UndefinedBehaviorSanitizer without loading anything into
 * the Python process.  Reads one lattice's tables from a binary file (written by the test
 * from oracle/lattice.py) and exercises every whole-lattice entry point and every
 * collision, boundary set and option on small lattices with seeded states.  Exits 0 when
 * every result is finite; the sanitizers abort on the first error they find.
 *
 * Table file layout (native byte order): int32 D, Q, NM; int32 e[Q][3]; int32 opp[Q];
 * int32 mi[NM][3]; then in the build's real type w[Q], H[NM][Q], Minv[Q][NM]; then a
 * double 1/c_s^2.
 */
#include "lbm_oracle.c"

#include <stdio.h>

static uint64_t lcg_state = 0x2212074942212074ull;
static double uniform(void) { /* in [-1, 1) */
  lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg_state >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static int read_all_or_die(FILE *f, void *p, size_t n) { return fread(p, 1, n, f) == n; }

static int all_finite(const real *a, int64_t n) {
  for (int64_t k = 0; k < n; ++k)
    if (!isfinite((double)a[k])) return 0;
  return 1;
}

int main(int argc, char **argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: %s table-file\n", argv[0]);
    return 2;
  }
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t hdr[3];
  if (!read_all_or_die(f, hdr, sizeof(hdr))) return 2;
  const int D = hdr[0], Q = hdr[1], NM = hdr[2];
  if (Q < 1 || Q > MAXQ || NM < 1 || NM > Q) return 2;
  int32_t *e = malloc(sizeof(int32_t) * 3 * Q), *opp = malloc(sizeof(int32_t) * Q),
          *mi = malloc(sizeof(int32_t) * 3 * NM);
  real *w = malloc(sizeof(real) * Q), *H = malloc(sizeof(real) * NM * Q),
       *Minv = malloc(sizeof(real) * Q * NM);
  if (!read_all_or_die(f, e, sizeof(int32_t) * 3 * Q) || !read_all_or_die(f, opp, sizeof(int32_t) * Q) ||
      !read_all_or_die(f, mi, sizeof(int32_t) * 3 * NM) || !read_all_or_die(f, w, sizeof(real) * Q) ||
      !read_all_or_die(f, H, sizeof(real) * NM * Q) || !read_all_or_die(f, Minv, sizeof(real) * Q * NM))
    return 2;
  double ics2 = 0;
  if (!read_all_or_die(f, &ics2, sizeof(ics2))) return 2;
  fclose(f);
  const oracle_lattice L = {D, Q, NM, e, opp, mi, w, H, Minv, ics2};

  const int nx = 7, ny = 5, nz = D == 2 ? 1 : 4;
  const int64_t N = (int64_t)nx * ny * nz;
  real *rho = malloc(sizeof(real) * N), *u = malloc(sizeof(real) * 3 * N),
       *g = malloc(sizeof(real) * 3 * N), *fa = malloc(sizeof(real) * Q * N),
       *fb = malloc(sizeof(real) * Q * N), *ro = malloc(sizeof(real) * N),
       *uo = malloc(sizeof(real) * 3 * N), *gs = malloc(sizeof(real) * 3);
  uint8_t *solid = malloc((size_t)N);
  for (int64_t n = 0; n < N; ++n) {
    rho[n] = (real)(1.0 + 0.02 * uniform());
    for (int a = 0; a < 3; ++a) {
      u[a * N + n] = (real)(a < D ? 0.05 * uniform() : 0.0);
      g[a * N + n] = (real)(a < D ? 1e-4 * uniform() : 0.0);
    }
    solid[n] = (uint8_t)(n % 11 == 5);
  }
  for (int a = 0; a < 3; ++a) gs[a] = (real)0.5;
  const int walls[3][3] = {{0, 0, 0}, {0, 1, 0}, {1, 0, 1}};
  int cases = 0, bad = 0;
  for (int coll = 0; coll < 3; ++coll)
    for (int wi = 0; wi < 3; ++wi)
      for (int so = 0; so < 2; ++so)
        for (int opt = 0; opt < 6; ++opt) {
          if (opt && coll != 1) continue;            /* options are the SMRT's */
          if (opt == 3 && D == 2) continue;          /* no traceless third order on D2Q9 */
          if (opt == 4 && Q != 27) continue;         /* orders 5-6 live on D3Q27 only */
          if (opt == 5 && L.NM < Q) continue;        /* order-4 force content: NM == Q */
          for (int s16 = 0; s16 < (sizeof(real) == 4 ? 2 : 1); ++s16) {
            oracle_params P;
            memset(&P, 0, sizeof(P));
            P.collision = coll;
            P.nx = nx;
            P.ny = ny;
            P.nz = nz;
            for (int a = 0; a < 3; ++a) P.wall[a] = walls[wi][a] && (a < D);
            P.store16 = s16;
            P.shift = s16 ? (real)1 : (real)0;
            P.omega = (real)(1.0 / 0.7);
            P.hforce = (real)(1.0 - 0.5 / 0.7);
            P.q2 = (real)(1.0 - 1.0 / 0.7);
            P.q3 = (real)(1.0 - 1.0 / 0.9);
            P.h2 = (real)(1.0 - 0.5 / 0.7);
            P.h3 = (real)(1.0 - 0.5 / 0.9);
            P.fq3 = (opt == 1 || opt == 5) ? (real)(1.0 - 0.5 / 0.9) : (real)0;
            P.fo4 = opt == 5;
            P.dqb = opt == 2 ? (real)(((1.0 - 1.0 / 1.3) - (1.0 - 1.0 / 0.7)) / D) : (real)0;
            P.dq31 = opt == 3 ? (real)(((1.0 - 1.0 / 1.4) - (1.0 - 1.0 / 0.9)) / 2) : (real)0;
            P.max_order = opt == 4 ? 6 : 4;
            P.solid = so ? solid : NULL;
            oracle_init(&L, &P, rho, u, g, fa);
            oracle_run(&L, &P, fa, fb, g, NULL, 3);
            oracle_step(&L, &P, fa, fb, g, (real)-0.5);
            oracle_moments(&L, &P, fb, g, (real)1, ro, uo);
            real node[MAXQ], out[MAXQ], feq[MAXQ], Fi[MAXQ];
            for (int i = 0; i < Q; ++i) node[i] = fb[(int64_t)i * N + 3];
            oracle_collide_node(&L, &P, node, gs, out);
            oracle_init_node(&L, &P, (real)1.01, gs, gs, out);
            oracle_bgk_terms(&L, (real)1.0, gs, gs, feq, Fi);
            ++cases;
            if (!all_finite(fb, Q * N) || !all_finite(ro, N) || !all_finite(uo, 3 * N) ||
                !all_finite(out, Q) || !all_finite(feq, Q) || !all_finite(Fi, Q))
              ++bad;
          }
        }
  free(e); free(opp); free(mi); free(w); free(H); free(Minv);
  free(rho); free(u); free(g); free(fa); free(fb); free(ro); free(uo); free(gs); free(solid);
  printf("%d cases, %d with non-finite results (real %zu bytes, plain %d)\n", cases, bad,
         sizeof(real), oracle_is_plain());
  return bad ? 1 : 0;
}

// Host check of the contraction plan (csrc/plan.cpp) on a job read from a text file: every output
// element of every task is covered by exactly one reduction item, each item's K splits tile the
// grid's point chunks [0, nchunks) in order without gaps or overlaps, every tile sits in one launch
// whose tile shape holds it, the issued FLOPs add up, and the splits of one item are even.
// Usage: plan_check <job file> <precision 0|1> <resident work-groups per launch> <budget GB> [options]
// (options: "share" and/or "overlap", e.g. "share,overlap").
// Job file: natoms, atoms (x y z Z), nbf, basis rows (atom n l m zeta), naux, aux rows, grid spec
// (n_mu n_nu n_phi q n_sp c1_scale c1_exp), npg, per-pair specs (A B + the 7 spec fields).
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "plan.h"

using namespace psint;

static int fail(const char* what, long a = 0, long b = 0) {
  printf("FAIL %s %ld %ld\n", what, a, b);
  return 1;
}

int main(int argc, char** argv) {
  if (argc < 5) return fail("usage");
  FILE* f = fopen(argv[1], "r");
  if (!f) return fail("open");
  int na = 0;
  if (fscanf(f, "%d", &na) != 1) return fail("read");
  std::vector<ps_atom> atoms(na);
  for (auto& a : atoms)
    if (fscanf(f, "%lf %lf %lf %lf", &a.xyz[0], &a.xyz[1], &a.xyz[2], &a.Z) != 4) return fail("atom");
  auto read_fns = [&](std::vector<ps_sto>& v) {
    int n = 0;
    if (fscanf(f, "%d", &n) != 1) return false;
    v.resize(n);
    for (auto& s : v)
      if (fscanf(f, "%d %d %d %d %lf", &s.atom, &s.n, &s.l, &s.m, &s.zeta) != 5) return false;
    return true;
  };
  std::vector<ps_sto> bf, ax;
  if (!read_fns(bf) || !read_fns(ax)) return fail("functions");
  ps_grid_spec sp;
  if (fscanf(f, "%d %d %d %d %d %lf %lf", &sp.n_mu, &sp.n_nu, &sp.n_phi, &sp.q, &sp.n_sp, &sp.c1_scale,
             &sp.c1_exp) != 7)
    return fail("spec");
  int npg = 0;
  if (fscanf(f, "%d", &npg) != 1) npg = 0;
  std::vector<ps_pair_grid> pgs(npg);
  for (auto& g : pgs)
    if (fscanf(f, "%d %d %d %d %d %d %d %lf %lf", &g.atom_a, &g.atom_b, &g.spec.n_mu, &g.spec.n_nu, &g.spec.n_phi,
               &g.spec.q, &g.spec.n_sp, &g.spec.c1_scale, &g.spec.c1_exp) != 9)
      return fail("pair spec");
  fclose(f);
  ps_job job{};
  job.atoms = atoms.data();
  job.n_atoms = na;
  job.basis = bf.data();
  job.n_bf = (int32_t)bf.size();
  job.aux = ax.data();
  job.n_aux = (int32_t)ax.size();
  job.grid = sp;
  job.pair_grids = pgs.data();
  job.n_pair_grids = npg;
  job.precision = atoi(argv[2]);
  TileShape ts;  // the library's defaults: FP64 4 x 4 with 16-point stages, mixed 4 x 4 with 32
  if (job.precision == PS_PREC_MIXED) ts.sc = 2;
  const int slots = atoi(argv[3]);
  ts.slots = ts.slots2 = ts.slots2n = ts.slots2_f64 = ts.slots2n_f64 = slots;
  for (int w = 1; w < 4; ++w) ts.slots_n[w] = slots;
  for (int w = 1; w <= 4; ++w) ts.slots_short[w] = slots;
  for (int w = 1; w <= 2; ++w) ts.slots_short_f64[w] = slots;
  for (int k = 0; k < 4; ++k) ts.slots_tall[k] = slots;
  const size_t budget = (size_t)(atof(argv[4]) * 1e9);
  Plan p;
  std::string err;
  const std::string opts = argc > 5 ? argv[5] : "";
  const bool share = opts.find("share") != std::string::npos;
  const bool overlap = opts.find("overlap") != std::string::npos;
  if (build_plan(&job, ts, 0, budget, &p, &err, share, overlap) != PS_OK) {
    printf("FAIL plan %s\n", err.c_str());
    return 1;
  }

  // array area: each pass's arrays and partial tiles inside its region, within the area; with
  // overlapped passes, consecutive passes' regions disjoint (one is written while the other is read)
  if (p.overlap && (!overlap || p.passes.size() < 2)) return fail("overlap without several passes");
  std::vector<std::pair<size_t, size_t>> region(p.passes.size());
  for (int k = 0; k < (int)p.passes.size(); ++k) {
    const Pass& ps = p.passes[k];
    const size_t end = ps.ws_offset + ps.ws_elems * 8;
    if (ps.ws_offset < ps.region_off || end > p.max_array_bytes) return fail("pass region", k);
    if (!p.overlap && ps.region_off != 0) return fail("region offset without overlap", k);
    region[k] = {ps.region_off, end};
    for (const auto& a : p.arrays) {
      if (a.grid < ps.grid0 || a.grid >= ps.grid1) continue;
      const size_t lo = (size_t)a.offset, hi = lo + (size_t)a.nf * p.grids[a.grid].dev.npad * a.es;
      if (lo < ps.region_off || hi > ps.ws_offset || lo % 256) return fail("array outside its pass's region", k, a.grid);
    }
    if (p.overlap && k > 0 && region[k].first < region[k - 1].second && region[k - 1].first < region[k].second)
      return fail("consecutive passes share memory", k);
  }

  // tiles by (pass, partial-tile offset): each pass reuses the workspace, each offset once per pass
  std::vector<int> pass_of_tile(p.tiles.size(), -1), pass_of_red(p.reds.size(), -1);
  for (int k = 0; k < (int)p.passes.size(); ++k) {
    for (int i = p.passes[k].tile0; i < p.passes[k].tile1; ++i) pass_of_tile[i] = k;
    for (const auto& ph : p.passes[k].red_by_phase)
      for (int r : ph) pass_of_red[r] = k;
  }
  std::map<std::pair<int, int64_t>, int> tile_at;
  for (int i = 0; i < (int)p.tiles.size(); ++i) {
    if (pass_of_tile[i] < 0) return fail("tile in no pass", i);
    if (!tile_at.emplace(std::make_pair(pass_of_tile[i], p.tiles[i].ws), i).second)
      return fail("two tiles of a pass share a partial tile", i);
  }
  for (size_t r = 0; r < p.reds.size(); ++r)
    if (pass_of_red[r] < 0) return fail("item reduced in no pass", (long)r);
  // launch of each tile, and the launch's shape holds the tile
  std::vector<int> launch_of(p.tiles.size(), -1);
  for (const Pass& ps : p.passes)
    for (const auto& l : ps.launches)
      for (int i = l.tile0; i < l.tile1; ++i) {
        if (launch_of[i] >= 0) return fail("tile in two launches", i);
        launch_of[i] = 1 + (int)(&l - ps.launches.data());
        const TileDev& t = p.tiles[i];
        TileShape ts2 = l.shape;  // a merged launch: the shape the tile names
        if (l.shape.wm == 0) {
          if (t.shape < 0 || t.shape > 7) return fail("merged tile without a shape", i);
          ts2.wm = kMergedShapes[t.shape][0];
          ts2.wn = kMergedShapes[t.shape][1];
          ts2.wr = kMergedShapes[t.shape][2];
        } else if (t.shape != 0) {
          return fail("shape named outside a merged launch", i);
        }
        if (t.nrows > ts2.bm() || t.np > ts2.bn()) return fail("tile larger than its shape", i);
        if (t.nu + t.nv > ts2.maxuv()) return fail("staged columns beyond the shape", i);
        // the launch's kernel reads its operands in the arrays' own element size: FP64 kernels for
        // FP64 jobs and a mixed job's FP64 tasks, FP32 kernels for a mixed job's FP32 operands
        const TaskHost& th = p.tasks[t.task];
        const size_t es = job.precision == PS_PREC_MIXED && !l.f64 ? 4 : 8;
        for (int a : {th.U, th.V, th.Y})
          if (p.arrays[a].es != es) return fail("launch precision differs from its operands", i, a);
      }
  for (size_t i = 0; i < p.tiles.size(); ++i)
    if (launch_of[i] < 0) return fail("tile in no launch", (long)i);

  // reduction items: splits tile [0, nchunks) in order, evenly; items cover each task once
  std::vector<std::vector<unsigned char>> cover(p.tasks.size());  // per task: row x column hits
  for (size_t t = 0; t < p.tasks.size(); ++t) cover[t].assign((size_t)p.tasks[t].dev.npairs * p.tasks[t].dev.ny, 0);
  std::vector<char> tile_used(p.tiles.size(), 0);
  double issued = 0.0;
  for (size_t r = 0; r < p.reds.size(); ++r) {
    const RedDev& R = p.reds[r];
    const TaskHost& th = p.tasks[R.task];
    const int64_t nch = p.grids[th.grid].dev.npad / KC;
    int64_t next = 0, lo = 1 << 30, hi = 0;
    for (int s = 0; s < R.nsplit; ++s) {
      auto it = tile_at.find(std::make_pair(pass_of_red[r], R.ws + (int64_t)s * R.bm * R.bn));
      if (it == tile_at.end()) return fail("split without a tile", (long)r, s);
      const TileDev& t = p.tiles[it->second];
      tile_used[it->second] = 1;
      if (t.task != R.task || t.row0 != R.row0 || t.nrows != R.nrows || t.p0 != R.p0 || t.np != R.np)
        return fail("split of another item", (long)r, s);
      if (t.kc0 != next || t.nkc <= 0 || t.nkc % TileShape::SC_MAX) return fail("split range", (long)r, s);
      next += t.nkc;
      lo = std::min<int64_t>(lo, t.nkc);
      hi = std::max<int64_t>(hi, t.nkc);
      issued += 2.0 * R.bm * R.bn * t.nkc * KC;
    }
    if (next != nch) return fail("splits do not end at the grid's last chunk", (long)r, (long)next);
    if (hi - lo > 2 * TileShape::SC_MAX) return fail("uneven splits", (long)r, (long)(hi - lo));
    auto& cv = cover[R.task];
    const int ny = p.tasks[R.task].dev.ny;
    if (R.row0 < 0 || R.row0 + R.nrows > p.tasks[R.task].dev.npairs || R.p0 < 0 || R.p0 + R.np > ny)
      return fail("item outside its task", (long)r);
    for (int i = 0; i < R.nrows; ++i)
      for (int c = 0; c < R.np; ++c)
        if (cv[(size_t)(R.row0 + i) * ny + R.p0 + c]++) return fail("element in two items", R.task, R.row0 + i);
  }
  for (size_t i = 0; i < p.tiles.size(); ++i)
    if (!tile_used[i]) return fail("tile of no item", (long)i);
  for (size_t t = 0; t < p.tasks.size(); ++t)
    for (size_t e = 0; e < cover[t].size(); ++e)
      if (cover[t][e] != 1) return fail("element of no item", (long)t, (long)e);
  if (issued != p.issued_flops) return fail("issued FLOPs", (long)(issued / 1e9), (long)(p.issued_flops / 1e9));

  // shared evaluation (cross-third-centre reuse): kept shares have all members in one pass and are
  // listed in that pass; their cells avoid every member's moved lines; each member's basis segment
  // skips exactly those cells; dropped shares leave no skipping segment; the launch covers the cells
  size_t kept = 0;
  std::vector<int> skipped_by(p.segs.size(), 0);
  for (int k = 0; k < (int)p.passes.size(); ++k) {
    const Pass& ps = p.passes[k];
    int64_t blk = 0;
    for (int x = ps.sseg0; x < ps.sseg1; ++x) {
      const ShareHost& sh = p.shares[p.ssegs[x]];
      ++kept;
      if (sh.dropped) return fail("dropped share listed", x);
      if (sh.dev.block0 != blk) return fail("share block offset", x);
      const GridDev& g0 = p.grids[sh.grids[0]].dev;
      blk += ((int64_t)sh.dev.n_si * sh.dev.n_sj * g0.nphi + 3) / 4;
      const int32_t* cells = p.ints.data() + sh.cells_off;
      for (size_t c = 0; c < sh.grids.size(); ++c) {
        const int gi = sh.grids[c];
        if (gi < ps.grid0 || gi >= ps.grid1) return fail("share member outside its pass", x, gi);
        const GridDev& d = p.grids[gi].dev;
        if (d.q != 4 || d.nmu != g0.nmu || d.nnu != g0.nnu || d.nphi != g0.nphi) return fail("share member shape", x, gi);
        const SegDev& sg = p.segs[sh.segs[c]].dev;
        if (!sg.skip || sg.grid != gi || sg.centre != sh.dev.centre) return fail("member segment", x, gi);
        skipped_by[sh.segs[c]]++;
        uint64_t mm[2] = {0, 0}, nm[2] = {0, 0};
        for (int t = 0; t < sh.dev.n_si; ++t) mm[cells[t] >> 6] |= 1ull << (cells[t] & 63);
        for (int t = 0; t < sh.dev.n_sj; ++t) nm[cells[sh.dev.n_si + t] >> 6] |= 1ull << (cells[sh.dev.n_si + t] & 63);
        if (mm[0] != sg.skip_mu[0] || mm[1] != sg.skip_mu[1] || nm[0] != sg.skip_nu[0] || nm[1] != sg.skip_nu[1])
          return fail("skip masks differ from the shared cells", x, gi);
        for (int t = 0; t < sh.dev.n_si; ++t)
          if (d.istar > 0 && (cells[t] == d.istar - 1 || cells[t] == d.istar)) return fail("shared mu cell at a moved line", x, gi);
        for (int t = 0; t < sh.dev.n_sj; ++t)
          if (d.jstar > 0 && (cells[sh.dev.n_si + t] == d.jstar - 1 || cells[sh.dev.n_si + t] == d.jstar))
            return fail("shared nu cell at a moved line", x, gi);
      }
    }
    if (blk != ps.shared_blocks) return fail("shared blocks of a pass", k);
  }
  for (size_t si = 0; si < p.segs.size(); ++si)
    if ((p.segs[si].dev.skip != 0) != (skipped_by[si] == 1)) return fail("segment skips without one share", (long)si);
  if (share && kept == 0) return fail("no share kept");
  std::map<std::string, int> shapes;  // tile shapes used, as wm.wn.sc.wr ("merged" if a launch merges them)
  for (const Pass& ps : p.passes)
    for (const auto& l : ps.launches) {
      char key[32];
      if (l.shape.wm == 0) {
        shapes["merged"]++;
        for (int i = l.tile0; i < l.tile1; ++i) {
          const int* m = kMergedShapes[p.tiles[i].shape];
          snprintf(key, sizeof key, "%d.%d.%d.%d", m[0], m[1], l.shape.sc, m[2]);
          shapes[key]++;
        }
      } else {
        snprintf(key, sizeof key, "%d.%d.%d.%d", l.shape.wm, l.shape.wn, l.shape.sc, l.shape.wr);
        shapes[key]++;
      }
    }
  printf("ok %zu tiles %zu items %zu passes %zu shares%s shapes", p.tiles.size(), p.reds.size(), p.passes.size(),
         kept, p.overlap ? " overlapped" : "");
  for (const auto& kv : shapes) printf(" %s", kv.first.c_str());
  printf("\n");
  return 0;
}

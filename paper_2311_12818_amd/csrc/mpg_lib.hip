// libmpg: kernels and the C ABI declared in include/mpg.h.
#include "mpg_internal.h"
#include "mpg_walk.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;
mpg_status fail(mpg_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

extern "C" const char* mpg_last_error(void) { return g_err.c_str(); }
extern "C" const char* mpg_version(void) { return "mpg 0.1 gfx950"; }

// ---------------------------------------------------------------------------
// scene
// ---------------------------------------------------------------------------
extern "C" mpg_status mpg_scene_create(const mpg_scene_desc* d, mpg_scene** out) {
  if (!d || !out) return fail(MPG_ERR_INVALID_ARG, "mpg_scene_create: NULL argument");
  if (d->n_tris < 0 || d->n_verts < 0 || d->n_objects <= 0 || d->n_spheres < 0)
    return fail(MPG_ERR_INVALID_ARG, "mpg_scene_create: negative size or no objects");
  if (d->n_tris > 0 && (!d->verts || !d->normals || !d->tris || !d->tri_obj))
    return fail(MPG_ERR_INVALID_ARG, "mpg_scene_create: missing triangle arrays");
  if (d->n_tris >= (1 << 24)) return fail(MPG_ERR_UNSUPPORTED, "mpg_scene_create: more than 2^24 triangles");
  if (d->n_spheres > 0 && (!d->spheres || !d->sphere_obj))
    return fail(MPG_ERR_INVALID_ARG, "mpg_scene_create: missing sphere arrays");
  if (!d->obj_material || !d->obj_ior) return fail(MPG_ERR_INVALID_ARG, "mpg_scene_create: missing object arrays");
  if (d->n_heightfields < 0 || (d->n_heightfields > 0 && !d->heightfields))
    return fail(MPG_ERR_INVALID_ARG, "mpg_scene_create: bad height-field list");
  for (int t = 0; t < d->n_tris; ++t) {
    for (int k = 0; k < 3; ++k)
      if (d->tris[3 * t + k] < 0 || d->tris[3 * t + k] >= d->n_verts)
        return fail(MPG_ERR_INVALID_ARG, "mpg_scene_create: triangle vertex index out of range");
    if (d->tri_obj[t] < 0 || d->tri_obj[t] >= d->n_objects)
      return fail(MPG_ERR_INVALID_ARG, "mpg_scene_create: triangle object id out of range");
  }
  for (int s = 0; s < d->n_spheres; ++s)
    if (d->sphere_obj[s] < 0 || d->sphere_obj[s] >= d->n_objects || !(d->spheres[4 * s + 3] > 0.0f))
      return fail(MPG_ERR_INVALID_ARG, "mpg_scene_create: bad sphere");
  for (int o = 0; o < d->n_objects; ++o)
    if (d->obj_material[o] != MPG_MAT_MIRROR && d->obj_material[o] != MPG_MAT_DIELECTRIC)
      return fail(MPG_ERR_INVALID_ARG, "mpg_scene_create: unknown material");

  mpg_scene* s = new mpg_scene();
  (void)hipGetDevice(&s->device);
  s->scale = d->scale;
  s->n_tris = d->n_tris;
  s->n_verts = d->n_verts;
  for (int i = 0; i < d->n_heightfields; ++i) s->hfs.push_back(d->heightfields[i]);
  std::vector<DevHF> dhf;
  for (const mpg_heightfield& h : s->hfs) {
    if (h.n_sines < 0 || h.n_sines > 8 || h.res < 2 || h.first_vert < 0 || h.first_tri < 0 ||
        h.first_vert + h.res * h.res > d->n_verts || h.first_tri + 2 * (h.res - 1) * (h.res - 1) > d->n_tris) {
      delete s;
      return fail(MPG_ERR_INVALID_ARG, "mpg_scene_create: height field outside the mesh or more than 8 sines");
    }
    DevHF q;
    std::memset(&q, 0, sizeof(q));
    q.first_vert = h.first_vert;
    q.n_verts = h.res * h.res;
    q.first_tri = h.first_tri;
    q.n_tris = 2 * (h.res - 1) * (h.res - 1);
    q.n_sines = h.n_sines;
    q.param_base = s->n_params;
    for (int k = 0; k < h.n_sines; ++k) {
      q.amp[k] = h.amp[k]; q.freq[k] = h.freq[k]; q.psi[k] = h.psi[k]; q.phase[k] = h.phase[k];
    }
    s->n_params += 2 * h.n_sines;
    dhf.push_back(q);
  }
  if (s->n_params > 64) {
    delete s;
    return fail(MPG_ERR_UNSUPPORTED, "mpg_scene_create: more than 64 height-field parameters");
  }
  auto bail = [&](hipError_t e, const char* what) {
    free_all(s->allocs);
    delete s;
    return fail(MPG_ERR_HIP, std::string("mpg_scene_create: ") + what + ": " + hipGetErrorString(e));
  };
  hipError_t e;
  DevScene& D = s->dev;
  std::memset(&D, 0, sizeof(D));
  D.n_tris = d->n_tris;
  D.n_spheres = d->n_spheres;
  D.n_objects = d->n_objects;
  // geometry
  std::vector<float4> vp(d->n_verts), vn(d->n_verts);
  float zmax = -INFINITY;
  for (int i = 0; i < d->n_verts; ++i) {
    vp[i] = make_float4(d->verts[3 * i], d->verts[3 * i + 1], d->verts[3 * i + 2], 0.f);
    float nx = d->normals[3 * i], ny = d->normals[3 * i + 1], nz = d->normals[3 * i + 2];
    float l = std::sqrt(nx * nx + ny * ny + nz * nz);
    vn[i] = make_float4(nx / l, ny / l, nz / l, 0.f);
  }
  std::vector<int4> ti(d->n_tris);
  for (int t = 0; t < d->n_tris; ++t) {
    ti[t] = make_int4(d->tris[3 * t], d->tris[3 * t + 1], d->tris[3 * t + 2], d->tri_obj[t]);
    for (int k = 0; k < 3; ++k) zmax = std::max(zmax, d->verts[3 * d->tris[3 * t + k] + 2]);
  }
  std::vector<float> nodes;
  std::vector<int32_t> order, ranges;
  int depth = 0;
  int n_nodes = 0;
  if (d->n_tris > 0) {
    float lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < 3 * d->n_verts; ++i) { lo = std::min(lo, d->verts[i]); hi = std::max(hi, d->verts[i]); }
    float pad = 1e-6f * std::max(1.0f, std::max(std::fabs(lo), std::fabs(hi)));
    s->pad = pad;
    n_nodes = mpg_host::build_bvh(d->verts, d->tris, d->n_tris, pad, nodes, order, ranges, &depth);
  }
  s->n_objects = d->n_objects;
  // top of the geometry that the height-field parameters do not move
  {
    std::vector<char> moving(d->n_verts, 0);
    for (const mpg_heightfield& h : s->hfs)
      for (int v = h.first_vert; v < h.first_vert + h.res * h.res; ++v) moving[v] = 1;
    for (int t = 0; t < d->n_tris; ++t)
      for (int k = 0; k < 3; ++k) {
        int v = d->tris[3 * t + k];
        if (!moving[v]) s->zmax_static = std::max(s->zmax_static, d->verts[3 * v + 2]);
      }
    for (int k = 0; k < d->n_spheres; ++k)
      s->zmax_static = std::max(s->zmax_static, d->spheres[4 * k + 2] + d->spheres[4 * k + 3]);
  }
  s->n_nodes = n_nodes;
  s->max_depth = depth;
  D.n_nodes = n_nodes;
  std::vector<float4> tv(3 * (size_t)d->n_tris);
  for (int k = 0; k < d->n_tris; ++k) {
    int t = order[k];
    for (int v = 0; v < 3; ++v) {
      const float* p = d->verts + 3 * (size_t)d->tris[3 * t + v];
      float w = 0.f;
      if (v == 0) std::memcpy(&w, &t, 4);
      tv[3 * (size_t)k + v] = make_float4(p[0], p[1], p[2], w);
    }
  }
  std::vector<int2> oi(d->n_objects);
  for (int o = 0; o < d->n_objects; ++o) {
    int ib;
    float ior = d->obj_ior[o];
    std::memcpy(&ib, &ior, 4);
    oi[o] = make_int2(d->obj_material[o], ib);
  }
  // per-primitive geometry record (positions and unit normals of the three
  // vertices, object, material and index of refraction): one load level for
  // the walk's vertex geometry instead of triangle ids, then vertices
  std::vector<float4> tg(6 * (size_t)d->n_tris);
  for (int t = 0; t < d->n_tris; ++t) {
    const int4 id = ti[t];
    const int vid[3] = {id.x, id.y, id.z};
    for (int v = 0; v < 3; ++v) {
      tg[6 * (size_t)t + v] = vp[vid[v]];
      tg[6 * (size_t)t + 3 + v] = vn[vid[v]];
    }
    std::memcpy(&tg[6 * (size_t)t].w, &id.w, 4);
    std::memcpy(&tg[6 * (size_t)t + 1].w, &oi[id.w].x, 4);
    std::memcpy(&tg[6 * (size_t)t + 2].w, &oi[id.w].y, 4);
  }
  std::vector<float4> sph(d->n_spheres);
  for (int k = 0; k < d->n_spheres; ++k) {
    sph[k] = make_float4(d->spheres[4 * k], d->spheres[4 * k + 1], d->spheres[4 * k + 2], d->spheres[4 * k + 3]);
    zmax = std::max(zmax, d->spheres[4 * k + 2] + d->spheres[4 * k + 3]);
  }
  // area prefix sums per object and over all objects (input order), summed in
  // FP64 on the host and stored as FP32 pairs hi + lo (hi the rounding, lo
  // the rounded remainder)
  int O = d->n_objects;
  std::vector<std::vector<double>> cd(O + 1);
  std::vector<std::vector<int>> cp(O + 1);
  std::vector<float4> ob(O, make_float4(INFINITY, INFINITY, -INFINITY, -INFINITY));
  auto add = [&](int key, int prim, double area) {
    double prev = cd[key].empty() ? 0.0 : cd[key].back();
    cd[key].push_back(prev + area);
    cp[key].push_back(prim);
  };
  for (int t = 0; t < d->n_tris; ++t) {
    double P[3][3];
    for (int v = 0; v < 3; ++v)
      for (int a = 0; a < 3; ++a) P[v][a] = d->verts[3 * (size_t)d->tris[3 * t + v] + a];
    double e1[3], e2[3];
    for (int a = 0; a < 3; ++a) { e1[a] = P[1][a] - P[0][a]; e2[a] = P[2][a] - P[0][a]; }
    double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2], cz = e1[0] * e2[1] - e1[1] * e2[0];
    double area = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
    int o = d->tri_obj[t];
    add(o, t, area);
    add(O, t, area);
    for (int v = 0; v < 3; ++v) {
      ob[o].x = std::min(ob[o].x, (float)P[v][0]); ob[o].y = std::min(ob[o].y, (float)P[v][1]);
      ob[o].z = std::max(ob[o].z, (float)P[v][0]); ob[o].w = std::max(ob[o].w, (float)P[v][1]);
    }
  }
  for (int k = 0; k < d->n_spheres; ++k) {
    double r = d->spheres[4 * k + 3];
    double area = 4.0 * M_PI * r * r;
    int o = d->sphere_obj[k];
    add(o, -1 - k, area);
    add(O, -1 - k, area);
    ob[o].x = std::min(ob[o].x, sph[k].x - sph[k].w); ob[o].y = std::min(ob[o].y, sph[k].y - sph[k].w);
    ob[o].z = std::max(ob[o].z, sph[k].x + sph[k].w); ob[o].w = std::max(ob[o].w, sph[k].y + sph[k].w);
  }
  std::vector<float2> cdf;
  std::vector<int> cprim;
  std::vector<int2> crange(O + 1);
  for (int k = 0; k <= O; ++k) {
    crange[k] = make_int2((int)cdf.size(), (int)cd[k].size());
    for (double c : cd[k]) {
      float hi = (float)c;
      cdf.push_back(make_float2(hi, (float)(c - (double)hi)));
    }
    cprim.insert(cprim.end(), cp[k].begin(), cp[k].end());
  }
  if ((e = upload(s->allocs, &D.nodes, (const float4*)nodes.data(), nodes.size() / 4)) != hipSuccess) return bail(e, "nodes");
  if ((e = upload(s->allocs, &D.tri_v, tv.data(), tv.size())) != hipSuccess) return bail(e, "triangles");
  if ((e = upload(s->allocs, &D.tri_idx, ti.data(), ti.size())) != hipSuccess) return bail(e, "triangle ids");
  if ((e = upload(s->allocs, &D.tri_geo, tg.data(), tg.size())) != hipSuccess) return bail(e, "triangle records");
  if ((e = upload(s->allocs, &D.vpos, vp.data(), vp.size())) != hipSuccess) return bail(e, "positions");
  if ((e = upload(s->allocs, &D.vnrm, vn.data(), vn.size())) != hipSuccess) return bail(e, "normals");
  if ((e = upload(s->allocs, &D.obj_info, oi.data(), oi.size())) != hipSuccess) return bail(e, "objects");
  if ((e = upload(s->allocs, &D.spheres, sph.data(), sph.size())) != hipSuccess) return bail(e, "spheres");
  std::vector<int> so(d->sphere_obj, d->sphere_obj + d->n_spheres);
  if ((e = upload(s->allocs, &D.sphere_obj, so.data(), so.size())) != hipSuccess) return bail(e, "sphere objects");
  if ((e = upload(s->allocs, &D.cdf, cdf.data(), cdf.size())) != hipSuccess) return bail(e, "cdf");
  if ((e = upload(s->allocs, &D.cdf_prim, cprim.data(), cprim.size())) != hipSuccess) return bail(e, "cdf prims");
  if ((e = upload(s->allocs, &D.cdf_range, crange.data(), crange.size())) != hipSuccess) return bail(e, "cdf ranges");
  if ((e = upload(s->allocs, &D.obj_bounds, ob.data(), ob.size())) != hipSuccess) return bail(e, "bounds");
  if ((e = upload(s->allocs, &s->dev_hf, dhf.data(), dhf.size())) != hipSuccess) return bail(e, "height fields");
  if ((e = upload(s->allocs, &s->order, order.data(), order.size())) != hipSuccess) return bail(e, "leaf order");
  if ((e = upload(s->allocs, &s->ranges, ranges.data(), ranges.size())) != hipSuccess) return bail(e, "node ranges");
  if ((e = dalloc(s->allocs, &s->zmax_bits, 1)) != hipSuccess) return bail(e, "scratch");
  if ((e = upload(s->allocs, &D.zmax, &zmax, 1)) != hipSuccess) return bail(e, "scene top");
  {
    const int32_t ok = MPG_OK;
    const int32_t* pe = nullptr;
    if ((e = upload(s->allocs, &pe, &ok, 1)) != hipSuccess) return bail(e, "error word");
    s->param_err = (int32_t*)pe;
  }
  *out = s;
  return MPG_OK;
}

extern "C" void mpg_scene_destroy(mpg_scene* s) {
  if (!s) return;
  free_all(s->allocs);
  delete s;
}

extern "C" mpg_status mpg_scene_stats(const mpg_scene* s, int32_t* n_nodes, int32_t* max_depth, int32_t* n_tris) {
  if (!s) return fail(MPG_ERR_INVALID_ARG, "mpg_scene_stats: NULL scene");
  if (n_nodes) *n_nodes = s->n_nodes;
  if (max_depth) *max_depth = s->max_depth;
  if (n_tris) *n_tris = s->n_tris;
  return MPG_OK;
}

extern "C" mpg_status mpg_walk_params_default(float scale, mpg_walk_params* p) {
  if (!p || !(scale > 0.0f)) return fail(MPG_ERR_INVALID_ARG, "mpg_walk_params_default: bad argument");
  p->max_iter = 20;
  p->tol_vertex = 1e-4f;
  p->tol_residual = 1e-5f;
  p->scale = scale;
  p->tmin_rel = 1e-5f;
  p->match_rel = 1e-3f;
  p->fp64_cond_threshold = 1e4f;
  p->fp64_graze_cos = 0.02f;
  p->cone_cos = 0.0f;
  p->form = MPG_FORM_PLAIN;
  p->bucketing = 1;
  p->waves_per_group = 4;
  p->stack_depth = 0;
  p->refill = 0;
  p->max_len = KMAX;
  p->defer_fp64 = 0;
  p->length_order = 0;
  return MPG_OK;
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
extern "C" mpg_status mpg_workspace_create(int32_t max_chains, mpg_workspace** out) {
  if (!out || max_chains < 0) return fail(MPG_ERR_INVALID_ARG, "mpg_workspace_create: bad argument");
  mpg_workspace* w = new mpg_workspace();
  w->cap = max_chains;
  hipError_t e;
  if ((e = dalloc(w->allocs, &w->perm, (size_t)max_chains + 8 * 64)) != hipSuccess ||
      (e = dalloc(w->allocs, &w->counters, MPG_WS_COUNTERS)) != hipSuccess ||
      (e = dalloc(w->allocs, &w->cells, (size_t)2 * KMAX * MPG_CELLS)) != hipSuccess ||
      (e = dalloc(w->allocs, &w->aux, (size_t)max_chains + 64)) != hipSuccess) {
    free_all(w->allocs);
    delete w;
    return fail(MPG_ERR_HIP, std::string("mpg_workspace_create: ") + hipGetErrorString(e));
  }
  *out = w;
  return MPG_OK;
}
extern "C" void mpg_workspace_destroy(mpg_workspace* w) {
  if (!w) return;
  free_all(w->allocs);
  delete w;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
__global__ void k_sample_seeds(DevScene S, DevGuide G, WalkParams P, EpView E, uint64_t seed,
                               uint64_t trial, float alpha, int32_t* prim_out, float* pos_out, int8_t* st) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  Stack stk = lane_stack(P.depth);
  if (c >= E.N) return;
  int n = E.len[c];
  if (n < 1 || n > KMAX || !finite3(ld_pt(E.xD, E.N, c)) || !finite3(ld_pt(E.nD, E.N, c))) {
    st[c] = ST_BAD_INPUT;
    return;
  }
  // always the argument's address (no guide: a zeroed DevGuide); a pointer
  // that may be null would make the compiler copy G to private memory
  const DevGuide* g = &G;
  switch (n) {
    case 1: seed_one<1>(S, g, P, E, c, seed, trial, alpha, prim_out, pos_out, st, stk); break;
    case 2: seed_one<2>(S, g, P, E, c, seed, trial, alpha, prim_out, pos_out, st, stk); break;
    case 3: seed_one<3>(S, g, P, E, c, seed, trial, alpha, prim_out, pos_out, st, stk); break;
    case 4: seed_one<4>(S, g, P, E, c, seed, trial, alpha, prim_out, pos_out, st, stk); break;
    case 5: seed_one<5>(S, g, P, E, c, seed, trial, alpha, prim_out, pos_out, st, stk); break;
    case 6: seed_one<6>(S, g, P, E, c, seed, trial, alpha, prim_out, pos_out, st, stk); break;
    case 7: seed_one<7>(S, g, P, E, c, seed, trial, alpha, prim_out, pos_out, st, stk); break;
    default: seed_one<8>(S, g, P, E, c, seed, trial, alpha, prim_out, pos_out, st, stk); break;
  }
}

// Plain form: one launch, one chain per lane, chains in input order; NMAX is
// the longest chain the launch handles (the register budget follows it).
template <int NMAX>
__global__ void __launch_bounds__(256) k_walk_plain(DevScene S, WalkParams P, EpView E, WalkIO io) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  Stack stk = lane_stack(P.depth);
  if (c >= E.N) return;
  walk_dispatch<NMAX>(S, P, E, io, c, stk);
}

template <int NMAX>
__global__ void __launch_bounds__(256) k_finish_pass(DevScene S, WalkParams P, EpView E, WalkIO io) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  Stack stk = lane_stack(P.depth);
  if (c >= E.N) return;
  finish_dispatch<NMAX>(S, P, E, io, c, stk);
}

// FP64 pass over the chains the walk left as ST_NEEDS_FP64.
template <int NMAX>
__global__ void __launch_bounds__(256) k_fp64_pass(DevScene S, WalkParams P, EpView E, WalkIO io) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  Stack stk = lane_stack(P.depth);
  if (c >= E.N) return;
  if (io.status[c] != ST_NEEDS_FP64) return;
  int n = E.len[c];
  switch (n) {
    case 1: fp64_one<1>(S, P, E, io, c, stk); break;
    case 2: if (NMAX >= 2) fp64_one<(NMAX >= 2 ? 2 : 1)>(S, P, E, io, c, stk); break;
    case 3: if (NMAX >= 3) fp64_one<(NMAX >= 3 ? 3 : 1)>(S, P, E, io, c, stk); break;
    case 4: if (NMAX >= 4) fp64_one<(NMAX >= 4 ? 4 : 1)>(S, P, E, io, c, stk); break;
    case 5: if (NMAX >= 5) fp64_one<(NMAX >= 5 ? 5 : 1)>(S, P, E, io, c, stk); break;
    case 6: if (NMAX >= 6) fp64_one<(NMAX >= 6 ? 6 : 1)>(S, P, E, io, c, stk); break;
    case 7: if (NMAX >= 7) fp64_one<(NMAX >= 7 ? 7 : 1)>(S, P, E, io, c, stk); break;
    default: if (NMAX >= 8) fp64_one<(NMAX >= 8 ? 8 : 1)>(S, P, E, io, c, stk); break;
  }
}

// Counting launch: the plain walk with every unit of work tallied per lane
// (box tests, triangle tests, sphere tests, rays, residual-only and Jacobian
// vertex evaluations, FP64 vertex evaluations); the tallies are reduced into
// counts[0..6], counts[7] = chains.  Used untimed to obtain the algorithmic
// work of a launch.
typedef void (*walk_kernel_t)(DevScene, WalkParams, EpView, WalkIO);
static walk_kernel_t plain_kernel(int nmax) {
  switch (nmax) {
    case 1: return k_walk_plain<1>;
    case 2: return k_walk_plain<2>;
    case 3: return k_walk_plain<3>;
    case 4: return k_walk_plain<4>;
    case 5: return k_walk_plain<5>;
    case 6: return k_walk_plain<6>;
    case 7: return k_walk_plain<7>;
    default: return k_walk_plain<8>;
  }
}
static walk_kernel_t finish_kernel(int nmax) {
  switch (nmax) {
    case 1: return k_finish_pass<1>;
    case 2: return k_finish_pass<2>;
    case 3: return k_finish_pass<3>;
    case 4: return k_finish_pass<4>;
    case 5: return k_finish_pass<5>;
    case 6: return k_finish_pass<6>;
    case 7: return k_finish_pass<7>;
    default: return k_finish_pass<8>;
  }
}
static walk_kernel_t fp64_kernel(int nmax) {
  switch (nmax) {
    case 1: return k_fp64_pass<1>;
    case 2: return k_fp64_pass<2>;
    case 3: return k_fp64_pass<3>;
    case 4: return k_fp64_pass<4>;
    case 5: return k_fp64_pass<5>;
    case 6: return k_fp64_pass<6>;
    case 7: return k_fp64_pass<7>;
    default: return k_fp64_pass<8>;
  }
}

mpg_status launch_finish_plain(const mpg_scene* s, const WalkParams& P, const EpView& E, const WalkIO& io,
                               int max_len, int threads, size_t lds, hipStream_t stream) {
  hipLaunchKernelGGL(finish_kernel(max_len), dim3((E.N + threads - 1) / threads), dim3(threads), lds, stream,
                     s->dev, P, E, io);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}

// ---------------------------------------------------------------------------
// host entry points
// ---------------------------------------------------------------------------
mpg_status check_params(const mpg_scene* s, const mpg_walk_params* p, WalkParams* w, int* waves) {
  if (!p) return fail(MPG_ERR_INVALID_ARG, "NULL walk params");
  if (p->max_iter < 0 || p->max_iter > 255) return fail(MPG_ERR_INVALID_ARG, "max_iter outside 0..255");
  if (!(p->scale > 0.0f)) return fail(MPG_ERR_INVALID_ARG, "scale must be positive");
  if (!(p->tol_vertex >= 0.0f) || !(p->tol_residual >= 0.0f) || !(p->tmin_rel >= 0.0f) || !(p->match_rel >= 0.0f))
    return fail(MPG_ERR_INVALID_ARG, "negative tolerance");
  if (p->bucketing < 0 || p->bucketing > 3) return fail(MPG_ERR_INVALID_ARG, "bucketing must be 0, 1, 2 or 3");
  if (p->waves_per_group != 1 && p->waves_per_group != 2 && p->waves_per_group != 4)
    return fail(MPG_ERR_INVALID_ARG, "waves_per_group must be 1, 2 or 4");
  int need = s->max_depth + 1;
  int depth = p->stack_depth > 0 ? p->stack_depth : need;
  if (depth < need) return fail(MPG_ERR_INVALID_ARG, "stack_depth below BVH depth + 1");
  if ((size_t)p->waves_per_group * depth * 64 * 4 > 64 * 1024)
    return fail(MPG_ERR_INVALID_ARG, "LDS stacks exceed 64 KiB per workgroup");
  w->max_iter = p->max_iter;
  float tv = p->tol_vertex * p->scale;
  w->tol_step2 = tv * tv;
  w->tol_residual = p->tol_residual;
  w->tmin = p->tmin_rel * p->scale;
  float m = p->match_rel * p->scale;
  w->match2 = m * m;
  w->fp64_cond = p->fp64_cond_threshold;
  w->graze_cos = p->fp64_graze_cos;
  w->cone_cos = p->cone_cos;
  w->depth = depth;
  *waves = p->waves_per_group;
  if (p->max_len < 1 || p->max_len > KMAX) return fail(MPG_ERR_INVALID_ARG, "max_len outside 1..8");
  if (p->length_order != 0) {
    unsigned seen = 0;
    for (int k = 0; k < KMAX; ++k) seen |= 1u << ((p->length_order >> (4 * k)) & 15u);
    if (seen != 0x1FEu) return fail(MPG_ERR_INVALID_ARG, "length_order is not a permutation of the lengths 1..8");
  }
  return MPG_OK;
}

mpg_status check_endpoints(const mpg_endpoints* e, EpView* v) {
  if (!e) return fail(MPG_ERR_INVALID_ARG, "NULL endpoints");
  if (e->N < 0) return fail(MPG_ERR_INVALID_ARG, "N < 0");
  if (e->N > 0 && (!e->d_xD || !e->d_nD || !e->d_xL || !e->d_len || !e->d_type || !e->d_obj1))
    return fail(MPG_ERR_INVALID_ARG, "NULL endpoint array");
  v->xD = e->d_xD; v->nD = e->d_nD; v->xL = e->d_xL; v->len = e->d_len; v->type = e->d_type; v->obj1 = e->d_obj1;
  v->off = e->d_offset;
  v->N = e->N;
  return MPG_OK;
}

extern "C" mpg_status sample_seeds(const mpg_scene* s, const mpg_guide* g, const mpg_walk_params* p,
                                   const mpg_endpoints* ep, uint64_t philox_seed, uint32_t trial, float alpha,
                                   mpg_chains* out, int8_t* d_status, mpg_workspace* ws, void* stream) {
  if (!s) return fail(MPG_ERR_INVALID_ARG, "sample_seeds: NULL scene");
  WalkParams P;
  int waves;
  EpView E;
  mpg_status st;
  if ((st = check_params(s, p, &P, &waves)) != MPG_OK) return st;
  if ((st = check_endpoints(ep, &E)) != MPG_OK) return st;
  if (E.N == 0) return MPG_OK;
  if (!out || !out->d_prim || !out->d_pos || !d_status) return fail(MPG_ERR_INVALID_ARG, "sample_seeds: NULL output");
  if (!(alpha >= 0.0f && alpha <= 1.0f)) return fail(MPG_ERR_INVALID_ARG, "sample_seeds: alpha outside [0, 1]");
  DevGuide G;
  std::memset(&G, 0, sizeof(G));
  if (g) G = g->dev();
  if (p->form == MPG_FORM_PERSISTENT && p->bucketing) {
    if (!ws || ws->cap < E.N) return fail(MPG_ERR_INVALID_ARG, "sample_seeds: workspace too small");
    return seeds_persistent(s, G, P, waves, p->bucketing, p->length_order, E, philox_seed, trial, alpha,
                            out->d_prim, out->d_pos, d_status, ws, (hipStream_t)stream);
  }
  int threads = 64 * waves;
  size_t lds = (size_t)waves * P.depth * 64 * 4;
  hipLaunchKernelGGL(k_sample_seeds, dim3((E.N + threads - 1) / threads), dim3(threads), lds, (hipStream_t)stream,
                     s->dev, G, P, E, philox_seed, (uint64_t)trial, alpha, out->d_prim, out->d_pos,
                     d_status);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}


extern "C" mpg_status manifold_walk_batch(const mpg_scene* s, const mpg_walk_params* p, const mpg_endpoints* ep,
                                          const mpg_chains* seeds, const int8_t* d_seed_status, mpg_chains* out,
                                          const mpg_walk_out* wout, mpg_workspace* ws, void* stream) {
  if (!s) return fail(MPG_ERR_INVALID_ARG, "manifold_walk_batch: NULL scene");
  WalkParams P;
  int waves;
  EpView E;
  mpg_status st;
  if ((st = check_params(s, p, &P, &waves)) != MPG_OK) return st;
  if ((st = check_endpoints(ep, &E)) != MPG_OK) return st;
  if (E.N == 0) return MPG_OK;
  if (!seeds || !seeds->d_prim || !seeds->d_pos || !out || !out->d_prim || !out->d_pos || !wout || !wout->d_status)
    return fail(MPG_ERR_INVALID_ARG, "manifold_walk_batch: NULL chains or status");
  WalkIO io;
  io.seed_prim = seeds->d_prim; io.seed_pos = seeds->d_pos; io.seed_status = d_seed_status;
  io.prim_out = out->d_prim; io.pos_out = out->d_pos;
  io.status = wout->d_status; io.iters = wout->d_iters; io.sol = wout->d_solution_id;
  io.G = wout->d_G; io.kappa = wout->d_kappa; io.resid = wout->d_residual;
  int threads = 64 * waves;
  size_t lds = (size_t)waves * P.depth * 64 * 4;
  dim3 grid((E.N + threads - 1) / threads);
  if (p->form == MPG_FORM_PERSISTENT) {
    if (!ws || ws->cap < E.N) return fail(MPG_ERR_INVALID_ARG, "manifold_walk_batch: workspace too small");
    mpg_status st2 = walk_persistent(s, P, waves, p->bucketing, p->refill, p->max_len, p->length_order, E, io, ws,
                                     (hipStream_t)stream);
    if (st2 != MPG_OK) return st2;
  } else if (p->form == MPG_FORM_PLAIN) {
    hipLaunchKernelGGL(plain_kernel(p->max_len), grid, dim3(threads), lds, (hipStream_t)stream, s->dev, P, E, io);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(finish_kernel(p->max_len), grid, dim3(threads), lds, (hipStream_t)stream, s->dev, P, E, io);
    HIP_TRY(hipGetLastError());
  } else {
    return fail(MPG_ERR_INVALID_ARG, "manifold_walk_batch: unknown form");
  }
  if (p->defer_fp64) return MPG_OK;
  hipLaunchKernelGGL(fp64_kernel(p->max_len), grid, dim3(threads), lds, (hipStream_t)stream, s->dev, P, E, io);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}

mpg_status walk_io(const mpg_chains* chains, const mpg_walk_out* wout, WalkIO* io) {
  if (!chains || !chains->d_prim || !chains->d_pos || !wout || !wout->d_status)
    return fail(MPG_ERR_INVALID_ARG, "NULL chains or status");
  io->seed_prim = chains->d_prim; io->seed_pos = chains->d_pos; io->seed_status = nullptr;
  io->prim_out = chains->d_prim; io->pos_out = chains->d_pos;
  io->status = wout->d_status; io->iters = wout->d_iters; io->sol = wout->d_solution_id;
  io->G = wout->d_G; io->kappa = wout->d_kappa; io->resid = wout->d_residual;
  return MPG_OK;
}

extern "C" mpg_status manifold_walk_fp64(const mpg_scene* s, const mpg_walk_params* p, const mpg_endpoints* ep,
                                         mpg_chains* chains, const mpg_walk_out* wout, void* stream) {
  if (!s) return fail(MPG_ERR_INVALID_ARG, "manifold_walk_fp64: NULL scene");
  WalkParams P;
  int waves;
  EpView E;
  WalkIO io;
  mpg_status st;
  if ((st = check_params(s, p, &P, &waves)) != MPG_OK) return st;
  if ((st = check_endpoints(ep, &E)) != MPG_OK) return st;
  if (E.N == 0) return MPG_OK;
  if ((st = walk_io(chains, wout, &io)) != MPG_OK) return st;
  int threads = 64 * waves;
  size_t lds = (size_t)waves * P.depth * 64 * 4;
  hipLaunchKernelGGL(fp64_kernel(p->max_len), dim3((E.N + threads - 1) / threads), dim3(threads), lds,
                     (hipStream_t)stream, s->dev, P, E, io);
  HIP_TRY(hipGetLastError());
  return MPG_OK;
}


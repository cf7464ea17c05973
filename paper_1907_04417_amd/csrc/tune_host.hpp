// Autotuner (included by mvamg_lib.hip inside its internal namespace, after
// the multi-system driver).  It times the kernel variants the library has for
// one uploaded hierarchy, on that hierarchy's own data and on the caller's
// stream, and keeps the fastest:
//   * grouped levels: the kernel instantiation G (64 / G lanes per row, any
//     power of two from the level's largest group up to 8), timed on a full
//     forward Gauss-Seidel sweep plus one residual;
//   * the coarsest block product of the block path (vector FMA or MFMA with
//     a given wave count and inner split);
//   * a batch: the number of chunks per problem of the per-problem reductions.
// Choices can be read and restored as text, so a caller can cache them per
// device and matrix signature and reuse them (results then repeat bitwise
// across runs; a different choice changes rounding only).

// Average milliseconds of fn over reps launches after one warm-up.
template <typename F>
double time_ms(hipStream_t st, int reps, F fn) {
  fn();
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreate(&e0));
  HIPCHECK(hipEventCreate(&e1));
  HIPCHECK(hipEventRecord(e0, st));
  for (int i = 0; i < reps; ++i) fn();
  HIPCHECK(hipEventRecord(e1, st));
  HIPCHECK(hipEventSynchronize(e1));
  float ms = 0.0f;
  HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms / reps;
}

std::string fmt_us(double ms) {
  char b[32];
  std::snprintf(b, sizeof b, "%.2f", 1e3 * ms);
  return b;
}

void tune_group_lanes(mvamg_hier* h, hipStream_t st, std::string& rep) {
  for (int l = 0; l + 1 < h->nl; ++l) {
    DevLevel& L = h->lv[l];
    if (L.sell) continue;
    double* r = L.r;
    double* x = L.x;
    k_fill<double><<<grid_for(L.n), kBlock, 0, st>>>(L.n, 1.0, r);
    k_fill<double><<<grid_for(L.n), kBlock, 0, st>>>(L.n, 0.0, x);
    LAUNCHCHECK("tune fill");
    int best = L.G;
    bool best_wide = false;
    double tbest = 1e30;
    // wave-per-group kernels with 64 / G lanes per row, then the block-per-group kernels
    std::vector<std::pair<int, bool>> cand;
    for (int G = L.G0; G <= kKmax; G *= 2) cand.emplace_back(G, false);
    cand.emplace_back(L.G0, true);
    for (const auto& gw : cand) {
      const int G = gw.first;
      const bool wide = gw.second;
      L.G = G;
      L.wide = wide;
      // the least of three timings of five sweeps each (a single timing
      // can be thrown off by a one-off delay)
      double t = 1e30;
      for (int rep = 0; rep < 3; ++rep)
        t = std::min(t, time_ms(st, 5, [&]() {
              for (int c = 1; c < L.ns; ++c) gs_stage<double>(h, l, L, c, r, x, 0, st);
              resid<double, 0>(h, l, L, r, x, L.s, M_NONE, st);
            }));
      rep += "level " + std::to_string(l) + (wide ? " wide" : " G=" + std::to_string(G)) + ": " + fmt_us(t) + " us; ";
      if (t < tbest) {
        tbest = t;
        best = G;
        best_wide = wide;
      }
    }
    L.G = best;
    L.wide = best_wide;
  }
}

void tune_block_coarse(mvamg_hier* h, hipStream_t st, std::string& rep) {
  ensure_block(h);
  DevCoarse& C = h->co;
  k_fill<double><<<grid_for((int64_t)C.n * kNB), kBlock, 0, st>>>((int64_t)C.n * kNB, 1.0, C.br);
  LAUNCHCHECK("tune fill");
  int best = kGemmDefault;
  double tbest = 1e30;
  for (int v = 0; v < kGemmVariantCount; ++v) {
    const double t = time_ms(st, 5, [&]() { launch_bgemm(h, v, C.br, C.bz, st); });
    rep += "gemm " + std::to_string(v) + ": " + fmt_us(t) + " us; ";
    if (t < tbest) {
      tbest = t;
      best = v;
    }
  }
  h->gemm_variant = best;
}

constexpr int kChunkCandidates[] = {4, 8, 16, 32, 64};

void tune_batch_chunks(mvamg_hier* h, hipStream_t st, std::string& rep) {
  if (h->nprob < 1) return;
  ensure_multi(h, h->nprob, kMaxChunks);
  k_fill<double><<<grid_for(h->n), kBlock, 0, st>>>(h->n, 1.0, h->r);
  LAUNCHCHECK("tune fill");
  int best = h->pchunks;
  double tbest = 1e30;
  for (int c : kChunkCandidates) {
    const double t = time_ms(st, 10, [&]() {
      k_pdot<1><<<dim3(c, h->nprob), kBlock, 0, st>>>(h->poff, h->iperm0, h->r, h->r, nullptr, nullptr, h->mb.part,
                                                      nullptr);
      k_mfinish<1><<<h->nprob, kBlock, 0, st>>>(h->nprob, c, h->mb.part, h->mb.scal, MM_STORE_TRR);
    });
    rep += "chunks " + std::to_string(c) + ": " + fmt_us(t) + " us; ";
    if (t < tbest) {
      tbest = t;
      best = c;
    }
  }
  h->pchunks = best;
}

std::string tune_text(const mvamg_hier* h) {
  std::string s;
  for (int l = 0; l + 1 < h->nl; ++l)
    if (!h->lv[l].sell)
      s += "G" + std::to_string(l) + "=" + std::to_string(h->lv[l].G) + ";W" + std::to_string(l) + "=" +
           std::to_string((int)h->lv[l].wide) + ";";
  s += "gemm=" + std::to_string(h->gemm_variant) + ";";
  if (h->nprob > 0) s += "chunks=" + std::to_string(h->pchunks) + ";";
  return s;
}

// Parses "key=value;..." (keys Gl, Wl, gemm, chunks) and applies it after
// checking every value; unknown keys are an error.
void apply_tune_text(mvamg_hier* h, const std::string& text) {
  std::vector<std::pair<std::string, int>> kv;
  size_t pos = 0;
  while (pos < text.size()) {
    size_t end = text.find(';', pos);
    if (end == std::string::npos) end = text.size();
    const std::string item = text.substr(pos, end - pos);
    pos = end + 1;
    if (item.empty()) continue;
    const size_t eq = item.find('=');
    if (eq == std::string::npos) throw Error(MVAMG_ERR_ARG, "tuning text: missing '=' in " + item);
    char* e = nullptr;
    const std::string val = item.substr(eq + 1);
    const long v = std::strtol(val.c_str(), &e, 10);
    if (val.empty() || *e) throw Error(MVAMG_ERR_ARG, "tuning text: bad value in " + item);
    kv.emplace_back(item.substr(0, eq), (int)v);
  }
  for (auto& p : kv) {
    const std::string& k = p.first;
    const int v = p.second;
    if (k == "gemm") {
      if (v < -1 || v >= kGemmVariantCount) throw Error(MVAMG_ERR_ARG, "tuning text: gemm variant out of range");
    } else if (k == "chunks") {
      if (h->nprob < 1 || v < 1 || v > 64) throw Error(MVAMG_ERR_ARG, "tuning text: chunks out of range");
    } else if (k.size() > 1 && (k[0] == 'G' || k[0] == 'W')) {
      char* e = nullptr;
      const long l = std::strtol(k.c_str() + 1, &e, 10);
      if (*e || l < 0 || l + 1 >= h->nl || h->lv[l].sell) throw Error(MVAMG_ERR_ARG, "tuning text: no grouped level " + k);
      const int g0 = h->lv[l].G0;
      if (k[0] == 'G' && (v < g0 || v > kKmax || (v & (v - 1)))) throw Error(MVAMG_ERR_ARG, "tuning text: bad G for " + k);
      if (k[0] == 'W' && v != 0 && v != 1) throw Error(MVAMG_ERR_ARG, "tuning text: W is 0 or 1 for " + k);
    } else {
      throw Error(MVAMG_ERR_ARG, "tuning text: unknown key " + k);
    }
  }
  for (auto& p : kv) {
    if (p.first == "gemm")
      h->gemm_variant = p.second;
    else if (p.first == "chunks")
      h->pchunks = p.second;
    else if (p.first[0] == 'W')
      h->lv[std::strtol(p.first.c_str() + 1, nullptr, 10)].wide = p.second != 0;
    else
      h->lv[std::strtol(p.first.c_str() + 1, nullptr, 10)].G = p.second;
  }
  if (h->nprob > 0) ensure_multi(h, h->nprob, h->pchunks);
  drop_graphs(h);
}

std::string signature_text(const mvamg_hier* h) {
  hipDeviceProp_t prop;
  HIPCHECK(hipGetDeviceProperties(&prop, h->device));
  std::string s = std::string("arch=") + prop.gcnArchName + ";cus=" + std::to_string(prop.multiProcessorCount) +
                  ";nprob=" + std::to_string(h->nprob) + ";n=";
  for (int l = 0; l < h->nl; ++l) s += (l ? "," : "") + std::to_string(h->lev_n[l]);
  s += ";nnz=";
  for (int l = 0; l < h->nl; ++l) s += (l ? "," : "") + std::to_string(h->lev_nnz[l]);
  return s;
}

void copy_text(const std::string& s, char* buf, size_t cap) {
  if (!buf || cap == 0) throw Error(MVAMG_ERR_ARG, "null or empty output buffer");
  if (s.size() + 1 > cap) throw Error(MVAMG_ERR_ARG, "output buffer too small (" + std::to_string(s.size() + 1) + " bytes needed)");
  std::memcpy(buf, s.c_str(), s.size() + 1);
}

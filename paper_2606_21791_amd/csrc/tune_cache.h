// JSON-lines cache of the autotuner (sg_autotune in sg.h), free of any device
// API so that it can be unit-tested on the host.  One object per line:
//   {"key": "<arch>|n<ceil log2 N>|<W>x<H>|<format>|sh<degree>|fb<fixed B>|mb<max B>",
//    "tile": .., "batch": .., "streams": .., "threads": .., "wgs_per_cu": ..,
//    "resume": .., "graphs": .., "grid": .., "inj_per_s": ..}
// ("grid" may be absent in older lines: 0).
// Later lines for the same key override earlier ones.
#pragma once

#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>

namespace sgtune {

struct Cfg {
  int tile = 16, batch = 32, streams = 16, threads = 2, wgs = 2, resume = 64, graphs = 0, grid = 0;
};

inline const char* dtype_name(int d) { return d == 0 ? "f32" : d == 1 ? "f16" : "bf16"; }

inline std::string make_key(const std::string& arch, long long n, int width, int height, int dtype, int sh_degree,
                            int fixed_batch, int max_batch) {
  int lg = 0;
  while ((1ll << lg) < n) ++lg;
  std::ostringstream k;
  k << arch << "|n" << lg << "|" << width << "x" << height << "|" << dtype_name(dtype) << "|sh" << sh_degree << "|fb"
    << fixed_batch << "|mb" << max_batch;
  return k.str();
}

inline bool json_int(const std::string& line, const char* name, int* v) {
  const std::string pat = std::string("\"") + name + "\": ";
  const size_t p = line.find(pat);
  if (p == std::string::npos) return false;
  return std::sscanf(line.c_str() + p + pat.size(), "%d", v) == 1;
}

inline bool lookup(const char* path, const std::string& key, Cfg* c, double* rate) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line;
  bool hit = false;
  const std::string kpat = "\"key\": \"" + key + "\"";
  while (std::getline(f, line)) {
    if (line.find(kpat) == std::string::npos) continue;
    Cfg x;
    if (!json_int(line, "tile", &x.tile) || !json_int(line, "batch", &x.batch) ||
        !json_int(line, "streams", &x.streams) || !json_int(line, "threads", &x.threads) ||
        !json_int(line, "wgs_per_cu", &x.wgs) || !json_int(line, "resume", &x.resume) ||
        !json_int(line, "graphs", &x.graphs))
      continue;
    if (!json_int(line, "grid", &x.grid)) x.grid = 0;
    const size_t p = line.find("\"inj_per_s\": ");
    double r = 0.0;
    if (p != std::string::npos) std::sscanf(line.c_str() + p + 13, "%lf", &r);
    *c = x;
    *rate = r;
    hit = true;
  }
  return hit;
}

inline bool append(const char* path, const std::string& key, const Cfg& c, double rate) {
  std::ofstream f(path, std::ios::app);
  if (!f) return false;
  f.precision(12);
  f << "{\"key\": \"" << key << "\", \"tile\": " << c.tile << ", \"batch\": " << c.batch
    << ", \"streams\": " << c.streams << ", \"threads\": " << c.threads << ", \"wgs_per_cu\": " << c.wgs
    << ", \"resume\": " << c.resume << ", \"graphs\": " << c.graphs << ", \"grid\": " << c.grid
    << ", \"inj_per_s\": " << rate << "}\n";
  return (bool)f;
}

}  // namespace sgtune

// Command-line driver of the library's host-only code (host_core.cpp), built
// by tests/test_host_sanitizers.py with the address and undefined-behaviour
// sanitizers.  Commands on stdin, whitespace-separated tokens:
//   T n        -> "T n" then the n*n DCT rows and the n*n Haar rows, one
//                 hexadecimal double per line
//   P families w h n_min n_max step level n_ch
//     then per channel: count, then per node: n split n_atoms idx.. coef..
//              -> "OK size hexbytes" or "ERR code message"
// Floating-point tokens are read with strtod (hexadecimal floats allowed).
#include <cstdio>
#include <cstdlib>
#include <iostream>
#include <string>
#include <vector>

#include "aqmp.h"
#include "host_core.h"

using namespace aqmp;

static double num(std::istream& in) {
  std::string t;
  in >> t;
  return std::strtod(t.c_str(), nullptr);
}

int main() {
  std::string cmd;
  while (std::cin >> cmd) {
    if (cmd == "T") {
      int n;
      std::cin >> n;
      std::vector<double> c((size_t)n * n), h((size_t)n * n);
      dct_table(n, c.data());
      haar_table(n, h.data());
      std::printf("T %d\n", n);
      for (double v : c) std::printf("%a\n", v);
      for (double v : h) std::printf("%a\n", v);
    } else if (cmd == "P") {
      StreamHeader hd{};
      int level, n_ch;
      std::cin >> hd.families >> hd.w >> hd.h >> hd.n_min >> hd.n_max;
      const double step = num(std::cin);
      std::cin >> level >> n_ch;
      std::vector<std::vector<StreamNode>> nodes(n_ch > 0 ? n_ch : 0);
      // first read everything, then point the nodes at stable storage
      struct Raw {
        int n, split, t;
        std::vector<int32_t> i;
        std::vector<double> c;
      };
      std::vector<std::vector<Raw>> raw(nodes.size());
      for (auto& ch : raw) {
        size_t cnt;
        std::cin >> cnt;
        ch.resize(cnt);
        for (auto& r : ch) {
          std::cin >> r.n >> r.split >> r.t;
          r.i.resize(r.t > 0 ? r.t : 0);
          r.c.resize(r.i.size());
          for (auto& v : r.i) std::cin >> v;
          for (auto& v : r.c) v = num(std::cin);
        }
      }
      std::vector<StreamChannel> chans(nodes.size());
      for (size_t c = 0; c < raw.size(); ++c) {
        for (auto& r : raw[c])
          nodes[c].push_back(StreamNode{r.n, r.split != 0, r.t, r.i.empty() ? nullptr : r.i.data(),
                                        r.c.empty() ? nullptr : r.c.data()});
        chans[c] = StreamChannel{nodes[c].data(), nodes[c].size()};
      }
      std::vector<uint8_t> out;
      std::string err;
      int rc = stream_write(hd, chans.empty() ? nullptr : chans.data(), n_ch, step, out, &err);
      if (rc == AQMP_OK && level >= 0) {
        std::vector<uint8_t> z;
        rc = stream_deflate(out, level, z);
        if (rc == AQMP_OK && z.size() > stream_deflate_bound(out.size())) {
          rc = -100;
          err = "deflate bound exceeded";
        }
        out.swap(z);
      }
      if (rc != AQMP_OK) {
        std::printf("ERR %d %s\n", rc, err.c_str());
      } else {
        std::printf("OK %zu ", out.size());
        for (uint8_t b : out) std::printf("%02x", b);
        std::printf("\n");
      }
    } else {
      std::fprintf(stderr, "unknown command %s\n", cmd.c_str());
      return 2;
    }
    std::fflush(stdout);
  }
  return 0;
}

// CPU harness for the stream header parser and the plan it rebuilds
// (parse_header, plan_from_header of the library's host format code),
// built with the address and undefined-behaviour sanitizers by
// tests/test_parser_fuzz.py.  Reads each file named on the command line and
// prints one line per file: "ok <blocks>" or "corrupt <message>".  Any
// memory error or undefined behaviour aborts the run through the
// sanitizers.
#include <cstdio>
#include <fstream>
#include <iterator>
#include <string>
#include <vector>

#include "dls_internal.h"

int main(int argc, char** argv) {
  for (int i = 1; i < argc; ++i) {
    std::ifstream f(argv[i], std::ios::binary);
    std::vector<uint8_t> buf((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    dls::StreamHeader h;
    std::string err = dls::parse_header(buf.data(), buf.size(), h);
    if (err.empty()) {
      dls::Plan pl;
      err = dls::plan_from_header(h, pl, 1024);
      if (err.empty() && int64_t(pl.blocks.size()) != h.nblocks) err = "plan size";
    }
    if (err.empty()) std::printf("ok %lld\n", static_cast<long long>(h.nblocks));
    else std::printf("corrupt %s\n", err.c_str());
  }
  return 0;
}

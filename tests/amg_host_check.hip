// CPU driver of the AMG hierarchy build of libsstep (csrc/amg.hip, host
// side only; no GPU call): reads a CSR matrix, builds the levels with the
// library's own functions and writes, per level, the aggregate of every row,
// the prolongator and the coarse operator, then the coarsest level's
// inverse.  tests/test_amg_host.py builds it with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code and compares the output with
// the oracle's hierarchy.
#include "amg.hip"

#include <cstdio>

namespace {

bool read_csr(const char *path, ssp::HostCsr &A) {
  FILE *f = fopen(path, "rb");
  if (!f) return false;
  int64_t n = 0, nnz = 0;
  bool ok = fread(&n, 8, 1, f) == 1 && fread(&nnz, 8, 1, f) == 1;
  std::vector<int32_t> rp(ok ? n + 1 : 0);
  A.n = A.m = n;
  A.ci.resize(ok ? nnz : 0);
  A.v.resize(ok ? nnz : 0);
  ok = ok && fread(rp.data(), 4, n + 1, f) == (size_t)(n + 1) &&
       fread(A.ci.data(), 4, nnz, f) == (size_t)nnz && fread(A.v.data(), 8, nnz, f) == (size_t)nnz;
  fclose(f);
  A.rp.assign(rp.begin(), rp.end());
  return ok;
}

void write_csr(FILE *o, const ssp::HostCsr &M) {
  const int64_t hdr[3] = {M.n, M.m, (int64_t)M.ci.size()};
  fwrite(hdr, 8, 3, o);
  fwrite(M.rp.data(), 8, M.n + 1, o);
  fwrite(M.ci.data(), 4, M.ci.size(), o);
  fwrite(M.v.data(), 8, M.v.size(), o);
}

}  // namespace

int main(int argc, char **argv) {
  if (argc != 5) {
    fprintf(stderr, "usage: amg_host_check matrix.bin out.bin max_coarse max_levels\n");
    return 2;
  }
  ssp::HostCsr F;
  if (!read_csr(argv[1], F)) {
    fprintf(stderr, "cannot read %s\n", argv[1]);
    return 2;
  }
  std::vector<ssp::HostCsr> As, Ps, Rs;
  std::vector<std::vector<int64_t>> aggs;
  std::string why;
  if (!ssp::build_levels(F, 0.08, atoll(argv[3]), atoi(argv[4]), As, Ps, Rs, aggs, why)) {
    fprintf(stderr, "%s\n", why.c_str());
    return 3;
  }
  std::vector<double> inv;
  if (!ssp::dense_inverse(As.back(), inv)) return 4;
  FILE *o = fopen(argv[2], "wb");
  if (!o) return 2;
  const int64_t levels = (int64_t)As.size();
  fwrite(&levels, 8, 1, o);
  for (size_t l = 0; l + 1 < As.size(); ++l) {
    fwrite(aggs[l].data(), 8, aggs[l].size(), o);
    write_csr(o, Ps[l]);
    write_csr(o, Rs[l]);
    write_csr(o, As[l + 1]);
  }
  fwrite(inv.data(), 8, inv.size(), o);
  fclose(o);
  printf("levels %lld\n", (long long)levels);
  return 0;
}
